// Fibers of the spectrally divided solution (paper, Section 3.1, eq. g_for_p):
//   W^(i, j) = sum_t U^(i, t) V^(j, t) / (lambda_i + lambda_j),
// with h^2 sigma folded into U^. One launch writes both C = W^(:, J) (side 0) and
// R^T = W^(I, :)^T (side 1): out(i, c) = sum_t A(i, t) b_c(t) / (lambda_i + lambda_{idx_c}),
// A = U^, b_c = V^(J_c, :) for side 0 and A = V^, b_c = U^(I_c, :) for side 1.
// Each thread owns one grid row i and keeps A(i, :) in registers; the gathered b_c rows and
// lambda_{idx_c} sit in LDS. Reads of A and writes of out are coalesced (column-major, one
// row per lane). The mixed-precision path runs this kernel in FP32 with FP32 accumulation.
#include "lrp_kernels.h"

namespace lrp {

template <typename T>
__global__ __launch_bounds__(256) void k_fiber(FiberArgs a) {
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  const int rF = st->rF;
  const int nc = side == 0 ? st->nJpre : st->nIpre;
  const int* idx = side == 0 ? st->Jpre : st->Ipre;
  const T* A = (const T*)(side == 0 ? a.Uh : a.Vh);
  const T* Bsrc = (const T*)(side == 0 ? a.Vh : a.Uh);
  const T* lam = (const T*)a.lam;
  T* out = (T*)(side == 0 ? a.C : a.Rt);

  __shared__ T b[kPMax][kPMax + 1];
  __shared__ T lb[kPMax];
  for (int e = threadIdx.x; e < nc * rF; e += blockDim.x) {
    const int cc = e / rF, tt = e % rF;
    b[cc][tt] = Bsrc[idx[cc] + (int64_t)tt * a.ldh];
  }
  for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) lb[cc] = lam[idx[cc]];
  __syncthreads();

  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  T ar[kPMax];
#pragma unroll
  for (int tt = 0; tt < kPMax; ++tt) ar[tt] = tt < rF ? A[i + (int64_t)tt * a.ldh] : T(0);
  const T li = lam[i];
  for (int cc = 0; cc < nc; ++cc) {
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int tt = 0; tt < kPMax; tt += 2) {
      if (tt < rF) s0 = fma(ar[tt], b[cc][tt], s0);
      if (tt + 1 < rF) s1 = fma(ar[tt + 1], b[cc][tt + 1], s1);
    }
    out[i + (int64_t)cc * a.ldc] = (s0 + s1) / (li + lb[cc]);
  }
}

int fiber_launch(const FiberArgs& a, bool fp32, hipStream_t s) {
  dim3 grid((unsigned)((a.n + 255) / 256), 2);
  prof_mark(s, K_FIBER);
  if (fp32)
    hipLaunchKernelGGL(k_fiber<float>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_fiber<double>, grid, dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // namespace lrp
