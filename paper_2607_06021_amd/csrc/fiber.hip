// Fibers of the spectrally divided solution (paper, Section 3.1, eq. g_for_p):
//   W^(i, j) = sum_t U^(i, t) V^(j, t) / (lambda_i + lambda_j),
// with h^2 sigma folded into U^. One launch writes both C = W^(:, J) (side 0) and
// R^T = W^(I, :)^T (side 1): out(i, c) = sum_t A(i, t) b_c(t) / (lambda_i + lambda_{idx_c}),
// A = U^, b_c = V^(J_c, :) for side 0 and A = V^, b_c = U^(I_c, :) for side 1.
// The gathered b_c rows and lambda_{idx_c} sit in LDS. Reads of A and writes of out are
// coalesced (column-major, one row per lane). The mixed-precision path runs this kernel in
// FP32 with FP32 accumulation.
#include "lrp_kernels.h"

namespace lrp {

// q / d for d > 0 normal: reciprocal from the hardware approximation, two Newton steps on the
// reciprocal and one correction of the quotient (FP64); FP32 uses the plain division.
__device__ inline double div_pos(double q, double d) {
  const double r = rcp_nr(d);
  const double x = q * r;
  return fma(r, fma(-d, x, q), x);
}
__device__ inline float div_pos(float q, float d) { return q / d; }

// Each thread owns one grid row i: A(i, 0..rF-1) in registers (the loops over t are unrolled
// to kPMax with a uniform bound test, so the row never leaves registers); the outputs of 8
// columns are accumulated at once (two partial sums each, so 16 independent FMA chains hide
// the FP latency), with b_c(t) read from LDS as broadcasts.
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

  constexpr int G = 8;
  __shared__ T b[kPMax + G][kPMax];  // rows beyond nc stay zero
  __shared__ T lb[kPMax + G];
  for (int e = threadIdx.x; e < (kPMax + G) * kPMax; e += blockDim.x) {
    const int cc = e / kPMax, tt = e % kPMax;
    b[cc][tt] = (cc < nc && tt < rF) ? Bsrc[idx[cc] + (int64_t)tt * a.ldh] : T(0);
  }
  for (int cc = threadIdx.x; cc < kPMax + G; cc += blockDim.x) lb[cc] = cc < nc ? lam[idx[cc]] : T(1);
  __syncthreads();

  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  T ar[kPMax];
#pragma unroll
  for (int tt = 0; tt < kPMax; ++tt) ar[tt] = tt < rF ? A[i + (int64_t)tt * a.ldh] : T(0);
  const T li = lam[i];
  for (int c0 = 0; c0 < nc; c0 += G) {
    T s0[G], s1[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s0[g] = s1[g] = T(0);
#pragma unroll
    for (int tt = 0; tt < kPMax; tt += 2) {
      if (tt < rF) {  // uniform
#pragma unroll
        for (int g = 0; g < G; ++g) {
          s0[g] = fma(ar[tt], b[c0 + g][tt], s0[g]);
          s1[g] = fma(ar[tt + 1], b[c0 + g][tt + 1], s1[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c0 + g < nc) out[i + (int64_t)(c0 + g) * a.ldc] = div_pos(s0[g] + s1[g], li + lb[c0 + g]);
  }
}

int fiber_launch(const FiberArgs& a, bool fp32, hipStream_t s) {
  dim3 grid((unsigned)((a.n + 255) / 256), 2);
  if (fp32)
    LRP_LAUNCH(K_FIBER, k_fiber<float>, grid, dim3(256), 0, s, a);
  else
    LRP_LAUNCH(K_FIBER, k_fiber<double>, grid, dim3(256), 0, s, a);
  return launch_status();
}

}  // namespace lrp
