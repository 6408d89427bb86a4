// U_k = Q U^ and V_k = Z V~ (paper, Algorithm 1: U = Q U^, V = Z V^): an n x p by p x r
// product per side. One thread per grid row keeps the r accumulators of its output row in
// registers; the p x r coefficient matrix sits in LDS (zero-padded to 64 x 64) and is read as
// a broadcast. Reads of Q and writes of the result are coalesced.
#include "lrp_kernels.h"

namespace lrp {

__global__ __launch_bounds__(256) void k_prod(ProdArgs a) {
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  const int kin = st->ncols[side];
  const int r = st->r[a.nb];
  __shared__ double B[kPMax * kPMax];
  const double* Bg = a.B[side];
  for (int e = threadIdx.x; e < kPMax * kPMax; e += blockDim.x) {
    const int m = e % kPMax, c = e / kPMax;
    B[m * kPMax + c] = (m < kin && c < r) ? Bg[m + (int64_t)c * a.pmax] : 0.0;  // row-major
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double acc[kPMax];
#pragma unroll
  for (int c = 0; c < kPMax; ++c) acc[c] = 0.0;
  const double* Q = a.Q[side] + i;
  for (int m = 0; m < kin; ++m) {
    const double q = Q[(int64_t)m * a.ldq];
    const double* Bm = B + m * kPMax;
#pragma unroll
    for (int c = 0; c < kPMax; ++c) acc[c] = fma(q, Bm[c], acc[c]);
  }
  double* out = a.out[side] + i;
#pragma unroll
  for (int c = 0; c < kPMax; ++c)
    if (c < r) out[(int64_t)c * a.ldo] = acc[c];
}

int prod_launch(const ProdArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n + 255) / 256), 2);
  hipLaunchKernelGGL(k_prod, grid, dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // namespace lrp
