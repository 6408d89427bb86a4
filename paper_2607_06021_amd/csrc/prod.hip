// U_k = Q U^ and V_k = Z V~ (paper, Algorithm 1: U = Q U^, V = Z V^): an n x p by p x r
// product per side, p, r <= 64, on the FP64 matrix cores (v_mfma_f64_16x16x4).
//
// Computed transposed, out^T = B^T Q^T, so that the MFMA result rows are output columns and
// each lane's results run down a column: the 16-lane groups of a store write 128 contiguous
// bytes of one column. Per 16-row tile a wave issues ceil(p/4) x ceil(r/16) MFMAs:
//   A operand (16 x 4): B^T(c0 + l%16, k0 + l/16) = B(k0 + l/16, c0 + l%16), held in registers
//                       for the whole launch (64 doubles per lane);
//   B operand (4 x 16): Q^T(k0 + l/16, i0 + l%16) = Q(i0 + l%16, k0 + l/16), read from HBM
//                       (16 consecutive rows of 4 columns per instruction);
//   result (16 x 16):   lane l, item v holds out(i0 + l%16, c0 + l/16 + 4 v).
// Columns of Q at or beyond p and rows of B at or beyond p read as 0, so stale memory never
// enters the sums.
#include "lrp_kernels.h"

namespace lrp {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kProdTilesPerWave = 4;
constexpr int kProdRowsPerBlock = 16 * kProdTilesPerWave * 4;  // 4 waves

__global__ __launch_bounds__(256) void k_prod(ProdArgs a) {
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  const int kin = st->ncols[side];
  const int r = st->r[a.nb];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const double* Bg = a.B[side];
  double bt[16][4];  // [k-step][column tile]
#pragma unroll
  for (int ks = 0; ks < 16; ++ks)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int m = 4 * ks + lk, c = 16 * nt + lr;
      bt[ks][nt] = (m < kin && c < r) ? Bg[m + (int64_t)c * a.pmax] : 0.0;
    }
  const double* Q = a.Q[side];
  double* out = a.out[side];
  const int64_t base = (int64_t)blockIdx.x * kProdRowsPerBlock + (int64_t)wave * 16 * kProdTilesPerWave;
  for (int tile = 0; tile < kProdTilesPerWave; ++tile) {
    const int64_t i = base + 16 * tile + lr;
    if (base + 16 * tile >= a.n) break;  // uniform across the wave
    const bool row_ok = i < a.n;
    double q[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int m = 4 * ks + lk;
      q[ks] = (row_ok && m < kin) ? Q[i + (int64_t)m * a.ldq] : 0.0;
    }
    d4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      if (4 * ks >= kin) break;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        if (16 * nt < r) acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(bt[ks][nt], q[ks], acc[nt], 0, 0, 0);
    }
    if (!row_ok) continue;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * nt + lk + 4 * v;
        if (c < r) out[i + (int64_t)c * a.ldo] = acc[nt][v];
      }
  }
}

int prod_launch(const ProdArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n + kProdRowsPerBlock - 1) / kProdRowsPerBlock), 2);
  hipLaunchKernelGGL(k_prod, grid, dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // namespace lrp
