// U_k = Q U^ and V_k = Z V~ (paper, Algorithm 1: U = Q U^, V = Z V^): an n x p by p x r
// product per side, p, r <= 64, on the FP64 matrix cores (v_mfma_f64_16x16x4).
//
// Computed transposed, out^T = B^T Q^T, so that the MFMA result rows are output columns and
// each lane's results run down a column: the 16-lane groups of a store write 128 contiguous
// bytes of one column. Per 16-row tile a wave issues ceil(p/4) x ceil(r/16) MFMAs:
//   A operand (16 x 4): B^T(c0 + l%16, k0 + l/16) = B(k0 + l/16, c0 + l%16), read from LDS
//                       (B is staged there once per workgroup);
//   B operand (4 x 16): Q^T(k0 + l/16, i0 + l%16) = Q(i0 + l%16, k0 + l/16), read from HBM
//                       (16 consecutive rows of 4 columns per instruction);
//   result (16 x 16):   lane l, item v holds out(i0 + l%16, c0 + l/16 + 4 v).
// Columns of Q at or beyond p and rows of B at or beyond p read as 0, so stale memory never
// enters the sums. The MFMAs run only over the live part of the padded 64 x 64 B: KS 4-row steps
// (p rounded up to 16) by NT 16-column tiles (r rounded up to 16), compile-time counts chosen
// once per launch by a uniform switch, so that every variant stays straight-line code (uniform
// branches inside the unrolled loop break its schedule). Each wave streams its row tiles (8; fewer at small n), loading
// the next tile's Q while the current one is on the matrix cores, and reads B's operands from
// LDS at every tile (216 registers, two waves per SIMD; B held in registers for the whole loop
// took 334 and left one wave per SIMD: 0.58 -> 0.53 ms per FP64 launch at n = 2^20 - 1).
#include "lrp_kernels.h"

namespace lrp {

typedef double d4 __attribute__((ext_vector_type(4)));

// 16-row tiles per wave: 8, or fewer (4, 2) where a launch of 8 would make fewer workgroups
// than twice the CU count. A tile's products are the same whatever wave computes them.
constexpr int kProdTilesMax = 8;

template <int KS, int NT>
__device__ __forceinline__ void prod_body(const ProdArgs& a, int side, int kin, int r, double* Bs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // B zero-padded to 64 x 64 in LDS (Bs: row-major, padded rows), then its live part held in
  // registers by every wave for all of its row tiles
  const double* Bg = a.B[side];
  for (int e = threadIdx.x; e < kPMax * kPMax; e += blockDim.x) {
    const int m = e % kPMax, c = e / kPMax;
    Bs[m * (kPMax + 1) + c] = (m < kin && c < r) ? Bg[m + (int64_t)c * a.pmax] : 0.0;
  }
  __syncthreads();
  const double* Q = a.Q[side];
  double* out = a.out[side];
  const int tiles = a.tiles;
  const int64_t base = (int64_t)blockIdx.x * 64 * tiles + (int64_t)wave * 16 * tiles;
  auto load_tile = [&](int tile, double (&q)[KS]) {
    const int64_t i = base + 16 * tile + lr;
    const bool row_ok = i < a.n;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int m = 4 * ks + lk;
      q[ks] = (row_ok && m < kin) ? Q[i + (int64_t)m * a.ldq] : 0.0;
    }
  };
  double qa[KS], qb[KS];
  load_tile(0, qa);
#pragma unroll 1
  for (int tile = 0; tile < tiles; tile += 2) {
    // even tile from qa while qb is loading, then odd tile from qb while qa is loading
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double(&qc)[KS] = h == 0 ? qa : qb;
      double(&qn)[KS] = h == 0 ? qb : qa;
      const int tcur = tile + h;
      if (tcur + 1 < tiles) load_tile(tcur + 1, qn);
      d4 acc[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt] = d4{0.0, 0.0, 0.0, 0.0};
      // B's operands are read from LDS at each tile: an offset the compiler cannot see through
      // keeps them from being hoisted out of the tile loop into registers (which held all of B
      // for the whole loop and left one wave per SIMD)
      int boff = lk * (kPMax + 1) + lr;
      asm volatile("" : "+v"(boff));
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(Bs[boff + 4 * ks * (kPMax + 1) + 16 * nt], qc[ks], acc[nt],
                                                         0, 0, 0);
      const int64_t i = base + 16 * tcur + lr;
      const bool row_ok = i < a.n;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * nt + lk + 4 * v;
          if (row_ok && c < r) out[i + (int64_t)c * a.ldo] = acc[nt][v];
        }
    }
  }
}

template <int KS>
__device__ __forceinline__ void prod_nt(const ProdArgs& a, int side, int kin, int r, double* Bs) {
  switch ((r + 15) >> 4) {  // uniform
    case 0:
    case 1: prod_body<KS, 1>(a, side, kin, r, Bs); break;
    case 2: prod_body<KS, 2>(a, side, kin, r, Bs); break;
    case 3: prod_body<KS, 3>(a, side, kin, r, Bs); break;
    default: prod_body<KS, 4>(a, side, kin, r, Bs); break;
  }
}

template <class Src>
__global__ __launch_bounds__(256) void k_prod(Src in) {
  const ProdArgs& a = kernel_args<ProdArgs>(in);
  const DevState* st = a.st;
  if (st->done || (a.gate_guess && !st->guess_ok)) return;
  const int side = blockIdx.y;
  const int kin = st->ncols[side];
  const int r = st->r[a.nb];
  __shared__ double Bs[kPMax * (kPMax + 1)];
  switch ((kin + 15) >> 4) {  // uniform: 4-row steps of B in groups of four
    case 0:
    case 1: prod_nt<4>(a, side, kin, r, Bs); break;
    case 2: prod_nt<8>(a, side, kin, r, Bs); break;
    case 3: prod_nt<12>(a, side, kin, r, Bs); break;
    default: prod_nt<16>(a, side, kin, r, Bs); break;
  }
}

int prod_launch(const ProdArgs& args, hipStream_t s) {
  ProdArgs a = args;
  a.tiles = kProdTilesMax;
  while (a.tiles > 2 && 2 * (a.n + 64 * a.tiles - 1) / (64 * a.tiles) < 2 * kCUs) a.tiles >>= 1;
  const int64_t rows = 64 * a.tiles;  // 4 waves
  dim3 grid((unsigned)((a.n + rows - 1) / rows), 2);
  LRP_LAUNCH_G(K_PROD, k_prod<ProdArgs>, k_prod<GroupRef>, grid, dim3(256), 0, s, a);
  return launch_status();
}

}  // namespace lrp
