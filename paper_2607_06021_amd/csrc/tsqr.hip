// Tall-skinny Householder QR (the thin QRs C = Q R_C and R^T = Z R_R of Algorithm 1).
//
// The n x p matrix is cut into 256-row blocks. Each block is factored by one workgroup with
// LAPACK's Householder convention (beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta,
// v = x/(alpha - beta), v_0 = 1). The p x p R factors are stacked and factored again, in
// groups of 256/p_max, up a tree until one block is left; its R is the R of the matrix.
// Q is formed top-down: each block applies its reflectors to [T; 0], where T is its p x p
// piece of the parent level's Q.
//
// Two sides (e.g. C and R^T) are processed by the same launch (blockIdx.y).
#include <mutex>

#include "lrp_kernels.h"

namespace lrp {


struct FactorArgs {
  const DevState* st;
  int ncols[2];
  const void* in[2];
  int in_f32;
  int64_t ldin;
  int64_t rows;
  int block_rows;
  int pmax;
  double* V[2];
  int64_t ldv;
  double* tau[2];
  double* Rout[2];
  int64_t ldr;
};

struct ApplyArgs {
  const DevState* st;
  int ncols[2];
  const double* V[2];
  int64_t ldv;
  const double* tau[2];
  int64_t rows;
  int block_rows;
  int pmax;
  const double* T[2];  // parent pieces (rows b*pmax .. b*pmax+p of a matrix with ld ldt); null = identity
  int64_t ldt;
  double* Y[2];
  int64_t ldy;
};

// An empty asm statement that takes a loaded value as input and output: the load must then
// complete unconditionally before it, so a following select on a lane condition cannot be
// turned into a branch around the load (which would serialise the loads, each with its own wait).
__device__ inline void keep_loaded(double& v) { asm volatile("" : "+v"(v)); }
__device__ inline void keep_loaded(float& v) { asm volatile("" : "+v"(v)); }

__device__ inline int side_cols(const DevState* st, const int* fixed, int side) {
  return st ? st->ncols[side] : fixed[side];
}

// Sum over the 16 lanes of a DPP row (lanes 16q .. 16q+15); every lane gets the total.
__device__ inline double row16_sum(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  x += __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false),
                        __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
  lo = __double2loint(x);
  hi = __double2hiint(x);
  x += __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false),
                        __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false));  // quad_perm [2,3,0,1]
  lo = __double2loint(x);
  hi = __double2hiint(x);
  x += __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false),
                        __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false));  // row_half_mirror
  lo = __double2loint(x);
  hi = __double2hiint(x);
  x += __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false),
                        __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false));  // row_mirror
  return x;
}

// Sum over the 64 lanes of the wave; every lane gets the same total. After the row sums, a
// 16-lane swap (odd rows of one copy exchanged with even rows of the other) pairs rows 0, 1 and
// 2, 3, and a 32-lane swap pairs the two halves; both operand orders agree on every lane.
__device__ inline double wave64_sum(double x) {
  x = row16_sum(x);
  int lo = __double2loint(x), hi = __double2hiint(x);
  const auto l16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  x = __hiloint2double(h16[0], l16[0]) + __hiloint2double(h16[1], l16[1]);
  lo = __double2loint(x);
  hi = __double2hiint(x);
  const auto l32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(h32[0], l32[0]) + __hiloint2double(h32[1], l32[1]);
}

// Thread layout of a 256-row block: wave w holds columns 4w .. 4w+3 and lane l rows l, l+64,
// l+128 and l+192 of each; register slot s of lane l holds column 4w + (s ^ m(l)), where
// m(l) = 2 (l & 1) + ((l >> 1) & 1). A column lives in one wave, so its dot products are wave
// reductions, and a reflector is read from LDS as four consecutive-word loads per lane (a
// quarter of the traffic of a layout with 16 lanes per column, where every lane re-reads 16
// elements shared with three other columns). The slot permutation lets the four dot products of
// a step be reduced together by halving exchanges (wave4_sums): each exchange between lanes l and
// l ^ 1, then l ^ 2, sends the slots that the partner keeps, with no per-lane selection.

__device__ inline int slot_perm(int l) { return ((l & 1) << 1) | ((l >> 1) & 1); }

template <int CTRL>
__device__ inline double dpp_d(double x) {
  return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false));
}

// Sums over the wave of the four per-slot partials d[s] (slot s of lane l = column s ^ m(l));
// on return d[s] is the total of that slot's column, the same value on every lane holding it.
//   * lanes l, l^1 (m differs in bit 1): keep slots 0, 1, add the partner's slots 2, 3;
//   * lanes l, l^2 (m differs in bit 0): keep slot 0, add the partner's slot 1; the lane now has
//     the quad's partial of column m(l);
//   * rotations by 8 and then 4 lanes inside each 16-lane row (both keep l mod 4, and the sums
//     are formed in the same order on the four lanes of a residue), then the 16- and 32-lane
//     swaps: every lane has the total of column m(l);
//   * slots 1, 2, 3 (columns m^1, m^2, m^3) are read from lanes l^2, l^1, l^3.
__device__ inline void wave4_sums(double (&d)[4]) {
  const double r0 = d[0] + dpp_d<0xB1>(d[2]);  // quad_perm [1,0,3,2]
  const double r1 = d[1] + dpp_d<0xB1>(d[3]);
  double u = r0 + dpp_d<0x4E>(r1);             // quad_perm [2,3,0,1]
  u += dpp_d<0x128>(u);                        // row_ror:8
  u += dpp_d<0x124>(u);                        // row_ror:4
  int lo = __double2loint(u), hi = __double2hiint(u);
  const auto l16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  u = __hiloint2double(h16[0], l16[0]) + __hiloint2double(h16[1], l16[1]);
  lo = __double2loint(u);
  hi = __double2hiint(u);
  const auto l32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  u = __hiloint2double(h32[0], l32[0]) + __hiloint2double(h32[1], l32[1]);
  d[0] = u;
  d[1] = dpp_d<0x4E>(u);  // lane l^2
  d[2] = dpp_d<0xB1>(u);  // lane l^1
  d[3] = dpp_d<0x1B>(u);  // lane l^3, quad_perm [3,2,1,0]
}

// Slot sl (per lane) of the lane's four columns, by two selects on its bits. The values pass
// through an empty asm statement first, so that the selects stay selects of registers (a select
// of two array elements may be turned into an element at a selected index, which would move the
// whole array to scratch memory).
__device__ inline void pick_slot(const double (&x)[4][4], int sl, double (&col)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double x0 = x[k][0], x1 = x[k][1], x2 = x[k][2], x3 = x[k][3];
    asm volatile("" : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3));
    const double lo = (sl & 1) ? x1 : x0;
    const double hi = (sl & 1) ? x3 : x2;
    col[k] = (sl & 2) ? hi : lo;
  }
}

// Householder vector of column c (rows 64k + l in col[k], already transformed by reflectors
// 0 .. c-1; c < 64 and the same on every lane). vb receives the whole reflector (v_c = 1, zeros
// above, the tail times scale below); col itself is left as it is (rows above c are
// R(0..c-1, c), and the tail is scaled when the reflectors are written out).
//
// With h = sqrt(alpha^2 + |x_tail|^2) and s = sign(alpha): beta = -s h, tau = (beta - alpha) /
// beta = 1 + |alpha| / h and 1 / (alpha - beta) = s / (|alpha| + h), so one reciprocal square
// root and one reciprocal give all three; the diagonal element alpha (row c, lane c of the first
// group) is read from the lane that holds it. Only a zero tail or an extreme magnitude leave this
// straight-line path.
__device__ inline void householder_column(const double (&col)[4], int c, int l, double* vb, double& beta,
                                          double& tau, double& scale) {
  double y[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) y[k] = 64 * k + l > c ? col[k] : 0.0;
  const double xnorm2 = wave64_sum(fma(y[0], y[0], y[1] * y[1]) + fma(y[2], y[2], y[3] * y[3]));
  const double alpha = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(col[0]), c),
                                        __builtin_amdgcn_readlane(__double2loint(col[0]), c)) +
                       0.0;  // a zero diagonal counts as +0
  const double h2 = fma(alpha, alpha, xnorm2);
  const double rh = rsq_nr(h2);
  const double h = h2 * rh;
  beta = -copysign(h, alpha);
  tau = fma(fabs(alpha), rh, 1.0);
  scale = copysign(rcp_nr(fabs(alpha) + h), alpha);
  if (xnorm2 == 0.0) {
    tau = 0.0;
    beta = alpha;
    scale = 0.0;
  } else if (!(h2 > 1e-290 && h2 < 1e290)) {  // extreme magnitudes: correctly rounded operations
    beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  vb[l] = l == c ? 1.0 : y[0] * scale;
#pragma unroll
  for (int k = 1; k < 4; ++k) vb[64 * k + l] = y[k] * scale;
}

// One workgroup per 256-row block. Column 0 builds its reflector first; then at step j, after
// the barrier that publishes v_j (double-buffered in LDS), every wave with a trailing column
// applies it to its four columns (four dot products reduced together), and the wave of column
// j+1 goes on at once to build v_{j+1}: one barrier per reflector. Nothing is written to global
// memory inside the loop, so the per-step barrier waits on LDS only.
__device__ __forceinline__ void factor_block(const FactorArgs& a) {
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, l = t & 63, c0 = 4 * (t >> 6), m = slot_perm(l);
  __shared__ double vbuf[2][kTsqrRows];
  __shared__ double tsh[kPMax];   // tau, R(c, c) and the reflector scale of column c
  __shared__ double rdsh[kPMax];
  __shared__ double vssh[kPMax];

  // Every load reads a valid element (row and column clamped into the block) and the unused ones
  // are replaced by zeros afterwards, so that all 16 loads are in flight together.
  double x[4][4];
  {
    int64_t cb[4];
    int rk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cb[q] = row0 + (int64_t)min(c0 + (q ^ m), p - 1) * a.ldin;
#pragma unroll
    for (int k = 0; k < 4; ++k) rk[k] = min(64 * k + l, nr - 1);
    if (a.in_f32) {
      const float* X = (const float*)a.in[side];
      float raw[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) raw[k][q] = X[cb[q] + rk[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          keep_loaded(raw[k][q]);
          x[k][q] = (c0 + (q ^ m) < p && 64 * k + l < nr) ? (double)raw[k][q] : 0.0;
        }
    } else {
      const double* X = (const double*)a.in[side];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) x[k][q] = X[cb[q] + rk[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          keep_loaded(x[k][q]);
          x[k][q] = (c0 + (q ^ m) < p && 64 * k + l < nr) ? x[k][q] : 0.0;
        }
    }
  }
  // After its reflector is built, column c is final: its registers keep R(0..c-1, c) above the
  // diagonal and the unscaled tail below it (the reflector is the tail times vssh[c]), and
  // rdsh[c] = R(c, c).
  if (c0 == 0) {
    double col[4], beta, tau, sc;
    pick_slot(x, m, col);  // column 0 is slot m
    householder_column(col, 0, l, vbuf[0], beta, tau, sc);
    if (l == 0) {
      tsh[0] = tau;
      rdsh[0] = beta;
      vssh[0] = sc;
    }
  }
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    if (c0 < p && c0 + 3 > j) {
      const double* vs = vbuf[j & 1];
      double v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = vs[64 * k + l];
      const double tau = tsh[j];
      double d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = fma(v[0], x[0][q], v[1] * x[1][q]) + fma(v[2], x[2][q], v[3] * x[3][q]);
      wave4_sums(d);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double wq = c0 + (q ^ m) > j ? d[q] * tau : 0.0;  // columns up to j are final
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k][q] = fma(-wq, v[k], x[k][q]);
      }
      const int cn = j + 1;
      if (cn < p && (cn & ~3) == c0) {
        const int sl = (cn & 3) ^ m;
        double col[4], beta, tn, sc;
        pick_slot(x, sl, col);
        householder_column(col, cn, l, vbuf[cn & 1], beta, tn, sc);
        if (l == 0) {
          tsh[cn] = tn;
          rdsh[cn] = beta;
          vssh[cn] = sc;
        }
      }
    }
    __syncthreads();
  }
  // write the reflectors, R and tau once
  double* V = a.V[side];
  double* Rb = a.Rout[side] + (int64_t)blockIdx.x * a.pmax;  // this block's R, rows 0..pmax-1
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + (q ^ m);
    if (c < p) {
      const double rd = rdsh[c], vsc = vssh[c];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = 64 * k + l;
        if (r < nr) V[row0 + r + (int64_t)c * a.ldv] = (r > c) ? x[k][q] * vsc : (r == c ? 1.0 : 0.0);
        if (r < a.pmax) Rb[r + (int64_t)c * a.ldr] = (r < c) ? x[k][q] : (r == c ? rd : 0.0);
      }
    }
  }
  if (t < p) a.tau[side][(int64_t)blockIdx.x * a.pmax + t] = tsh[t];
}

// Two builds of the same body: one register-lean enough (64 VGPRs, a few loop-invariant values
// spilled) for two 16-wave workgroups per CU, for the levels with more workgroups than CUs, where
// the second workgroup's steps fill the first one's latency; and one without that limit for the
// upper levels, where each CU runs a single block and the spills would only lengthen its chain.
template <class Src>
__global__ __launch_bounds__(kTsqrThreads) void k_tsqr_factor(Src in) {
  factor_block(kernel_args<FactorArgs>(in));
}
template <class Src>
__global__ __launch_bounds__(kTsqrThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_tsqr_factor_w8(
    Src in) {
  factor_block(kernel_args<FactorArgs>(in));
}

// Q formation in compact WY form on the FP64 matrix cores. The block's reflectors give
// H_0 H_1 .. H_{p-1} = I - V T V^T with T upper triangular and T^{-1} = diag(1/tau) +
// striu(V^T V) (the strictly upper part holds v_i . v_k), so with Y0 = [T_par; 0]:
//   X = V^T Y0 = V(0:p, :)^T T_par                 (MFMA; the transpose of V's top at the root)
//   (diag(1/tau) + striu(V^T V)) Z = X             (back substitution, row i from rows > i:
//                                                   Z(i,:) = tau_i (X(i,:) - sum_k S(i,k) Z(k,:)),
//                                                   so a zero tau gives a zero row)
//   Y = Y0 - V Z                                   (MFMA)
// MFMA v_mfma_f64_16x16x4: operand A lane l = A(l%16, l/16), B lane l = B(l/16, l%16), result
// item v of lane l = D(l/16 + 4v, l%16). Y is formed transposed (Y^T = Y0^T - Z^T V^T) so that
// each 16-lane group of a store writes 16 consecutive rows of one column.
typedef double wy4 __attribute__((ext_vector_type(4)));
constexpr int kWyThreads = 512;  // 8 waves
constexpr int kWyLd = kPMax + 1;

template <class Src>
__global__ __launch_bounds__(kWyThreads) void k_tsqr_apply_wy(Src in) {
  const ApplyArgs& a = kernel_args<ApplyArgs>(in);
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int kHalf = kTsqrRows / 2;    // rows of V staged at a time
  constexpr int kWaves = kWyThreads / 64;
  __shared__ double Vs[kHalf * kWyLd];  // V(r, c) of one half at Vs[r kWyLd + c], zero past p / nr
  __shared__ double S[kPMax * kWyLd];   // v_i . v_k (upper tiles; the rest zero)
  __shared__ double XZ[kPMax * kWyLd];  // X, then Z in place; zero outside p x p
  __shared__ double tsh[kPMax];
  const double* V = a.V[side] + row0;  // V(r, c) = V[r + c ldv], r < nr, c < p
  const int64_t ldv = a.ldv;
  const double* T = a.T[side];
  const int64_t toff = (int64_t)blockIdx.x * a.pmax;
  const int pt = (p + 15) >> 4;  // 16-column tiles in use
  const int pk = (p + 3) >> 2;   // 4-row steps over p
  const int ntiles = pt * (pt + 1) / 2;

  for (int e = t; e < kPMax * kWyLd; e += kWyThreads) {
    S[e] = 0.0;
    XZ[e] = 0.0;
  }
  if (t < kPMax) tsh[t] = t < p ? a.tau[side][toff + t] : 0.0;

  // upper tiles q = wave, wave + 8 of S (I <= J), accumulated over both halves
  int tI[2], tJ[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    int q = wave + kWaves * m, I = 0;
    while (q >= pt - I && I < pt) {
      q -= pt - I;
      ++I;
    }
    tI[m] = I;
    tJ[m] = I + q;
  }
  wy4 sacc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  wy4 xacc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  double vb0[16], vb1[16];  // -V(16 R + lr, 4 s + lk) for this wave's row tiles R = wave, wave + 8

  // the loads of both halves of V are issued here, so that the second half's arrive while the
  // first half's products run (clamped indices: every load reads a valid element)
  constexpr int kPer = kHalf * kPMax / kWyThreads;  // 16
  double raw[2][kPer];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kWyThreads * m, r = e % kHalf, c = e / kHalf;
      raw[h][m] = V[min(h * kHalf + r, nr - 1) + (int64_t)min(c, p - 1) * ldv];
    }
  // and the parent piece T_par (p x p), kept in registers until V's staging buffer is free
  constexpr int kTPer = kPMax * kPMax / kWyThreads;  // 8
  double tpre[kTPer];
  if (T) {
#pragma unroll
    for (int m = 0; m < kTPer; ++m) {
      const int e = t + kWyThreads * m, r = e % kPMax, c = e / kPMax;
      tpre[m] = T[toff + min(r, p - 1) + (int64_t)min(c, p - 1) * a.ldt];
    }
  }

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int hr0 = h * kHalf;
    if (hr0 < nr) {  // uniform
    // stage rows hr0 .. hr0 + 127 of V
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kWyThreads * m, r = e % kHalf, c = e / kHalf;
      keep_loaded(raw[h][m]);
      Vs[r * kWyLd + c] = (hr0 + r < nr && c < p) ? raw[h][m] : 0.0;
    }
    __syncthreads();
    const int nks = (min(nr - hr0, kHalf) + 3) >> 2;  // 4-row steps in this half
    // S += V_h^T V_h on this wave's tiles (rows below 16 I are zero in the I columns)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (wave + kWaves * m >= ntiles) continue;
      const int I = tI[m], J = tJ[m];
      for (int ks = max(0, (16 * I - hr0) >> 2); ks < nks; ++ks) {
        const double* row = Vs + (4 * ks + lk) * kWyLd;
        sacc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * I + lr], row[16 * J + lr], sacc[m], 0, 0, 0);
      }
    }
    // X = V(0:p, :)^T T_par from the first half (p <= 64 rows)
    if (h == 0 && T) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int q = wave + kWaves * m;
        if (q >= pt * pt) continue;
        const int I = q / pt, J = q % pt;
        for (int k0 = 4 * I; k0 < pk; k0 += 4) {
          double tv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = 4 * (k0 + u) + lk;
            tv[u] = T[toff + min(r, p - 1) + (int64_t)min(16 * J + lr, p - 1) * a.ldt];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = 4 * (k0 + u) + lk;
            keep_loaded(tv[u]);
            const double b = (r < p && 16 * J + lr < p) ? tv[u] : 0.0;
            xacc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[r * kWyLd + 16 * I + lr], b, xacc[m], 0, 0, 0);
          }
        }
      }
    }
    // operands of the final product for this wave's row tile in this half
    {
      const int R = wave + kWaves * h;
      const int lrow = 16 * R + lr - hr0;  // row within the half
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const double x = -Vs[lrow * kWyLd + 4 * ks + lk];
        if (h == 0)
          vb0[ks] = x;
        else
          vb1[ks] = x;
      }
    }
    __syncthreads();
    }
  }
  // V's staging buffer now holds T_par (zero outside p x p) for the final product
  if (T) {
#pragma unroll
    for (int m = 0; m < kTPer; ++m) {
      const int e = t + kWyThreads * m, r = e % kPMax, c = e / kPMax;
      keep_loaded(tpre[m]);
      Vs[r * kWyLd + c] = (r < p && c < p) ? tpre[m] : 0.0;
    }
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    if (wave + kWaves * m >= ntiles) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(16 * tI[m] + lk + 4 * v) * kWyLd + 16 * tJ[m] + lr] = sacc[m][v];
  }
  if (T) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int q = wave + kWaves * m;
      if (q >= pt * pt) continue;
      const int I = q / pt, J = q % pt;
#pragma unroll
      for (int v = 0; v < 4; ++v) XZ[(16 * I + lk + 4 * v) * kWyLd + 16 * J + lr] = xacc[m][v];
    }
  } else {
    for (int e = t; e < p * p; e += kWyThreads) {
      const int i = e / p, j = e % p;
      XZ[i * kWyLd + j] = V[j + (int64_t)i * ldv];  // X = V(0:p, 0:p)^T; j, i < p <= nr
    }
  }
  __syncthreads();

  // ---- back substitution by 16-row blocks from the bottom. In block b, wave 0 solves the
  // block's triangle with one lane per column (the 16 rows in registers; after z_w is known the
  // rows above it in the block are updated at once, so the dependent chain is one multiply and one
  // fma per row); then every wave takes output tiles of the update of the rows above the block,
  // X(0:16b, :) -= S(0:16b, block) Z(block, :), on the matrix cores. S is read once per block,
  // not once per column.
  for (int b = pt - 1; b >= 0; --b) {  // uniform
    const int r0 = 16 * b;
    if (wave == 0) {
      double x[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) x[w] = XZ[(r0 + w) * kWyLd + lane];
#pragma unroll
      for (int w = 15; w >= 0; --w) {
        const double z = tsh[r0 + w] * x[w];  // zero past p (tau and X are zero there)
        XZ[(r0 + w) * kWyLd + lane] = z;
#pragma unroll
        for (int w2 = 0; w2 < w; ++w2) x[w2] = fma(-S[(r0 + w2) * kWyLd + r0 + w], z, x[w2]);
      }
    }
    __syncthreads();
    if (b == 0) break;
    for (int q = wave; q < b * pt; q += kWaves) {  // tile (I, J): rows 16 I, columns 16 J
      const int I = q / pt, J = q % pt;
      wy4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = XZ[(16 * I + lk + 4 * v) * kWyLd + 16 * J + lr];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-S[(16 * I + lr) * kWyLd + r0 + 4 * kk + lk],
                                                   XZ[(r0 + 4 * kk + lk) * kWyLd + 16 * J + lr], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) XZ[(16 * I + lk + 4 * v) * kWyLd + 16 * J + lr] = acc[v];
    }
    __syncthreads();
  }

  // ---- Y^T = Y0^T - Z^T V^T for this wave's row tiles
  double* Y = a.Y[side] + row0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int R = wave + kWaves * h;
    const int row = 16 * R + lr;
    if (16 * R >= nr) continue;  // uniform
    wy4 acc[4];
    if (T) {  // Y0 = [T_par; 0], T_par staged in LDS (zero outside p x p)
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[J][v] = row < p ? Vs[row * kWyLd + 16 * J + lk + 4 * v] : 0.0;
    } else {
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[J][v] = (row < p && row == 16 * J + lk + 4 * v) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      if (ks >= pk) break;
      const double* Zk = XZ + (4 * ks + lk) * kWyLd + lr;
#pragma unroll
      for (int J = 0; J < 4; ++J)
        if (J < pt) acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(Zk[16 * J], h == 0 ? vb0[ks] : vb1[ks], acc[J], 0, 0, 0);
    }
    if (row < nr) {
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * J + lk + 4 * v;
          if (col < p) Y[row + (int64_t)col * a.ldy] = acc[J][v];
        }
    }
  }
}

// The same Q formation in a build lean enough for two workgroups per CU (at most 80 KB of LDS
// and 128 VGPRs), for the tree levels with more workgroups than CUs: V is staged by 64-row
// quarters into one 64 x kWyLd buffer, which holds S once V is consumed; the parent piece T_par
// and the final product's V operands are read from memory where they are used (the block read
// them moments before, so they come from L2) instead of waiting in registers. Every sum is formed
// in the same order as in k_tsqr_apply_wy, so the two builds give the same result.
template <class Src>
__global__ __launch_bounds__(kWyThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_tsqr_apply_lean(Src in) {
  const ApplyArgs& a = kernel_args<ApplyArgs>(in);
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int kQuarter = kPMax;         // rows of V staged at a time (= the rows of S)
  constexpr int kWaves = kWyThreads / 64;
  __shared__ double QS[kQuarter * kWyLd];  // V(r, c) of one quarter, zero past p / nr; then S
  __shared__ double XZ[kPMax * kWyLd];     // X, then Z in place; zero outside p x p
  __shared__ double tsh[kPMax];
  const double* V = a.V[side] + row0;  // V(r, c) = V[r + c ldv], r < nr, c < p
  const int64_t ldv = a.ldv;
  const double* T = a.T[side];
  const int64_t toff = (int64_t)blockIdx.x * a.pmax;
  const int pt = (p + 15) >> 4;
  const int pk = (p + 3) >> 2;
  const int ntiles = pt * (pt + 1) / 2;

  for (int e = t; e < kPMax * kWyLd; e += kWyThreads) XZ[e] = 0.0;
  if (t < kPMax) tsh[t] = t < p ? a.tau[side][toff + t] : 0.0;

  int tI[2], tJ[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    int q = wave + kWaves * m, I = 0;
    while (q >= pt - I && I < pt) {
      q -= pt - I;
      ++I;
    }
    tI[m] = I;
    tJ[m] = I + q;
  }
  wy4 sacc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  wy4 xacc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  constexpr int kPer = kQuarter * kPMax / kWyThreads;  // 8

  for (int qr0 = 0; qr0 < nr; qr0 += kQuarter) {  // uniform
    double raw[kPer];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kWyThreads * m, r = e % kQuarter, c = e / kQuarter;
      raw[m] = V[min(qr0 + r, nr - 1) + (int64_t)min(c, p - 1) * ldv];
    }
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = t + kWyThreads * m, r = e % kQuarter, c = e / kQuarter;
      keep_loaded(raw[m]);
      QS[r * kWyLd + c] = (qr0 + r < nr && c < p) ? raw[m] : 0.0;
    }
    __syncthreads();
    const int nks = (min(nr - qr0, kQuarter) + 3) >> 2;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (wave + kWaves * m >= ntiles) continue;
      const int I = tI[m], J = tJ[m];
      for (int ks = max(0, (16 * I - qr0) >> 2); ks < nks; ++ks) {
        const double* row = QS + (4 * ks + lk) * kWyLd;
        sacc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * I + lr], row[16 * J + lr], sacc[m], 0, 0, 0);
      }
    }
    if (qr0 == 0 && T) {  // X = V(0:p, :)^T T_par (p <= 64 rows: the first quarter)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int q = wave + kWaves * m;
        if (q >= pt * pt) continue;
        const int I = q / pt, J = q % pt;
        for (int k0 = 4 * I; k0 < pk; k0 += 4) {
          double tv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = 4 * (k0 + u) + lk;
            tv[u] = T[toff + min(r, p - 1) + (int64_t)min(16 * J + lr, p - 1) * a.ldt];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = 4 * (k0 + u) + lk;
            keep_loaded(tv[u]);
            const double b = (r < p && 16 * J + lr < p) ? tv[u] : 0.0;
            xacc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(QS[r * kWyLd + 16 * I + lr], b, xacc[m], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  // the staging buffer becomes S: zero, then the upper tiles
  for (int e = t; e < kPMax * kWyLd; e += kWyThreads) QS[e] = 0.0;
  __syncthreads();
  double* S = QS;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    if (wave + kWaves * m >= ntiles) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(16 * tI[m] + lk + 4 * v) * kWyLd + 16 * tJ[m] + lr] = sacc[m][v];
  }
  if (T) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int q = wave + kWaves * m;
      if (q >= pt * pt) continue;
      const int I = q / pt, J = q % pt;
#pragma unroll
      for (int v = 0; v < 4; ++v) XZ[(16 * I + lk + 4 * v) * kWyLd + 16 * J + lr] = xacc[m][v];
    }
  } else {
    for (int e = t; e < p * p; e += kWyThreads) {
      const int i = e / p, j = e % p;
      XZ[i * kWyLd + j] = V[j + (int64_t)i * ldv];  // X = V(0:p, 0:p)^T; j, i < p <= nr
    }
  }
  __syncthreads();

  // back substitution by 16-row blocks from the bottom (as in k_tsqr_apply_wy)
  for (int b = pt - 1; b >= 0; --b) {  // uniform
    const int r0 = 16 * b;
    if (wave == 0) {
      double x[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) x[w] = XZ[(r0 + w) * kWyLd + lane];
#pragma unroll
      for (int w = 15; w >= 0; --w) {
        const double z = tsh[r0 + w] * x[w];
        XZ[(r0 + w) * kWyLd + lane] = z;
#pragma unroll
        for (int w2 = 0; w2 < w; ++w2) x[w2] = fma(-S[(r0 + w2) * kWyLd + r0 + w], z, x[w2]);
      }
    }
    __syncthreads();
    if (b == 0) break;
    for (int q = wave; q < b * pt; q += kWaves) {
      const int I = q / pt, J = q % pt;
      wy4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = XZ[(16 * I + lk + 4 * v) * kWyLd + 16 * J + lr];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-S[(16 * I + lr) * kWyLd + r0 + 4 * kk + lk],
                                                   XZ[(r0 + 4 * kk + lk) * kWyLd + 16 * J + lr], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) XZ[(16 * I + lk + 4 * v) * kWyLd + 16 * J + lr] = acc[v];
    }
    __syncthreads();
  }

  // Y^T = Y0^T - Z^T V^T for this wave's row tiles; T_par and V from memory
  double* Y = a.Y[side] + row0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int R = wave + kWaves * h;
    const int row = 16 * R + lr;
    if (16 * R >= nr) continue;  // uniform
    double vb[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int c = 4 * ks + lk;
      vb[ks] = V[min(row, nr - 1) + (int64_t)min(c, p - 1) * ldv];
    }
    wy4 acc[4];
    if (T) {
      double tp[4][4];
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * J + lk + 4 * v;
          tp[J][v] = T[toff + min(row, p - 1) + (int64_t)min(c, p - 1) * a.ldt];
        }
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * J + lk + 4 * v;
          keep_loaded(tp[J][v]);
          acc[J][v] = (row < p && c < p) ? tp[J][v] : 0.0;
        }
    } else {
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[J][v] = (row < p && row == 16 * J + lk + 4 * v) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      keep_loaded(vb[ks]);
      vb[ks] = (row < nr && 4 * ks + lk < p) ? -vb[ks] : 0.0;
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      if (ks >= pk) break;
      const double* Zk = XZ + (4 * ks + lk) * kWyLd + lr;
#pragma unroll
      for (int J = 0; J < 4; ++J)
        if (J < pt) acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(Zk[16 * J], vb[ks], acc[J], 0, 0, 0);
    }
    if (row < nr) {
#pragma unroll
      for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * J + lk + 4 * v;
          if (col < p) Y[row + (int64_t)col * a.ldy] = acc[J][v];
        }
    }
  }
}

// ----------------------------------------------------------------------------------------
// Tree layout: level 0 factors n rows in blocks of kTsqrRows; each level above stacks the R
// factors of g = kTsqrRows / pmax blocks. `get(bytes)` supplies each buffer (nullptr: failure);
// buffers of sides >= nsides, and level 0's Y when Q is written to the caller's matrix
// (level0_y false), are not requested.
template <typename Get>
static int tsqr_layout(TsqrPlan* p, int64_t n, int pmax, int nsides, bool level0_y, Get&& get) {
  if (pmax < 1 || pmax > kPMax || n < 1) return LRP_EINVAL;
  *p = TsqrPlan{};
  p->n = n;
  p->pmax = pmax;
  int64_t rows = n;
  int br = kTsqrRows;
  int L = 0;
  const int g = kTsqrRows / pmax;  // R factors per block above the leaves
  while (true) {
    if (L >= kMaxLevels) return LRP_EINVAL;
    TsqrLevel& lv = p->lev[L];
    lv.rows = rows;
    lv.block_rows = br;
    lv.nblocks = (int)((rows + br - 1) / br);
    for (int s = 0; s < nsides; ++s) {
      const size_t vb = sizeof(double) * (size_t)rows * pmax;
      const size_t tb = sizeof(double) * (size_t)lv.nblocks * pmax;
      const size_t rb = sizeof(double) * (size_t)lv.nblocks * pmax * pmax;
      // no initialisation: every element of R that is read (columns below the active width,
      // all pmax rows) is written by the factorization first. (A plain memset here would run
      // on the null stream, unordered with the context's non-blocking stream.)
      if (!(lv.V[s] = get(vb)) || !(lv.tau[s] = get(tb)) || !(lv.Rout[s] = get(rb))) return LRP_ENOMEM;
      if ((L > 0 || level0_y) && !(lv.Y[s] = get(vb))) return LRP_ENOMEM;
    }
    ++L;
    if (lv.nblocks == 1) break;
    rows = (int64_t)lv.nblocks * pmax;
    br = g * pmax;
  }
  p->nlevels = L;
  return LRP_OK;
}

int tsqr_plan(TsqrPlan* p, int64_t n, int pmax) {
  return tsqr_layout(p, n, pmax, 2, true, [](size_t bytes) -> double* {
    void* q = nullptr;
    return hipMalloc(&q, bytes) == hipSuccess ? (double*)q : nullptr;
  });
}

int tsqr_run(const TsqrPlan& p, const TsqrIO& io, hipStream_t s) {
  const int ns = io.nsides;
  // bottom-up factorization
  for (int L = 0; L < p.nlevels; ++L) {
    const TsqrLevel& lv = p.lev[L];
    FactorArgs f{};
    f.st = io.st;
    f.ncols[0] = io.ncols[0];
    f.ncols[1] = io.ncols[1];
    if (L == 0) {
      f.in[0] = io.X[0];
      f.in[1] = io.X[1];
      f.in_f32 = io.x_f32;
      f.ldin = io.ldx;
    } else {
      const TsqrLevel& pv = p.lev[L - 1];
      f.in[0] = pv.Rout[0];
      f.in[1] = pv.Rout[1];
      f.in_f32 = 0;
      f.ldin = (int64_t)pv.nblocks * p.pmax;
    }
    f.rows = lv.rows;
    f.block_rows = lv.block_rows;
    f.pmax = p.pmax;
    f.ldv = lv.rows;
    f.ldr = (int64_t)lv.nblocks * p.pmax;
    for (int q = 0; q < 2; ++q) {
      f.V[q] = lv.V[q];
      f.tau[q] = lv.tau[q];
      f.Rout[q] = lv.Rout[q];
    }
    if ((int64_t)lv.nblocks * ns > kCUs)
      LRP_LAUNCH_G(K_TSQR_FACTOR, k_tsqr_factor_w8<FactorArgs>, k_tsqr_factor_w8<GroupRef>, dim3(lv.nblocks, ns), dim3(kTsqrThreads), 0, s, f);
    else
      LRP_LAUNCH_G(K_TSQR_FACTOR, k_tsqr_factor<FactorArgs>, k_tsqr_factor<GroupRef>, dim3(lv.nblocks, ns), dim3(kTsqrThreads), 0, s, f);
  }
  // top-down formation of Q
  for (int L = p.nlevels - 1; L >= 0; --L) {
    const TsqrLevel& lv = p.lev[L];
    ApplyArgs a{};
    a.st = io.st;
    a.ncols[0] = io.ncols[0];
    a.ncols[1] = io.ncols[1];
    a.ldv = lv.rows;
    a.rows = lv.rows;
    a.block_rows = lv.block_rows;
    a.pmax = p.pmax;
    for (int q = 0; q < 2; ++q) {
      a.V[q] = lv.V[q];
      a.tau[q] = lv.tau[q];
      a.T[q] = (L == p.nlevels - 1) ? nullptr : p.lev[L + 1].Y[q];
      a.Y[q] = (L == 0 && io.Q[q]) ? io.Q[q] : lv.Y[q];
    }
    a.ldt = (L == p.nlevels - 1) ? 0 : p.lev[L + 1].rows;
    a.ldy = (L == 0 && io.Q[0]) ? io.ldq : lv.rows;
    if ((int64_t)lv.nblocks * ns > kCUs)
      LRP_LAUNCH_G(K_TSQR_APPLY, k_tsqr_apply_lean<ApplyArgs>, k_tsqr_apply_lean<GroupRef>, dim3(lv.nblocks, ns), dim3(kWyThreads), 0, s, a);
    else
      LRP_LAUNCH_G(K_TSQR_APPLY, k_tsqr_apply_wy<ApplyArgs>, k_tsqr_apply_wy<GroupRef>, dim3(lv.nblocks, ns), dim3(kWyThreads), 0, s, a);
  }
  return launch_status();
}

// ----------------------------------------------------------------------------------------
// The QR without allocation: the tree's workspace is a static device array (one copy per GPU,
// held until the process ends), found once per device with hipGetSymbolAddress. The host never
// uses the array's name as an address; kernels get the device pointer.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LRP_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LRP_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LRP_OK;
}

// Workspace bytes of a one-sided tree for n rows and p columns (each buffer 256-byte aligned).
static size_t tsqr_noalloc_bytes(int64_t n, int p, int* rc) {
  size_t total = 0;
  TsqrPlan plan;
  *rc = tsqr_layout(&plan, n, p, 1, false, [&](size_t bytes) -> double* {
    total += (bytes + 255) & ~size_t(255);
    return reinterpret_cast<double*>(256);  // any non-null value: nothing is dereferenced
  });
  return total;
}

__global__ void k_copy_r(const double* __restrict__ src, int lds, int p, double* __restrict__ R, int64_t ldr) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  const int i = e % p, j = e / p;
  R[i + (int64_t)j * ldr] = i <= j ? src[i + (int64_t)j * lds] : 0.0;
}

}  // namespace lrp

extern "C" {

int64_t lrp_tsqr_noalloc_max_bytes(void) { return (int64_t)lrp::kScratchBytes; }

int lrp_tsqr_noalloc(int64_t n, int32_t ncols, const double* A, int64_t lda, double* Q, int64_t ldq, double* R,
                     int64_t ldr, void* stream) {
  using namespace lrp;
  if (!A || !Q || !R || n < 1 || ncols < 1 || ncols > kPMax || ncols > n) return LRP_EINVAL;
  if (lda < n || ldq < n || ldr < ncols) return LRP_EINVAL;
  const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (uintptr_t)(((ncols - 1) * lda + n) * 8);
  const uintptr_t q0 = (uintptr_t)Q, q1 = q0 + (uintptr_t)(((ncols - 1) * ldq + n) * 8);
  if (a0 < q1 && q0 < a1) return LRP_EINVAL;
  int rc = LRP_OK;
  const size_t need = tsqr_noalloc_bytes(n, ncols, &rc);
  if (rc != LRP_OK) return LRP_EINVAL;
  if (need > kScratchBytes) return LRP_ESIZE;
  void* base = nullptr;
  rc = scratch_ptr(&base);
  if (rc != LRP_OK) return rc;
  unsigned char* cur = static_cast<unsigned char*>(base);
  TsqrPlan plan;
  rc = tsqr_layout(&plan, n, ncols, 1, false, [&](size_t bytes) -> double* {
    double* q = reinterpret_cast<double*>(cur);
    cur += (bytes + 255) & ~size_t(255);
    return q;
  });
  if (rc != LRP_OK) return rc;
  TsqrIO io{};
  io.st = nullptr;
  io.ncols[0] = ncols;
  io.ncols[1] = 0;
  io.nsides = 1;
  io.X[0] = A;
  io.x_f32 = 0;
  io.ldx = lda;
  io.Q[0] = Q;
  io.ldq = ldq;
  hipStream_t s = (hipStream_t)stream;
  rc = tsqr_run(plan, io, s);
  if (rc != LRP_OK) return rc;
  const int pp = ncols * ncols;
  hipLaunchKernelGGL(k_copy_r, dim3((pp + 255) / 256), dim3(256), 0, s, tsqr_R(plan, 0), ncols, ncols, R, ldr);
  return launch_status();
}

}  // extern "C"
