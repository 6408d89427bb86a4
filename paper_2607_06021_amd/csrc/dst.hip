// Orthonormal DST-I of the columns of an n x c matrix, n + 1 = M a power of two.
//
// (Z x)_i = sqrt(2/M) sum_k x_k sin(pi i k / M) (Section 3: the eigenvectors of T).
// Two real columns a, b share one complex FFT of length L = 2M of the odd extension
// z = ext(a) + i ext(b), ext(x) = [0, x_1..x_{M-1}, 0, -x_{M-1}..-x_1]. Its DFT is
// Z_k = 2 y_b(k) - 2 i y_a(k) with y(k) = sum_j x_j sin(pi j k / M), so
// (Z a)_k = -Im Z_k / sqrt(2M) and (Z b)_k = Re Z_k / sqrt(2M), k = 1..M-1.
//
// FFTs are Stockham autosort (decimation in time): every thread holds E = 16 elements of one
// sequence in registers, element tt + TP e (TP = P/E threads per sequence), does radix-16
// butterflies (radix 2/4/8 for the remainder of log2 P) in registers and exchanges through LDS
// between stages; the output ends up in the same register layout as the input.
//
// L <= 4096: one pass, whole sequences per workgroup.
// L  > 4096: four-step, L = L1 L2, input index j = j1 + L1 j2, output index k = k2 + L2 k1.
//   Pass 1: for each j1, A_j1(k2) = DFT over j2 (length L2) of z[j1 + L1 j2];
//           B_j1(k2) = W_L^{j1 k2} A_j1(k2).
//   Pass 2: for each k2, Z[k2 + L2 k1] = DFT over j1 (length L1) of B_j1(k2).
//   Odd symmetry halves both passes. Since z[L - j] = -z[j], column L1 - j1 of pass 1 is column
//   j1 reversed and negated, so A_{L1-j1}(k2) = -W_L2^{-k2} A_j1(-k2) and, for k2 > 0,
//   B_{L1-j1}(k2) = -W_L1^{-j1} B_j1(L2 - k2) (B_{L1-j1}(0) = -B_j1(0)). Pass 1 therefore
//   transforms only j1 = 0..L1/2, reading every input element once, and stores the
//   intermediate S[k2][j1], j1 = 0..L1/2: S = B_j1(k2) for k2 <= L2/2, and for k2 > L2/2 the
//   element B_{L1-j1}(L2-k2) = -W_L^{-j1 (L2-k2)} A_j1(k2) that column L2 - k2 of pass 2 needs.
//   Since Z[L - k] = -Z[k], pass 2 transforms only k2 = 0..L2/2: outputs k1 < L1/2 of column
//   k2 are Z[k2 + L2 k1], outputs k1 >= L1/2 give Z[(L2-k2) + L2 (L1-1-k1)] of the mirror column.
//   Each pass moves about n elements per column in and out.
// Twiddles come from tables built on the device from sincospi (exact arguments 2k/P).
#include <type_traits>

#include "lrp_kernels.h"

#define TRY_DST(expr)                 \
  do {                                \
    const int rc_ = (expr);           \
    if (rc_ != LRP_OK) return rc_;    \
  } while (0)

namespace lrp {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cneg(cx<T> a) {
  return {-a.x, -a.y};
}

// W_M^k = exp(-2 pi i k / M) for k < count, written as FP64 and FP32 tables.
__global__ void k_twiddle(double2* t64, float2* t32, int M, int count) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)M, &s, &c);
  t64[k] = make_double2(c, -s);
  t32[k] = make_float2((float)c, (float)-s);
}

// ---------------------------------------------------------------- register DFTs (forward)
// cos(pi/8), sin(pi/8), sqrt(1/2)
constexpr double kC8 = 0.92387953251128675613;
constexpr double kS8 = 0.38268343236508977173;
constexpr double kR2 = 0.70710678118654752440;

// v * W_16^J, J in [0, 16)
template <typename T, int J>
__device__ __forceinline__ cx<T> w16(cx<T> v) {
  constexpr int j = J & 15;
  if constexpr (j == 0) return v;
  else if constexpr (j == 4) return {v.y, -v.x};
  else if constexpr (j == 8) return {-v.x, -v.y};
  else if constexpr (j == 12) return {-v.y, v.x};
  else if constexpr (j == 2) return {T(kR2) * (v.x + v.y), T(kR2) * (v.y - v.x)};
  else if constexpr (j == 6) return {T(kR2) * (v.y - v.x), T(-kR2) * (v.x + v.y)};
  else if constexpr (j == 10) return {T(-kR2) * (v.x + v.y), T(kR2) * (v.x - v.y)};
  else if constexpr (j == 14) return {T(kR2) * (v.x - v.y), T(kR2) * (v.x + v.y)};
  else {
    // cos(pi j / 8) - i sin(pi j / 8) for odd j
    constexpr double c = (j == 1 || j == 15) ? kC8 : (j == 3 || j == 13) ? kS8 : (j == 5 || j == 11) ? -kS8 : -kC8;
    constexpr double s = (j == 1 || j == 7) ? kS8 : (j == 3 || j == 5) ? kC8 : (j == 9 || j == 15) ? -kS8 : -kC8;
    return cmul(v, cx<T>{T(c), T(-s)});
  }
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = {t1.x + t3.y, t1.y - t3.x};  // t1 - i t3
  a3 = {t1.x - t3.y, t1.y + t3.x};  // t1 + i t3
}

template <typename T, int R>
__device__ __forceinline__ void dft(cx<T> (&v)[R]) {
  if constexpr (R == 2) {
    const cx<T> t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // j = m + 2 j2: length-4 DFTs over j2, twiddle W_8^{m k2}, length-2 DFT over m
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    const cx<T> o0 = v[1], o1 = w16<T, 2>(v[3]), o2 = w16<T, 4>(v[5]), o3 = w16<T, 6>(v[7]);
    const cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  } else {
    static_assert(R == 16, "radix");
    // j = m + 4 j2: length-4 DFTs over j2 (result k2 at v[m + 4 k2]), twiddle W_16^{m k2},
    // then length-4 DFTs over m; output k2 + 4 k1.
    dft4(v[0], v[4], v[8], v[12]);
    dft4(v[1], v[5], v[9], v[13]);
    dft4(v[2], v[6], v[10], v[14]);
    dft4(v[3], v[7], v[11], v[15]);
    cx<T> u[16];
    u[0] = v[0];
    u[1] = v[1];
    u[2] = v[2];
    u[3] = v[3];
    u[4] = v[4];
    u[5] = w16<T, 1>(v[5]);
    u[6] = w16<T, 2>(v[6]);
    u[7] = w16<T, 3>(v[7]);
    u[8] = v[8];
    u[9] = w16<T, 2>(v[9]);
    u[10] = w16<T, 4>(v[10]);
    u[11] = w16<T, 6>(v[11]);
    u[12] = v[12];
    u[13] = w16<T, 3>(v[13]);
    u[14] = w16<T, 6>(v[14]);
    u[15] = w16<T, 9>(v[15]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      cx<T> a0 = u[4 * k2], a1 = u[4 * k2 + 1], a2 = u[4 * k2 + 2], a3 = u[4 * k2 + 3];
      dft4(a0, a1, a2, a3);
      v[k2] = a0;
      v[k2 + 4] = a1;
      v[k2 + 8] = a2;
      v[k2 + 12] = a3;
    }
  }
}

// LDS index with one padding slot per 16 elements (spreads power-of-two strides over banks)
__device__ __forceinline__ int pad(int p) { return p + (p >> 4); }
// LDS elements per sequence of length P; odd, so that equal positions of neighbouring
// sequences fall in different banks.
__host__ __device__ constexpr int seq_len(int P) { return P + P / 16 + 1; }

// One Stockham stage of radix R on a sequence of length P whose preceding stages have
// combined LS points. On entry x[e] is stage input element tt + TP e; on exit x[e] is the
// stage output in the same layout (through LDS unless this is the last stage).
template <typename T, int E, int P, int R, int LS>
__device__ __forceinline__ void stage(cx<T> (&x)[E], cx<T>* lds, int tt, const cx<T>* __restrict__ tw) {
  constexpr int TP = P / E, NB = E / R;
  constexpr bool kLast = (LS * R == P);
  constexpr int TWS = P / (LS * R);  // W_{LS R}^{s k} = W_P^{s k TWS}
  cx<T> y[E];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tt + TP * i;
    const int k = b & (LS - 1);
    cx<T> v[R];
#pragma unroll
    for (int s = 0; s < R; ++s) v[s] = x[i + NB * s];
    if constexpr (LS > 1) {
#pragma unroll
      for (int s = 1; s < R; ++s) v[s] = cmul(v[s], tw[s * k * TWS]);
    }
    dft<T, R>(v);
#pragma unroll
    for (int q = 0; q < R; ++q) y[i + NB * q] = v[q];
  }
  if constexpr (kLast) {
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = y[e];
  } else {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = tt + TP * i;
      const int k = b & (LS - 1);
#pragma unroll
      for (int q = 0; q < R; ++q) lds[pad((b - k) * R + k + q * LS)] = y[i + NB * q];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = lds[pad(tt + TP * e)];
  }
}

template <typename T, int E, int P, int LS>
__device__ __forceinline__ void stages16(cx<T> (&x)[E], cx<T>* lds, int tt, const cx<T>* __restrict__ tw) {
  if constexpr (LS < P) {
    stage<T, E, P, 16, LS>(x, lds, tt, tw);
    stages16<T, E, P, LS * 16>(x, lds, tt, tw);
  }
}

// Forward DFT of one sequence of length 2^LOGP held as x[e] = element tt + (P/E) e; tw[j] = W_P^j.
// Every thread of the block must call it (it contains barriers).
template <typename T, int LOGP, int E>
__device__ __forceinline__ void fft_seq(cx<T> (&x)[E], cx<T>* lds, int tt, const cx<T>* __restrict__ tw) {
  constexpr int P = 1 << LOGP;
  constexpr int R0 = 1 << (LOGP % 4 == 0 ? 4 : LOGP % 4);
  stage<T, E, P, R0, 1>(x, lds, tt, tw);
  stages16<T, E, P, R0>(x, lds, tt, tw);
}

// ---------------------------------------------------------------- data access helpers
__device__ inline bool dst_resolve(const DstArgs& a, const double*& X, int& ncols) {
  X = a.X;
  ncols = a.ncols;
  if (a.st) {
    const DevState* st = a.st;
    if (st->status < 0) return false;
    if (a.pick_ret) {
      X = st->ret ? a.X1 : a.X;
      ncols = st->zero ? 0 : st->r_final;
    }
  }
  return true;
}

__device__ inline void col_scales(const DstArgs& a, int ca, int cb, int ncols, double& sa, double& sb) {
  sa = a.outscale;
  sb = a.outscale;
  if (a.scale) {
    if (ca < ncols) sa *= a.scale[ca];
    if (cb < ncols) sb *= a.scale[cb];
  }
}

// Element j of the odd extension of the pair (xa, xb); null columns read as 0.
template <typename T>
__device__ __forceinline__ cx<T> load_z(const double* __restrict__ xa, const double* __restrict__ xb,
                                        int64_t M, int64_t j) {
  int64_t src;
  T sg;
  if (j >= 1 && j < M) {
    src = j - 1;
    sg = T(1);
  } else if (j > M) {
    src = 2 * M - j - 1;
    sg = T(-1);
  } else {
    return {T(0), T(0)};
  }
  const T va = xa ? (T)xa[src] : T(0);
  const T vb = xb ? (T)xb[src] : T(0);
  return {va * sg, vb * sg};
}

// Output k (1..M-1) of the pair: column a gets -Im Z sa, column b gets Re Z sb (0 beyond ncols).
template <typename T>
__device__ __forceinline__ void put_pair(const DstArgs& a, int ca, int cb, int ncols, int64_t k, cx<T> Z,
                                         double sa, double sb) {
  const double va = ca < ncols ? -(double)Z.y * sa : 0.0;
  const double vb = cb < ncols ? (double)Z.x * sb : 0.0;
  if (a.Yf) {  // FP32 destination (spectral factors of the mixed-precision path)
    a.Yf[(k - 1) + (int64_t)ca * a.ldy] = (float)va;
    if (cb < a.ncols_out) a.Yf[(k - 1) + (int64_t)cb * a.ldy] = (float)vb;
  } else {
    a.Y[(k - 1) + (int64_t)ca * a.ldy] = va;
    if (cb < a.ncols_out) a.Y[(k - 1) + (int64_t)cb * a.ldy] = vb;
  }
}

__host__ __device__ constexpr int single_seqs(int logL) {
  return (1 << logL) / 16 >= 64 ? 1 : 64 / ((1 << logL) >= 16 ? (1 << logL) / 16 : 1);
}
// Largest power-of-two tile (columns per workgroup) with at most `cap` columns, at most 512
// threads (16 elements each) and at most lds_max bytes of LDS: the whole 160 KB of a CU for the
// wide tiles (longer row pieces), half of it for the narrow ones (two workgroups per CU).
constexpr int kLdsWide = 160 * 1024, kLdsNarrow = 80 * 1024;
__host__ __device__ constexpr int lds_pass1(int log2, int tj, int esz) { return tj * seq_len(1 << log2) * esz; }
__host__ __device__ constexpr int lds_pass2(int log1, int tk, int esz) {
  return (tk * seq_len(1 << log1) > (1 << log1) * (tk + 1) ? tk * seq_len(1 << log1) : (1 << log1) * (tk + 1)) * esz;
}
__host__ __device__ constexpr int tile1_for(int log2, int esz, int cap, int lds_max) {
  int t = cap;
  while (t > 1 && (lds_pass1(log2, t, esz) > lds_max || t * ((1 << log2) / 16) > 512)) t >>= 1;
  return t;
}
__host__ __device__ constexpr int tile2_for(int log1, int esz, int cap, int lds_max) {
  int t = cap;
  while (t > 1 && (lds_pass2(log1, t, esz) > lds_max || t * ((1 << log1) / 16) > 512)) t >>= 1;
  return t;
}
// Column tiles of the four-step passes: the widest that fit (CAP = 0), or at most CAP columns --
// narrow tiles for launches that would otherwise leave CUs idle (few column pairs). A column's
// transform is the same whatever tile it sits in.
constexpr int kNarrow1 = 8, kNarrow2 = 4;
template <typename T, int CAP = 0>
__host__ __device__ constexpr int tile1_of(int log2) {
  return tile1_for(log2, (int)sizeof(cx<T>), CAP ? CAP : 32, CAP ? kLdsNarrow : kLdsWide);
}
template <typename T, int CAP = 0>
__host__ __device__ constexpr int tile2_of(int log1) {
  return tile2_for(log1, (int)sizeof(cx<T>), CAP ? CAP : 16, CAP ? kLdsNarrow : kLdsWide);
}

// ---------------------------------------------------------------- L <= 4096: one pass
template <typename T, int LOGL>
__global__ __launch_bounds__(512) void k_dst_single(DstArgs a) {
  constexpr int L = 1 << LOGL, E = L < 16 ? L : 16, TP = L / E;
  constexpr int SEQS = single_seqs(LOGL), SEQ = seq_len(L);
  __shared__ cx<T> lds[SEQS * SEQ];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int tt = threadIdx.x % TP, sl = threadIdx.x / TP;
  const int ca = 2 * (blockIdx.x * SEQS + sl), cb = ca + 1;
  const int64_t M = L / 2;
  const double* xa = ca < ncols ? X + (int64_t)ca * a.ldx : nullptr;
  const double* xb = cb < ncols ? X + (int64_t)cb * a.ldx : nullptr;
  cx<T> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) x[e] = load_z<T>(xa, xb, M, tt + TP * e);
  fft_seq<T, LOGL, E>(x, lds + sl * SEQ, tt, reinterpret_cast<const cx<T>*>(a.t1));
  if (ca >= a.ncols_out) return;
  double sa, sb;
  col_scales(a, ca, cb, ncols, sa, sb);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tt + TP * e;
    if (k >= 1 && k < M) put_pair<T>(a, ca, cb, ncols, k, x[e], sa, sb);
  }
}

// XCD-aware order of the full tiles: the hardware hands consecutive workgroups to the 8 XCDs in
// turn, so workgroup b runs on XCD b mod 8. Giving the workgroups of one XCD consecutive tiles
// (b = 8 q + x takes tile x per + q) lets the neighbouring pieces of a cache line that adjacent
// tiles read or write meet in that XCD's L2 instead of going to memory separately. The tail
// past 8 per stays in place.
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int per = nb >> 3;
  return b < 8 * per ? (b & 7) * per + (b >> 3) : b;
}

// ---------------------------------------------------------------- four-step pass 1
// Block: TJ columns j1 (lane-fastest, so global reads and writes are coalesced) x L2/16 threads;
// TJ = 16 (FP64) or 32 (FP32) columns, so each row of the input is read in 128- or 256-byte pieces.
template <typename T, int LOG2, int CAP = 0>
__global__ __launch_bounds__(512) void k_dst_pass1(DstArgs a) {
  constexpr int L2 = 1 << LOG2, E = 16, TP = L2 / E;
  constexpr int TJ = tile1_of<T, CAP>(LOG2), SEQ = seq_len(L2);
  __shared__ cx<T> lds[TJ * SEQ];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int L1 = 1 << a.logL1;
  // blocks: the L1/(2 TJ) full column tiles of every pair first, then the tile holding the
  // single column j1 = L1/2 of every pair, so that the light tiles form the tail of the grid
  const int nfull = (L1 / 2) / TJ;
  const int npairs = gridDim.x / (nfull + 1);
  const int b = blockIdx.x < nfull * npairs ? xcd_order(blockIdx.x, nfull * npairs) : blockIdx.x;
  const int tile = b < nfull * npairs ? b % nfull : nfull;
  const int pair = b < nfull * npairs ? b / nfull : b - nfull * npairs;  // within this batch
  const int ca = 2 * (a.pair0 + pair), cb = ca + 1;
  if (ca >= a.ncols_out || ca >= ncols) return;  // all-zero pairs are written by pass 2 alone
  const int cl = threadIdx.x % TJ, tt = threadIdx.x / TJ;
  const int64_t M = (int64_t)L1 * L2 / 2;
  const int j1 = tile * TJ + cl;
  const bool valid = j1 <= L1 / 2;
  const double* xa = valid ? X + (int64_t)ca * a.ldx : nullptr;
  const double* xb = valid && cb < ncols ? X + (int64_t)cb * a.ldx : nullptr;
  cx<T> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) x[e] = load_z<T>(xa, xb, M, j1 + (int64_t)L1 * (tt + TP * e));
  fft_seq<T, LOG2, E>(x, lds + cl * SEQ, tt, reinterpret_cast<const cx<T>*>(a.t2));
  if (!valid) return;
  const cx<T>* thi = reinterpret_cast<const cx<T>*>(a.t1);  // W_L^{L2 h} = W_L1^h
  const cx<T>* tlo = reinterpret_cast<const cx<T>*>(a.tl);  // W_L^b, b < L2
  cx<T>* S = reinterpret_cast<cx<T>*>(a.work) + (int64_t)pair * L2 * a.s1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k2 = tt + TP * e;
    const bool hi = k2 > L2 / 2;
    const int64_t m = (int64_t)j1 * (hi ? L2 - k2 : k2);  // <= L/4
    const cx<T> w = cmul(thi[m >> LOG2], tlo[m & (L2 - 1)]);
    S[(int64_t)k2 * a.s1 + j1] = hi ? cneg(cmulc(x[e], w)) : cmul(x[e], w);
  }
}

// ---------------------------------------------------------------- four-step pass 2
// Block: TK columns k2 (k2 = 0..L2/2) x L1/16 threads (lane-fastest along the sequence, so rows
// of the intermediate are read contiguously); outputs are staged in LDS and written TK at a time.
template <typename T, int LOG1, int CAP = 0>
__global__ __launch_bounds__(512) void k_dst_pass2(DstArgs a) {
  constexpr int L1 = 1 << LOG1, E = 16, TP = L1 / E;
  constexpr int TK = tile2_of<T, CAP>(LOG1), SEQ = seq_len(L1);
  constexpr int OST = TK + 1;  // staging row stride
  constexpr int NLDS = TK * SEQ > L1 * OST ? TK * SEQ : L1 * OST;
  __shared__ cx<T> lds[NLDS];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int L2 = 1 << a.logL2;
  // blocks ordered as in pass 1: full tiles of k2 < L2/2 first, the k2 = L2/2 tiles last
  const int nfull = (L2 / 2) / TK;
  const int npairs = gridDim.x / (nfull + 1);
  const int b = blockIdx.x < nfull * npairs ? xcd_order(blockIdx.x, nfull * npairs) : blockIdx.x;
  const int tile = b < nfull * npairs ? b % nfull : nfull;
  const int pair = b < nfull * npairs ? b / nfull : b - nfull * npairs;  // within this batch
  const int ca = 2 * (a.pair0 + pair), cb = ca + 1;
  if (ca >= a.ncols_out) return;
  const int k0 = tile * TK;
  const int nthreads = TK * TP;
  double sa, sb;
  col_scales(a, ca, cb, ncols, sa, sb);
  // staged entry g: kl = g % TK, row = g / TK; rows < L1/2 hold Z[k2 + L2 row] of column
  // k2 = k0 + kl, rows L1/2 + m hold Z[(L2 - k2) + L2 m] (already negated).
  auto write_out = [&](bool zero) {
    for (int g = threadIdx.x; g < L1 * TK; g += nthreads) {
      const int kl = g % TK, row = g / TK;
      const int k2 = k0 + kl;
      int64_t k;
      if (row < L1 / 2) {
        if (k2 > L2 / 2) continue;
        k = k2 + (int64_t)L2 * row;
        if (k == 0) continue;
      } else {
        if (k2 == 0 || k2 >= L2 / 2) continue;
        k = (L2 - k2) + (int64_t)L2 * (row - L1 / 2);
      }
      const cx<T> Z = zero ? cx<T>{T(0), T(0)} : lds[row * OST + kl];
      put_pair<T>(a, ca, cb, ncols, k, Z, sa, sb);
    }
  };
  if (ca >= ncols) {  // both columns zero
    write_out(true);
    return;
  }
  const int tt = threadIdx.x % TP, kl = threadIdx.x / TP;
  const int k2 = k0 + kl;
  const bool valid = k2 <= L2 / 2;
  const cx<T>* S = reinterpret_cast<const cx<T>*>(a.work) + (int64_t)pair * L2 * a.s1;
  const cx<T>* t1 = reinterpret_cast<const cx<T>*>(a.t1);  // W_L1^j
  cx<T> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j1 = tt + TP * e;
    cx<T> v{T(0), T(0)};
    if (valid) {
      if (j1 <= L1 / 2) {
        v = S[(int64_t)k2 * a.s1 + j1];
      } else {
        const int jm = L1 - j1;
        if (k2 == 0)
          v = cneg(S[jm]);
        else if (k2 == L2 / 2)
          v = cneg(cmulc(S[(int64_t)k2 * a.s1 + jm], t1[jm]));
        else
          v = S[(int64_t)(L2 - k2) * a.s1 + jm];
      }
    }
    x[e] = v;
  }
  fft_seq<T, LOG1, E>(x, lds + kl * SEQ, tt, t1);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k1 = tt + TP * e;
    if (k1 < L1 / 2)
      lds[k1 * OST + kl] = x[e];
    else
      lds[(L1 / 2 + (L1 - 1 - k1)) * OST + kl] = cneg(x[e]);
  }
  __syncthreads();
  write_out(false);
}

// ----------------------------------------------------------------------------------------
// n + 1 not a power of two: Bluestein's chirp-z method. With w = W_L (L = 2(n+1)) and
// c_j = w^{j^2/2} = exp(-pi i (j^2 mod 2L)/L), jk = (j^2 + k^2 - (k-j)^2)/2 gives
//   Z_k = sum_j z_j w^{jk} = c_k sum_j (z_j c_j) conj(c_{k-j}),
// a circular convolution of a_j = z_j c_j (zero past L) with b_m = conj(c_|m|) (|m| < L) over
// M >= 2L - 1 points: Z_k = c_k IDFT_M(DFT_M(a) DFT_M(b))_k, and IDFT(x) = conj(DFT(conj x))/M.
// DFT_M(b) is a table built at set-up. Per column pair: a forward FFT of a (the chirp folded
// into the loads), the product with the table (conjugated, folded into the FFT's stores), a
// second forward FFT, and the outputs c_k conj(.)/M for k = 1..n (folded into its stores).
// M <= 4096: one kernel; above, each FFT is four-step (M = M1 M2, input j = j1 + M1 j2, output
// k = k2 + M2 k1: pass 1 transforms over j2 for each j1 and applies W_M^{j1 k2}, pass 2
// transforms over j1 for each k2).
struct BsArgs {
  DstArgs d;           // columns, destination, scales (as the power-of-two path)
  int64_t N;           // n + 1 (L = 2N)
  int logM1;           // four-step: M1 = 2^logM1 (pass-2 length); M2 = 2^logM2 (pass-1 length)
  int64_t s1;          // row stride of the pass-1 -> pass-2 intermediate (complex elements)
  const void* chirp;   // L entries
  const void* bhat;    // M entries
  const void *t1, *t2, *tl;  // W_M1^j (or W_M^j for one pass), W_M2^j, W_M^b (b < M2)
  void* S;             // intermediate, per pair M2 s1
  void* B;             // between the FFTs, per pair M
  int pair0;           // first column pair of this round
  int npairs;          // column pairs in this round
  int plain;           // set-up only: FFT of B into B (no chirp, table or DST stores)
};

// Element j of a = z c (zero past L) for the pair (xa, xb).
template <typename T>
__device__ __forceinline__ cx<T> bs_input(const double* xa, const double* xb, int64_t N, const cx<T>* chirp, int64_t j) {
  if (j >= 2 * N) return {T(0), T(0)};
  return cmul(load_z<T>(xa, xb, N, j), chirp[j]);
}

// Output k of the pair: Z_k = c_k conj(v)/M.
template <typename T>
__device__ __forceinline__ void bs_output(const BsArgs& a, int ca, int cb, int ncols, int64_t k, cx<T> v, T invM,
                                          double sa, double sb) {
  if (k < 1 || k >= a.N) return;
  const cx<T> c = reinterpret_cast<const cx<T>*>(a.chirp)[k];
  const cx<T> vc{v.x * invM, -v.y * invM};
  put_pair<T>(a.d, ca, cb, ncols, k, cmul(c, vc), sa, sb);
}

template <typename T, int LOGM>
__global__ __launch_bounds__(512) void k_dst_bs_single(BsArgs a) {
  constexpr int M = 1 << LOGM, E = 16, TP = M / E;
  constexpr int SEQS = single_seqs(LOGM), SEQ = seq_len(M);
  __shared__ cx<T> lds[SEQS * SEQ];
  const double* X;
  int ncols;
  if (!dst_resolve(a.d, X, ncols)) return;
  const int tt = threadIdx.x % TP, sl = threadIdx.x / TP;
  const int lp = blockIdx.x * SEQS + sl;  // pair within this round (the last block may run past)
  const bool mine = lp < a.npairs;
  const int pair = a.pair0 + lp;
  const int ca = 2 * pair, cb = ca + 1;
  const double* xa = mine && ca < ncols ? X + (int64_t)ca * a.d.ldx : nullptr;
  const double* xb = mine && cb < ncols ? X + (int64_t)cb * a.d.ldx : nullptr;
  const cx<T>* chirp = reinterpret_cast<const cx<T>*>(a.chirp);
  const cx<T>* bhat = reinterpret_cast<const cx<T>*>(a.bhat);
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.t1);
  cx<T> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) x[e] = bs_input<T>(xa, xb, a.N, chirp, tt + TP * e);
  fft_seq<T, LOGM, E>(x, lds + sl * SEQ, tt, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const cx<T> v = cmul(x[e], bhat[tt + TP * e]);
    x[e] = {v.x, -v.y};
  }
  fft_seq<T, LOGM, E>(x, lds + sl * SEQ, tt, tw);
  if (!mine || ca >= a.d.ncols_out) return;
  double sa, sb;
  col_scales(a.d, ca, cb, ncols, sa, sb);
  const T invM = T(1.0 / (double)M);
#pragma unroll
  for (int e = 0; e < E; ++e) bs_output<T>(a, ca, cb, ncols, tt + TP * e, x[e], invM, sa, sb);
}

// Pass 1: TJ consecutive j1 (lane-fastest, contiguous reads) x M2/16 threads; the transform over
// j2, the twiddle W_M^{j1 k2}, the intermediate S[k2][j1]. FROM_X: the input is a = z c from the
// columns; otherwise the buffer B.
template <typename T, int LOG2, bool FROM_X>
__global__ __launch_bounds__(512) void k_dst_bs_pass1(BsArgs a) {
  constexpr int M2 = 1 << LOG2, E = 16, TP = M2 / E;
  constexpr int TJ = tile1_of<T>(LOG2), SEQ = seq_len(M2);
  __shared__ cx<T> lds[TJ * SEQ];
  const double* X = nullptr;
  int ncols = 0;
  if (!a.plain && !dst_resolve(a.d, X, ncols)) return;
  const int M1 = 1 << a.logM1;
  const int64_t M = (int64_t)M1 * M2;
  const int ntiles = M1 / TJ;
  const int tile = blockIdx.x % ntiles;
  const int pair = a.pair0 + blockIdx.x / ntiles;
  const int ca = 2 * pair, cb = ca + 1;
  if (!a.plain && ca >= ncols) return;  // a zero pair: the last pass writes its zeros
  const int cl = threadIdx.x % TJ, tt = threadIdx.x / TJ;
  const int j1 = tile * TJ + cl;
  cx<T> x[E];
  if (FROM_X) {
    const double* xa = X + (int64_t)ca * a.d.ldx;
    const double* xb = cb < ncols ? X + (int64_t)cb * a.d.ldx : nullptr;
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(a.chirp);
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = bs_input<T>(xa, xb, a.N, chirp, j1 + (int64_t)M1 * (tt + TP * e));
  } else {
    const cx<T>* Bp = reinterpret_cast<const cx<T>*>(a.B) + (int64_t)(pair - a.pair0) * M;
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = Bp[j1 + (int64_t)M1 * (tt + TP * e)];
  }
  fft_seq<T, LOG2, E>(x, lds + cl * SEQ, tt, reinterpret_cast<const cx<T>*>(a.t2));
  const cx<T>* thi = reinterpret_cast<const cx<T>*>(a.t1);  // W_M^{M2 h} = W_M1^h
  const cx<T>* tlo = reinterpret_cast<const cx<T>*>(a.tl);  // W_M^b, b < M2
  cx<T>* S = reinterpret_cast<cx<T>*>(a.S) + (int64_t)(pair - a.pair0) * M2 * a.s1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k2 = tt + TP * e;
    const int64_t m = (int64_t)j1 * k2;
    S[(int64_t)k2 * a.s1 + j1] = cmul(x[e], cmul(thi[m >> LOG2], tlo[m & (M2 - 1)]));
  }
}

// Pass 2: TK consecutive k2 x M1/16 threads (lane-fastest along the sequence, contiguous reads of
// S); outputs staged in LDS so that each row k1 goes out as TK consecutive k2. TO_DST: the DST
// outputs; otherwise conj(X_k bhat_k) into B (plain: X_k itself).
template <typename T, int LOG1, bool TO_DST>
__global__ __launch_bounds__(512) void k_dst_bs_pass2(BsArgs a) {
  constexpr int M1 = 1 << LOG1, E = 16, TP = M1 / E;
  constexpr int TK = tile2_of<T>(LOG1), SEQ = seq_len(M1);
  constexpr int OST = TK + 1;
  constexpr int NLDS = TK * SEQ > M1 * OST ? TK * SEQ : M1 * OST;
  __shared__ cx<T> lds[NLDS];
  const double* X = nullptr;
  int ncols = 0;
  if (!a.plain && !dst_resolve(a.d, X, ncols)) return;
  const int64_t M2 = int64_t(1) << (a.d.logL2);  // M2 travels in d.logL2
  const int64_t M = M1 * M2;
  const int ntiles = (int)(M2 / TK);
  const int tile = blockIdx.x % ntiles;
  const int pair = a.pair0 + blockIdx.x / ntiles;
  const int ca = 2 * pair, cb = ca + 1;
  if (TO_DST && ca >= a.d.ncols_out) return;
  const int k0 = tile * TK;
  const int nthreads = TK * TP;
  const bool zero = !a.plain && ca >= ncols;
  if (!TO_DST && zero) return;
  const int tt = threadIdx.x % TP, kl = threadIdx.x / TP;
  if (!zero) {
    const cx<T>* S = reinterpret_cast<const cx<T>*>(a.S) + (int64_t)(pair - a.pair0) * M2 * a.s1;
    cx<T> x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = S[(int64_t)(k0 + kl) * a.s1 + tt + TP * e];
    fft_seq<T, LOG1, E>(x, lds + kl * SEQ, tt, reinterpret_cast<const cx<T>*>(a.t1));
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) lds[(tt + TP * e) * OST + kl] = x[e];  // row k1, column k2 - k0
    __syncthreads();
  }
  if (TO_DST) {
    double sa, sb;
    col_scales(a.d, ca, cb, ncols, sa, sb);
    const T invM = T(1.0 / (double)M);
    for (int g = threadIdx.x; g < M1 * TK; g += nthreads) {
      const int c = g % TK, k1 = g / TK;
      const int64_t k = k0 + c + M2 * k1;
      if (k < 1 || k >= a.N) continue;
      if (zero)
        put_pair<T>(a.d, ca, cb, ncols, k, cx<T>{T(0), T(0)}, sa, sb);
      else
        bs_output<T>(a, ca, cb, ncols, k, lds[k1 * OST + c], invM, sa, sb);
    }
  } else {
    const cx<T>* bhat = reinterpret_cast<const cx<T>*>(a.bhat);
    cx<T>* Bp = reinterpret_cast<cx<T>*>(a.B) + (int64_t)(pair - a.pair0) * M;
    for (int g = threadIdx.x; g < M1 * TK; g += nthreads) {
      const int c = g % TK, k1 = g / TK;
      const int64_t k = k0 + c + M2 * k1;
      cx<T> v = lds[k1 * OST + c];
      if (!a.plain) {
        v = cmul(v, bhat[k]);
        v.y = -v.y;
      }
      Bp[k] = v;
    }
  }
}

// Set-up for M <= 4096: the forward FFT of one FP64 sequence B in place.
template <int LOGM>
__global__ __launch_bounds__(256) void k_fft_plain_single(double2* B, const double2* tw) {
  constexpr int M = 1 << LOGM, E = 16, TP = M / E;
  __shared__ cx<double> lds[seq_len(M)];
  const int tt = threadIdx.x;
  cx<double>* Bc = reinterpret_cast<cx<double>*>(B);
  cx<double> x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) x[e] = Bc[tt + TP * e];
  fft_seq<double, LOGM, E>(x, lds, tt, reinterpret_cast<const cx<double>*>(tw));
#pragma unroll
  for (int e = 0; e < E; ++e) Bc[tt + TP * e] = x[e];
}

// Set-up: the circular chirp b (M entries, conj(c_|m|) for |m| < L, 0 between) into B, FP64.
__global__ void k_bs_bvec(double2* B, const double2* chirp, int64_t L, int64_t M) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double2 v = make_double2(0.0, 0.0);
  if (m < L) v = make_double2(chirp[m].x, -chirp[m].y);
  else if (M - m < L) v = make_double2(chirp[M - m].x, -chirp[M - m].y);
  B[m] = v;
}

__global__ void k_bs_chirp(double2* c64, float2* c32, int64_t L) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  const int64_t q = (j * j) % (2 * L);  // j < 2^23, so j^2 fits in 64 bits
  double s, c;
  sincospi((double)q / (double)L, &s, &c);
  c64[j] = make_double2(c, -s);
  c32[j] = make_float2((float)c, (float)-s);
}

__global__ void k_copy_c64_c32(const double2* a, double2* b64, float2* b32, int64_t M) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  b64[j] = a[j];
  b32[j] = make_float2((float)a[j].x, (float)a[j].y);
}

// ----------------------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------------------
static int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

// Intermediate bytes of one pass-1/pass-2 round of the four-step DST (the memory-side cache
// holds 256 MB; the round's input and output stream through it as well).
constexpr int64_t kDstBatchBytes = int64_t(96) << 20;

int dst_plan(DstPlan* p, int64_t n, int max_cols) {
  const int64_t M = n + 1;
  *p = DstPlan{};
  p->n = n;
  p->max_pairs = (max_cols + 1) / 2;
  if ((M & (M - 1)) != 0) {  // Bluestein
    const int logM = ilog2(4 * M - 1);
    if (M < 3 || logM > 24) return LRP_EINVAL;
    p->bluestein = 1;
    p->logM = logM;
    p->logL = logM;
    p->four_step = logM > 12;
    p->logL2 = p->four_step ? logM / 2 : 0;
    p->logL1 = logM - p->logL2;
    const int64_t L1 = int64_t(1) << p->logL1, L2 = int64_t(1) << p->logL2;
    p->t1_count = (int)L1;
    p->t2_count = p->four_step ? (int)L2 : 0;
    p->s1 = p->four_step ? L1 + 16 : 0;
    p->batch_pairs = std::min(p->max_pairs, 8);
    p->work_bytes = p->four_step ? (int64_t)p->batch_pairs * L2 * p->s1 * 16 : 0;
    return LRP_OK;
  }
  const int logL = ilog2(2 * M);
  if (logL < 3 || logL > 24) return LRP_EINVAL;
  p->logL = logL;
  if (logL <= 12) {
    p->four_step = 0;
    p->logL1 = logL;
    p->logL2 = 0;
  } else {
    p->four_step = 1;
    p->logL2 = logL / 2;
    p->logL1 = logL - p->logL2;
  }
  const int L1 = 1 << p->logL1, L2 = 1 << p->logL2;
  p->t1_count = L1;
  p->t2_count = p->four_step ? L2 : 0;
  p->s1 = p->four_step ? L1 / 2 + 16 : 0;
  // column pairs per pass-1/pass-2 round: their intermediate (up to kDstBatchBytes) is written
  // by pass 1 and read back by pass 2 at once, so it can stay in the memory-side cache (MALL)
  const int64_t per_pair = p->four_step ? (int64_t)L2 * p->s1 * 16 : 0;
  p->batch_pairs = p->four_step ? (int)std::max<int64_t>(1, std::min<int64_t>(p->max_pairs, kDstBatchBytes / per_pair))
                                : p->max_pairs;
  p->work_bytes = (int64_t)p->batch_pairs * per_pair;
  return LRP_OK;
}

int64_t dst_bytes(const DstPlan& p) {
  int64_t b = 24 * (int64_t)(p.t1_count + 2 * std::max(p.t2_count, 1)) + p.work_bytes;
  if (p.bluestein) {
    const int64_t M = int64_t(1) << p.logM, L = 2 * (p.n + 1);
    b += 24 * (L + M) + (int64_t)p.batch_pairs * M * 16;
  }
  return b;
}

template <typename T>
static int dalloc_n(T** q, int64_t count) {
  *q = nullptr;
  return hipMalloc((void**)q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) == hipSuccess ? LRP_OK : LRP_ENOMEM;
}

int dst_alloc(DstPlan* p) {
  const int c1 = p->t1_count, c2 = std::max(p->t2_count, 1);
  if (dalloc_n(&p->t1_64, c1) || dalloc_n(&p->t1_32, c1) || dalloc_n(&p->t2_64, c2) || dalloc_n(&p->t2_32, c2) ||
      dalloc_n(&p->tl_64, c2) || dalloc_n(&p->tl_32, c2))
    return LRP_ENOMEM;
  if (p->four_step && hipMalloc(&p->work, (size_t)p->work_bytes) != hipSuccess) return LRP_ENOMEM;
  if (p->bluestein) {
    const int64_t M = int64_t(1) << p->logM, L = 2 * (p->n + 1);
    if (dalloc_n(&p->chirp_64, L) || dalloc_n(&p->chirp_32, L) || dalloc_n(&p->bhat_64, M) ||
        dalloc_n(&p->bhat_32, M))
      return LRP_ENOMEM;
    if (hipMalloc(&p->work2, (size_t)p->batch_pairs * M * 16) != hipSuccess) return LRP_ENOMEM;
  }
  return LRP_OK;
}

void dst_free(DstPlan* p) {
  void* bufs[] = {p->t1_64, p->t2_64, p->tl_64, p->t1_32, p->t2_32, p->tl_32, p->work,
                  p->chirp_64, p->chirp_32, p->bhat_64, p->bhat_32, p->work2};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  p->t1_64 = p->t2_64 = p->tl_64 = p->chirp_64 = p->bhat_64 = nullptr;
  p->t1_32 = p->t2_32 = p->tl_32 = p->chirp_32 = p->bhat_32 = nullptr;
  p->work = p->work2 = nullptr;
}

template <typename T>
static int bs_launch(const DstPlan& p, BsArgs b, hipStream_t s);

int dst_tables(DstPlan* p, hipStream_t s) {
  if (p->bluestein) {
    const int64_t L1 = int64_t(1) << p->logL1, L2 = int64_t(1) << p->logL2;
    const int64_t M = int64_t(1) << p->logM, L = 2 * (p->n + 1);
    // W_M1^k (W_M^k for one pass), W_M2^k, W_M^b (b < M2)
    hipLaunchKernelGGL(k_twiddle, dim3((unsigned)((L1 + 255) / 256)), dim3(256), 0, s, p->t1_64, p->t1_32, (int)L1,
                       (int)L1);
    if (p->four_step) {
      hipLaunchKernelGGL(k_twiddle, dim3((unsigned)((L2 + 255) / 256)), dim3(256), 0, s, p->t2_64, p->t2_32, (int)L2,
                         (int)L2);
      hipLaunchKernelGGL(k_twiddle, dim3((unsigned)((L2 + 255) / 256)), dim3(256), 0, s, p->tl_64, p->tl_32, (int)M,
                         (int)L2);
    }
    hipLaunchKernelGGL(k_bs_chirp, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, p->chirp_64, p->chirp_32, L);
    // bhat = DFT_M(b), FP64: b into the first pair's slot of work2, transformed in place
    double2* B = static_cast<double2*>(p->work2);
    hipLaunchKernelGGL(k_bs_bvec, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, B, p->chirp_64, L, M);
    BsArgs b{};
    b.plain = 1;
    b.N = p->n + 1;
    b.B = B;
    b.npairs = 1;
    TRY_DST(bs_launch<double>(*p, b, s));
    hipLaunchKernelGGL(k_copy_c64_c32, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, B, p->bhat_64,
                       p->bhat_32, M);
    return launch_status();
  }
  const int L1 = 1 << p->logL1, L2 = 1 << p->logL2;
  const int L = 1 << p->logL;
  // t1: W_{L1}^k, k < L1 ; t2: W_{L2}^k, k < L2 ; tl: W_L^b, b < L2
  hipLaunchKernelGGL(k_twiddle, dim3((L1 + 255) / 256), dim3(256), 0, s, p->t1_64, p->t1_32, L1, L1);
  if (p->four_step) {
    hipLaunchKernelGGL(k_twiddle, dim3((L2 + 255) / 256), dim3(256), 0, s, p->t2_64, p->t2_32, L2, L2);
    hipLaunchKernelGGL(k_twiddle, dim3((L2 + 255) / 256), dim3(256), 0, s, p->tl_64, p->tl_32, L, L2);
  }
  return launch_status();
}

template <typename T>
static void launch_single(int logL, int npairs, const DstArgs& a, hipStream_t s) {
#define LRP_SINGLE(LG)                                                                      \
  case LG: {                                                                                \
    constexpr int seqs = single_seqs(LG), tp = (1 << LG) < 16 ? 1 : (1 << LG) / 16;        \
    LRP_LAUNCH(K_DST_SINGLE, (k_dst_single<T, LG>), dim3((npairs + seqs - 1) / seqs), dim3(seqs * tp), 0, s, a); \
    break;                                                                                  \
  }
  switch (logL) {
    LRP_SINGLE(3) LRP_SINGLE(4) LRP_SINGLE(5) LRP_SINGLE(6) LRP_SINGLE(7)
    LRP_SINGLE(8) LRP_SINGLE(9) LRP_SINGLE(10) LRP_SINGLE(11) LRP_SINGLE(12)
    default: break;
  }
#undef LRP_SINGLE
}

// A pass launch of fewer workgroups than this runs the narrow-tile build.
constexpr int kDstMinBlocks = 2 * 256;

template <typename T>
static void launch_four_step(int logL1, int logL2, int npairs, const DstArgs& a, hipStream_t s) {
  const int L1 = 1 << logL1, L2 = 1 << logL2;
#define LRP_P1(LG)                                                                                    \
  case LG: {                                                                                          \
    constexpr int tj = tile1_of<T>(LG), tn = tile1_of<T, kNarrow1>(LG);                               \
    if ((L1 / 2 / tj + 1) * npairs < kDstMinBlocks && tn < tj)                                        \
      LRP_LAUNCH(K_DST_PASS1, (k_dst_pass1<T, LG, kNarrow1>), dim3((L1 / 2 / tn + 1) * npairs),         \
                 dim3(tn * ((1 << LG) / 16)), 0, s, a);                                               \
    else                                                                                              \
      LRP_LAUNCH(K_DST_PASS1, (k_dst_pass1<T, LG>), dim3((L1 / 2 / tj + 1) * npairs),                   \
                 dim3(tj * ((1 << LG) / 16)), 0, s, a);                                               \
    break;                                                                                            \
  }
#define LRP_P2(LG)                                                                                    \
  case LG: {                                                                                          \
    constexpr int tk = tile2_of<T>(LG), tn = tile2_of<T, kNarrow2>(LG);                               \
    if ((L2 / 2 / tk + 1) * npairs < kDstMinBlocks && tn < tk)                                        \
      LRP_LAUNCH(K_DST_PASS2, (k_dst_pass2<T, LG, kNarrow2>), dim3((L2 / 2 / tn + 1) * npairs),         \
                 dim3(tn * ((1 << LG) / 16)), 0, s, a);                                               \
    else                                                                                              \
      LRP_LAUNCH(K_DST_PASS2, (k_dst_pass2<T, LG>), dim3((L2 / 2 / tk + 1) * npairs),                   \
                 dim3(tk * ((1 << LG) / 16)), 0, s, a);                                               \
    break;                                                                                            \
  }
  switch (logL2) {
    LRP_P1(6) LRP_P1(7) LRP_P1(8) LRP_P1(9) LRP_P1(10) LRP_P1(11) LRP_P1(12)
    default: break;
  }
  switch (logL1) {
    LRP_P2(7) LRP_P2(8) LRP_P2(9) LRP_P2(10) LRP_P2(11) LRP_P2(12)
    default: break;
  }
#undef LRP_P1
#undef LRP_P2
}

template <typename T, bool FROM_X>
static int bs_pass1(int logL2, int M1, int np, const BsArgs& b, hipStream_t s) {
#define LRP_BSP1(LG)                                                                                \
  case LG: {                                                                                        \
    constexpr int tj = tile1_of<T>(LG);                                                             \
    LRP_LAUNCH(K_DST_PASS1, (k_dst_bs_pass1<T, LG, FROM_X>), dim3((M1 / tj) * np),                 \
               dim3(tj * ((1 << LG) / 16)), 0, s, b);                                              \
    return launch_status();                                                                         \
  }
  switch (logL2) {
    LRP_BSP1(6) LRP_BSP1(7) LRP_BSP1(8) LRP_BSP1(9) LRP_BSP1(10) LRP_BSP1(11) LRP_BSP1(12)
    default: return LRP_EINVAL;
  }
#undef LRP_BSP1
}

template <typename T, bool TO_DST>
static int bs_pass2(int logL1, int M2, int np, const BsArgs& b, hipStream_t s) {
#define LRP_BSP2(LG)                                                                                \
  case LG: {                                                                                        \
    constexpr int tk = tile2_of<T>(LG);                                                             \
    LRP_LAUNCH(K_DST_PASS2, (k_dst_bs_pass2<T, LG, TO_DST>), dim3((M2 / tk) * np),                 \
               dim3(tk * ((1 << LG) / 16)), 0, s, b);                                              \
    return launch_status();                                                                         \
  }
  switch (logL1) {
    LRP_BSP2(7) LRP_BSP2(8) LRP_BSP2(9) LRP_BSP2(10) LRP_BSP2(11) LRP_BSP2(12)
    default: return LRP_EINVAL;
  }
#undef LRP_BSP2
}

// The Bluestein transform of b.npairs pairs from b.pair0; plain (set-up): the forward FFT of
// b.B (one FP64 sequence) in place.
template <typename T>
static int bs_launch(const DstPlan& p, BsArgs b, hipStream_t s) {
  const bool f32 = std::is_same<T, float>::value;
  b.t1 = f32 ? (const void*)p.t1_32 : (const void*)p.t1_64;
  b.t2 = f32 ? (const void*)p.t2_32 : (const void*)p.t2_64;
  b.tl = f32 ? (const void*)p.tl_32 : (const void*)p.tl_64;
  b.chirp = f32 ? (const void*)p.chirp_32 : (const void*)p.chirp_64;
  b.bhat = f32 ? (const void*)p.bhat_32 : (const void*)p.bhat_64;
  b.S = p.work;
  b.s1 = p.s1;
  b.logM1 = p.logL1;
  b.d.logL2 = p.logL2;
  const int np = b.npairs;
  if (!p.four_step) {
    if (b.plain) {
#define LRP_FPS(LG)                                                                                  \
  case LG:                                                                                           \
    hipLaunchKernelGGL((k_fft_plain_single<LG>), dim3(1), dim3((1 << LG) / 16), 0, s,               \
                       static_cast<double2*>(b.B), p.t1_64);                                         \
    return launch_status();
      switch (p.logM) {
        LRP_FPS(4) LRP_FPS(5) LRP_FPS(6) LRP_FPS(7) LRP_FPS(8) LRP_FPS(9) LRP_FPS(10) LRP_FPS(11) LRP_FPS(12)
        default: return LRP_EINVAL;
      }
#undef LRP_FPS
    }
#define LRP_BS1(LG)                                                                                 \
  case LG: {                                                                                        \
    constexpr int seqs = single_seqs(LG);                                                           \
    LRP_LAUNCH(K_DST_SINGLE, (k_dst_bs_single<T, LG>), dim3((np + seqs - 1) / seqs),               \
               dim3(seqs * ((1 << LG) / 16)), 0, s, b);                                            \
    return launch_status();                                                                         \
  }
    switch (p.logM) {
      LRP_BS1(4) LRP_BS1(5) LRP_BS1(6) LRP_BS1(7) LRP_BS1(8) LRP_BS1(9) LRP_BS1(10) LRP_BS1(11) LRP_BS1(12)
      default: return LRP_EINVAL;
    }
#undef LRP_BS1
  }
  const int M1 = 1 << p.logL1, M2 = 1 << p.logL2;
  if (b.plain) {
    TRY_DST((bs_pass1<T, false>(p.logL2, M1, np, b, s)));
    return bs_pass2<T, false>(p.logL1, M2, np, b, s);
  }
  TRY_DST((bs_pass1<T, true>(p.logL2, M1, np, b, s)));    // DFT of a = z c
  TRY_DST((bs_pass2<T, false>(p.logL1, M2, np, b, s)));   // conj(. bhat) into B
  TRY_DST((bs_pass1<T, false>(p.logL2, M1, np, b, s)));   // DFT of B
  return bs_pass2<T, true>(p.logL1, M2, np, b, s);         // c_k conj(.)/M: the DST outputs
}

int dst_launch(const DstPlan& p, DstArgs a, bool fp32, hipStream_t s) {
  const int npairs = (a.ncols_out + 1) / 2;
  if (npairs <= 0) return LRP_OK;
  if (npairs > p.max_pairs) return LRP_EINVAL;
  if (p.bluestein) {
    a.outscale *= 1.0 / std::sqrt(2.0 * (double)(p.n + 1));
    BsArgs b{};
    b.d = a;
    b.N = p.n + 1;
    b.B = p.work2;
    for (int p0 = 0; p0 < npairs; p0 += p.batch_pairs) {
      b.pair0 = p0;
      b.npairs = std::min(p.batch_pairs, npairs - p0);
      const int rc = fp32 ? bs_launch<float>(p, b, s) : bs_launch<double>(p, b, s);
      if (rc != LRP_OK) return rc;
    }
    return LRP_OK;
  }
  a.logL = p.logL;
  a.logL1 = p.logL1;
  a.logL2 = p.logL2;
  a.s1 = p.s1;
  a.t1 = fp32 ? (const void*)p.t1_32 : (const void*)p.t1_64;
  a.t2 = fp32 ? (const void*)p.t2_32 : (const void*)p.t2_64;
  a.tl = fp32 ? (const void*)p.tl_32 : (const void*)p.tl_64;
  a.outscale *= 1.0 / std::sqrt(2.0 * (double)(p.n + 1));
  if (!p.four_step) {
    if (fp32)
      launch_single<float>(p.logL, npairs, a, s);
    else
      launch_single<double>(p.logL, npairs, a, s);
  } else {
    a.work = p.work;
    // FP32 intermediates take half the bytes, so twice the pairs fit the work buffer
    const int bp = fp32 ? std::min(p.max_pairs, 2 * p.batch_pairs) : p.batch_pairs;
    for (int p0 = 0; p0 < npairs; p0 += bp) {
      a.pair0 = p0;
      const int nb = std::min(bp, npairs - p0);
      if (fp32)
        launch_four_step<float>(p.logL1, p.logL2, nb, a, s);
      else
        launch_four_step<double>(p.logL1, p.logL2, nb, a, s);
    }
  }
  return launch_status();
}

}  // namespace lrp
