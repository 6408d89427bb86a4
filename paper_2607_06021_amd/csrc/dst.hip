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
#include "lrp_kernels.h"

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
// threads (16 elements each) and at most kLdsMax bytes of LDS.
constexpr int kLdsMax = 80 * 1024;  // two workgroups per CU
__host__ __device__ constexpr int lds_pass1(int log2, int tj, int esz) { return tj * seq_len(1 << log2) * esz; }
__host__ __device__ constexpr int lds_pass2(int log1, int tk, int esz) {
  return (tk * seq_len(1 << log1) > (1 << log1) * (tk + 1) ? tk * seq_len(1 << log1) : (1 << log1) * (tk + 1)) * esz;
}
__host__ __device__ constexpr int tile1_for(int log2, int esz, int cap) {
  int t = cap;
  while (t > 1 && (lds_pass1(log2, t, esz) > kLdsMax || t * ((1 << log2) / 16) > 512)) t >>= 1;
  return t;
}
__host__ __device__ constexpr int tile2_for(int log1, int esz, int cap) {
  int t = cap;
  while (t > 1 && (lds_pass2(log1, t, esz) > kLdsMax || t * ((1 << log1) / 16) > 512)) t >>= 1;
  return t;
}
template <typename T>
__host__ __device__ constexpr int tile1_of(int log2) { return tile1_for(log2, (int)sizeof(cx<T>), 32); }
template <typename T>
__host__ __device__ constexpr int tile2_of(int log1) { return tile2_for(log1, (int)sizeof(cx<T>), 16); }

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

// ---------------------------------------------------------------- four-step pass 1
// Block: TJ columns j1 (lane-fastest, so global reads and writes are coalesced) x L2/16 threads;
// TJ = 16 (FP64) or 32 (FP32) columns, so each row of the input is read in 128- or 256-byte pieces.
template <typename T, int LOG2>
__global__ __launch_bounds__(512) void k_dst_pass1(DstArgs a) {
  constexpr int L2 = 1 << LOG2, E = 16, TP = L2 / E;
  constexpr int TJ = tile1_of<T>(LOG2), SEQ = seq_len(L2);
  __shared__ cx<T> lds[TJ * SEQ];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int L1 = 1 << a.logL1;
  // blocks: the L1/(2 TJ) full column tiles of every pair first, then the tile holding the
  // single column j1 = L1/2 of every pair, so that the light tiles form the tail of the grid
  const int nfull = (L1 / 2) / TJ;
  const int npairs = gridDim.x / (nfull + 1);
  const int b = blockIdx.x;
  const int tile = b < nfull * npairs ? b % nfull : nfull;
  const int pair = b < nfull * npairs ? b / nfull : b - nfull * npairs;
  const int ca = 2 * pair, cb = ca + 1;
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
template <typename T, int LOG1>
__global__ __launch_bounds__(512) void k_dst_pass2(DstArgs a) {
  constexpr int L1 = 1 << LOG1, E = 16, TP = L1 / E;
  constexpr int TK = tile2_of<T>(LOG1), SEQ = seq_len(L1);
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
  const int b = blockIdx.x;
  const int tile = b < nfull * npairs ? b % nfull : nfull;
  const int pair = b < nfull * npairs ? b / nfull : b - nfull * npairs;
  const int ca = 2 * pair, cb = ca + 1;
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
// Host side
// ----------------------------------------------------------------------------------------
static int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

int dst_plan(DstPlan* p, int64_t n, int max_cols) {
  const int64_t M = n + 1;
  const int logL = ilog2(2 * M);
  if (logL < 3 || logL > 24) return LRP_EINVAL;
  p->n = n;
  p->logL = logL;
  p->max_pairs = (max_cols + 1) / 2;
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
  p->work_bytes = p->four_step ? (int64_t)p->max_pairs * L2 * p->s1 * 16 : 0;
  return LRP_OK;
}

int dst_tables(DstPlan* p, hipStream_t s) {
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

template <typename T>
static void launch_four_step(int logL1, int logL2, int npairs, const DstArgs& a, hipStream_t s) {
  const int L1 = 1 << logL1, L2 = 1 << logL2;
#define LRP_P1(LG)                                                                          \
  case LG: {                                                                                \
    constexpr int tj = tile1_of<T>(LG);                                                     \
    LRP_LAUNCH(K_DST_PASS1, (k_dst_pass1<T, LG>), dim3((L1 / 2 / tj + 1) * npairs),              \
                       dim3(tj * ((1 << LG) / 16)), 0, s, a);                               \
    break;                                                                                  \
  }
#define LRP_P2(LG)                                                                          \
  case LG: {                                                                                \
    constexpr int tk = tile2_of<T>(LG);                                                     \
    LRP_LAUNCH(K_DST_PASS2, (k_dst_pass2<T, LG>), dim3((L2 / 2 / tk + 1) * npairs),              \
                       dim3(tk * ((1 << LG) / 16)), 0, s, a);                               \
    break;                                                                                  \
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

int dst_launch(const DstPlan& p, DstArgs a, bool fp32, hipStream_t s) {
  const int npairs = (a.ncols_out + 1) / 2;
  if (npairs <= 0) return LRP_OK;
  if (npairs > p.max_pairs) return LRP_EINVAL;
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
    if (fp32)
      launch_four_step<float>(p.logL1, p.logL2, npairs, a, s);
    else
      launch_four_step<double>(p.logL1, p.logL2, npairs, a, s);
  }
  return launch_status();
}

}  // namespace lrp
