// Stopping test of Algorithm 4 (paper): rho = ||U_k S_k V_k^T - U' S' V'^T||_F / ||S_k||_F,
// with (U', S', V') the previous iterate, and the decision max(rho, indicator) < eps.
//
// rho is formed without cancellation (never as ||A||^2 + ||B||^2 - 2 <A, B>): with
// M_u = U_k^T U', Y = U' - U_k M_u, N_v = V_k^T V', Y' = V' - V_k N_v formed explicitly,
//   X_k - X_{k-1} = U_k (S_k - M_u S' N_v^T) V_k^T - U_k M_u S' Y'^T - Y S' N_v^T V_k^T - Y S' Y'^T,
// four mutually orthogonal terms, so rho^2 ||S_k||^2 is the sum of
//   ||S_k - M_u S' N_v^T||^2, tr(M_u S' G' S' M_u^T), tr(N_v S' G S' N_v^T), tr(S' G S' G'),
// with G = Y^T Y and G' = Y'^T Y' Gram matrices of explicitly formed small numbers.
// rho is only needed when the core's cheap bound on the indicator allows a stop (the decision
// needs both), so the n-length kernels return at once otherwise; the indicator itself and the
// decision follow in k_eta. All reductions have a fixed order.
#include "lrp_kernels.h"

namespace lrp {

constexpr int kRhoChunk = 64;   // rows per staged chunk (pass A)
constexpr int kRhoChunkB = 32;  // (pass B)

struct RhoKArgs {
  DevState* st;
  const double* A[2];  // U_k / V_k
  const double* B[2];  // U' / V'
  int64_t ldu;
  int64_t n;
  int rows_per_block;
  int nb_new, nb_old;
  const double* M;     // M_u, N_v (for the second pass)
  double* part;
};

// st->k is the index of the pass being computed (the decision kernel advances it).
__device__ inline bool rho_needed(const DevState* st) {
  return !st->done && st->k >= 1 && st->eta_need;
}

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kRS = kPMax + 1;  // row stride of the LDS chunks

constexpr int kRhoThreads = 256;

// Stage rows [r0, r0 + 64) of the first ca columns of XA into SA and of the first cb columns of
// XB into SB (row-major, stride 65), zero beyond the columns and beyond n. Every load reads a
// valid element (clamped row and column); all 32 loads of a thread are issued before any is
// used, so they are in flight together.
template <int CH = kRhoChunk>
__device__ inline void stage2(double* SA, const double* XA, int ca, double* SB, const double* XB, int cb,
                              int64_t ldu, int64_t n, int64_t r0) {
  constexpr int kPer = CH * kPMax / kRhoThreads;  // 16 for 64-row chunks
  double va[kPer], vb[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int e = threadIdx.x + kRhoThreads * m, row = e % CH, c = e / CH;
    const int64_t i = min(r0 + row, n - 1);
    va[m] = XA[i + (int64_t)min(c, max(ca - 1, 0)) * ldu];
    vb[m] = XB[i + (int64_t)min(c, max(cb - 1, 0)) * ldu];
  }
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int e = threadIdx.x + kRhoThreads * m, row = e % CH, c = e / CH;
    const bool rok = r0 + row < n;
    asm volatile("" : "+v"(va[m]));
    asm volatile("" : "+v"(vb[m]));
    SA[row * kRS + c] = (c < ca && rok) ? va[m] : 0.0;
    SB[row * kRS + c] = (c < cb && rok) ? vb[m] : 0.0;
  }
}

// acc[nt] += X^T Y over the 64 rows of a chunk for output rows 16 w .. 16 w + 15 and all 64
// output columns (FP64 MFMA 16x16x4; the chunk rows are the contraction index).
// A operand: X^T(16 w + l%16, k0 + l/16) = X[k0 + l/16][16 w + l%16]; B operand:
// Y[k0 + l/16][16 nt + l%16]; result item v of lane l: row 16 w + l/16 + 4 v, column 16 nt + l%16.
// Only the NT live output column tiles run (Y is zero beyond them); a wave whose output rows
// are all beyond X's live columns skips the chunk (its output stays zero).
template <int NT, int CH = kRhoChunk>
__device__ inline void gram_chunk(const double* X, const double* Y, int w, int lr, int lk, d4 (&acc)[4]) {
#pragma unroll
  for (int ks = 0; ks < CH / 4; ++ks) {
    const int row = 4 * ks + lk;
    const double xa = X[row * kRS + 16 * w + lr];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, Y[row * kRS + 16 * nt + lr], acc[nt], 0, 0, 0);
  }
}

__device__ inline void store_partial(double* out, int w, int lr, int lk, const d4 (&acc)[4]) {
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(16 * w + lk + 4 * v) * kPMax + 16 * nt + lr] = acc[nt][v];
}

// Pass A: partial M = A^T B over the block's rows (output tiles: NT = ceil(ro/16) columns,
// rows below r).
template <int NT>
__device__ __forceinline__ void rho_a_body(const RhoKArgs& a, int side, int r, int ro, double* As, double* Bs) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  d4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t rend = min(a.n, row0 + a.rows_per_block);
  for (int64_t r0 = row0; r0 < rend; r0 += kRhoChunk) {
    stage2(As, a.A[side], r, Bs, a.B[side], ro, a.ldu, rend, r0);
    __syncthreads();
    if (16 * w < r) gram_chunk<NT>(As, Bs, w, lr, lk, acc);  // uniform per wave
    __syncthreads();
  }
  store_partial(a.part + ((int64_t)blockIdx.x * 2 + side) * kPMax * kPMax, w, lr, lk, acc);
}

template <class Src>
__global__ __launch_bounds__(kRhoThreads) void k_rho_a(Src in) {
  const RhoKArgs& a = kernel_args<RhoKArgs>(in);
  DevState* st = a.st;
  if (!rho_needed(st)) return;
  const int side = blockIdx.y;
  const int r = st->r[a.nb_new], ro = st->r[a.nb_old];
  __shared__ double As[kRhoChunk * kRS], Bs[kRhoChunk * kRS];
  switch ((ro + 15) >> 4) {  // uniform
    case 0:
    case 1: rho_a_body<1>(a, side, r, ro, As, Bs); break;
    case 2: rho_a_body<2>(a, side, r, ro, As, Bs); break;
    case 3: rho_a_body<3>(a, side, r, ro, As, Bs); break;
    default: rho_a_body<4>(a, side, r, ro, As, Bs); break;
  }
}

// Pass B: Y = B - A M (rows of the chunk, MFMA with M as the second operand), then partial
// G = Y^T Y. Live tiles only: KS 4-column steps of A (r rounded up to 16), NT output column
// tiles (ceil(ro/16)); the waves whose G rows lie beyond ro skip the Gram product. Chunks of 32
// rows keep the LDS at 66 KB, so that two workgroups share a CU; the T product's tiles (2 row
// tiles x NT column tiles) are spread over the four waves. Every element is summed in the same
// order as with 64-row chunks.
template <int KS, int NT>
__device__ __forceinline__ void rho_b_body(const RhoKArgs& a, int side, int r, int ro, double* As, double* Bs,
                                           double* Ms) {
  constexpr int CH = kRhoChunkB;
  const double* Mg = a.M + (int64_t)side * kPMax * kPMax;
  for (int e = threadIdx.x; e < kPMax * kPMax; e += blockDim.x) Ms[(e / kPMax) * kRS + e % kPMax] = Mg[e];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  const int rt = w & 1, nt0 = w >> 1;  // T tiles of this wave: row tile rt, column tiles nt0, nt0 + 2
  d4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t rend = min(a.n, row0 + a.rows_per_block);
  for (int64_t r0 = row0; r0 < rend; r0 += CH) {
    stage2<CH>(As, a.A[side], r, Bs, a.B[side], ro, a.ldu, rend, r0);
    __syncthreads();
    // T = A M for chunk rows 16 rt .. 16 rt + 15, column tiles nt0 + 2 j: A operand
    // A[16 rt + l%16][k0 + l/16], B operand M[k0 + l/16][16 nt + l%16]; result item v: row
    // 16 rt + l/16 + 4 v, column 16 nt + l%16
    d4 tm[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) tm[j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const double xa = As[(16 * rt + lr) * kRS + 4 * ks + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int nt = nt0 + 2 * j;
        if (nt < NT)  // uniform per wave
          tm[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, Ms[(4 * ks + lk) * kRS + 16 * nt + lr], tm[j], 0, 0, 0);
      }
    }
    // Y = B - T in place of B (each element is read and written by its own lane)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int nt = nt0 + 2 * j;
      if (nt < NT) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* y = &Bs[(16 * rt + lk + 4 * v) * kRS + 16 * nt + lr];
          *y = *y - tm[j][v];
        }
      }
    }
    __syncthreads();
    if (16 * w < ro) gram_chunk<NT, CH>(Bs, Bs, w, lr, lk, acc);  // uniform per wave
    __syncthreads();
  }
  store_partial(a.part + ((int64_t)blockIdx.x * 2 + side) * kPMax * kPMax, w, lr, lk, acc);
}

template <int KS>
__device__ __forceinline__ void rho_b_nt(const RhoKArgs& a, int side, int r, int ro, double* As, double* Bs,
                                         double* Ms) {
  switch ((ro + 15) >> 4) {  // uniform
    case 0:
    case 1: rho_b_body<KS, 1>(a, side, r, ro, As, Bs, Ms); break;
    case 2: rho_b_body<KS, 2>(a, side, r, ro, As, Bs, Ms); break;
    case 3: rho_b_body<KS, 3>(a, side, r, ro, As, Bs, Ms); break;
    default: rho_b_body<KS, 4>(a, side, r, ro, As, Bs, Ms); break;
  }
}

template <class Src>
__global__ __launch_bounds__(kRhoThreads) void k_rho_b(Src in) {
  const RhoKArgs& a = kernel_args<RhoKArgs>(in);
  DevState* st = a.st;
  if (!rho_needed(st)) return;
  const int side = blockIdx.y;
  const int r = st->r[a.nb_new], ro = st->r[a.nb_old];
  __shared__ double As[kRhoChunkB * kRS], Bs[kRhoChunkB * kRS];
  __shared__ double Ms[kPMax * kRS];
  switch ((r + 15) >> 4) {  // uniform: 4-column steps of A in groups of four
    case 0:
    case 1: rho_b_nt<4>(a, side, r, ro, As, Bs, Ms); break;
    case 2: rho_b_nt<8>(a, side, r, ro, As, Bs, Ms); break;
    case 3: rho_b_nt<12>(a, side, r, ro, As, Bs, Ms); break;
    default: rho_b_nt<16>(a, side, r, ro, As, Bs, Ms); break;
  }
}

// Sum the per-block partials in block order: out[side][e] = sum_b part[b][side][e]. Only the
// live rows x cols block is read (rows: r_new for M, r_old for G; cols: r_old); every partial
// outside it is an exact zero, and so is the sum written there.
struct RhoReduceArgs {
  const DevState* st;
  const double* part;  // nblocks x 2 x kPMax x kPMax
  int nblocks;
  double* out;         // 2 x kPMax x kPMax
  int nb_rows, nb_cols;
};

template <class Src>
__global__ __launch_bounds__(256) void k_rho_reduce(Src in) {
  const RhoReduceArgs& a = kernel_args<RhoReduceArgs>(in);
  const DevState* st = a.st;
  const double* part = a.part;
  const int nblocks = a.nblocks;
  double* out = a.out;
  const int nb_rows = a.nb_rows, nb_cols = a.nb_cols;
  if (!rho_needed(st)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // 0 .. 2*4096
  if (e >= 2 * kPMax * kPMax) return;
  const int side = e / (kPMax * kPMax), q = e % (kPMax * kPMax);
  if (q / kPMax >= st->r[nb_rows] || q % kPMax >= st->r[nb_cols]) {
    out[e] = 0.0;
    return;
  }
  // 16 loads in flight per step, added into four partial sums in a fixed order
  double sm[4] = {0.0, 0.0, 0.0, 0.0};
  const double* src = part + (int64_t)side * kPMax * kPMax + q;
  const int64_t stride = 2 * kPMax * kPMax;
  int b = 0;
  for (; b + 15 < nblocks; b += 16) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = src[(int64_t)(b + k) * stride];
#pragma unroll
    for (int k = 0; k < 16; ++k) sm[k & 3] += v[k];
  }
  for (; b < nblocks; ++b) sm[0] += src[(int64_t)b * stride];
  out[e] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

struct RhoFinalArgs {
  DevState* st;
  const double* M;  // M_u, N_v   (row a: new column, col m: old column)
  const double* G;  // G_u = Y^T Y, G_v = Y'^T Y'
  int nb_new, nb_old;
  int maxiter;
  TraceBuf trace;
};

template <class Src>
__global__ __launch_bounds__(256) void k_rho_final(Src in) {
  const RhoFinalArgs& a = kernel_args<RhoFinalArgs>(in);
  DevState* st = a.st;
  if (st->done) return;
  const bool need = rho_needed(st);
  __shared__ double red[4];
  // M_u S' and the small matrices N_v, G_u, G_v in LDS (the loops below read them at a
  // data-dependent length, so from memory every read would wait on its own latency)
  __shared__ double Am[kPMax][kPMax + 1], Nvs[kPMax][kPMax + 1], Gus[kPMax][kPMax + 1], Gvs[kPMax][kPMax + 1];
  __shared__ double Sos[kPMax];
  double rho = INFINITY;
  if (need) {
    const int r = st->r[a.nb_new], ro = st->r[a.nb_old];
    const double* S = st->S[a.nb_new];
    const double* So = Sos;
    const double* Mu = a.M;
    // every thread's loads are issued together (unrolled, fixed count), not one wait each
    constexpr int kPer = kPMax * kPMax / 256;  // 16 (the kernel runs 256 threads)
    if (threadIdx.x < kPMax) Sos[threadIdx.x] = st->S[a.nb_old][threadIdx.x];
    {
      double vn[kPer], vu[kPer], vv[kPer], vm[kPer];
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const int e = threadIdx.x + 256 * m;
        vn[m] = a.M[kPMax * kPMax + e];
        vu[m] = a.G[e];
        vv[m] = a.G[kPMax * kPMax + e];
        vm[m] = Mu[e];
      }
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const int e = threadIdx.x + 256 * m, aa = e / kPMax, c = e % kPMax;
        Nvs[aa][c] = vn[m];
        Gus[aa][c] = vu[m];
        Gvs[aa][c] = vv[m];
        Am[aa][c] = vm[m];  // M_u for now; times S' below
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int e = threadIdx.x + 256 * m, aa = e / kPMax, c = e % kPMax;
      Am[aa][c] = (aa < r && c < ro) ? Am[aa][c] * So[c] : 0.0;  // M_u S'
    }
    __syncthreads();
    // N_v S' (Bm) is formed where it is used, with the same rounding as a stored product
    auto Bm = [&](int aa, int m) { return (aa < r && m < ro) ? Nvs[aa][m] * So[m] : 0.0; };
    // T1 to T3 over 4 x 4 blocks of entries, thread t taking rows a0 .. a0+3 and columns
    // c0 .. c0+3 (the 256 threads tile 64 x 64), so that every operand read from LDS serves four
    // entries; each entry sums over m in increasing order.
    double part = 0.0;
    const int a0 = 4 * (threadIdx.x >> 4), c0 = 4 * (threadIdx.x & 15);
    if (a0 < r && c0 < r) {  // T1: ||S_k - M_u S' N_v^T||^2
      double sq[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) sq[i][j] = (a0 + i == c0 + j && a0 + i < r) ? S[a0 + i] : 0.0;
      for (int m = 0; m < ro; ++m) {
        double am[4], nv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          am[i] = Am[a0 + i][m];
          nv[i] = Nvs[c0 + i][m];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) sq[i][j] = fma(-am[i], nv[j], sq[i][j]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (a0 + i < r && c0 + j < r) part = fma(sq[i][j], sq[i][j], part);
    }
    if (a0 < r && c0 < ro) {  // T2 and T3
      double p2[4][4], p3[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) p2[i][j] = p3[i][j] = 0.0;
      for (int m = 0; m < ro; ++m) {
        double am[4], bm[4], gv[4], gu[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          am[i] = Am[a0 + i][m];
          bm[i] = Bm(a0 + i, m);
          gv[i] = Gvs[m][c0 + i];
          gu[i] = Gus[m][c0 + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            p2[i][j] = fma(am[i], gv[j], p2[i][j]);
            p3[i][j] = fma(bm[i], gu[j], p3[i][j]);
          }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (a0 + i < r && c0 + j < ro) {
            part = fma(p2[i][j], Am[a0 + i][c0 + j], part);
            part = fma(p3[i][j], Bm(a0 + i, c0 + j), part);
          }
    }
    for (int e = threadIdx.x; e < ro * ro; e += blockDim.x) {  // T4
      const int m = e / ro, m2 = e % ro;
      part += So[m] * Gus[m][m2] * So[m2] * Gvs[m2][m];
    }
    const double tot = block_sum256(part, red);
    rho = sqrt(fmax(tot, 0.0)) / st->nrm;
  }
  if (threadIdx.x == 0) {
    const int kp = st->k;
    st->rho = rho;
    st->rhob[a.nb_new] = rho;
    if (kp < a.maxiter) a.trace.rho[kp] = rho;
  }
}

int rho_plan(RhoPlan* p, int64_t n) {
  p->n = n;
  const int64_t chunks = (n + 255) / 256;
  const int64_t per = (chunks + 511) / 512;  // 256-row chunks per block, <= 512 blocks
  p->nblocks = (int)((chunks + per - 1) / per);
  if (hipMalloc(&p->part, sizeof(double) * (size_t)p->nblocks * 2 * kPMax * kPMax) != hipSuccess)
    return LRP_ENOMEM;
  if (hipMalloc(&p->M, sizeof(double) * 2 * kPMax * kPMax) != hipSuccess) return LRP_ENOMEM;
  if (hipMalloc(&p->G, sizeof(double) * 2 * kPMax * kPMax) != hipSuccess) return LRP_ENOMEM;
  return LRP_OK;
}

int rho_launch(const RhoPlan& p, const RhoArgs& ra, hipStream_t s) {
  const int64_t chunks = (p.n + 255) / 256;
  const int64_t per = (chunks + 511) / 512;
  RhoKArgs a{};
  a.st = ra.st;
  for (int q = 0; q < 2; ++q) {
    a.A[q] = ra.Unew[q];
    a.B[q] = ra.Uold[q];
  }
  a.ldu = ra.ldu;
  a.n = p.n;
  a.rows_per_block = (int)(per * 256);
  a.nb_new = ra.nb_new;
  a.nb_old = ra.nb_old;
  a.part = p.part;
  const int red_blocks = (2 * kPMax * kPMax + 255) / 256;
  LRP_LAUNCH_G(K_RHO_A, k_rho_a<RhoKArgs>, k_rho_a<GroupRef>, dim3(p.nblocks, 2), dim3(kRhoThreads), 0, s, a);
  const RhoReduceArgs rd{ra.st, p.part, p.nblocks, p.M, ra.nb_new, ra.nb_old};
  LRP_LAUNCH_G(K_RHO_REDUCE, k_rho_reduce<RhoReduceArgs>, k_rho_reduce<GroupRef>, dim3(red_blocks), dim3(256), 0, s,
               rd);
  a.M = p.M;
  LRP_LAUNCH_G(K_RHO_B, k_rho_b<RhoKArgs>, k_rho_b<GroupRef>, dim3(p.nblocks, 2), dim3(kRhoThreads), 0, s, a);
  const RhoReduceArgs rg{ra.st, p.part, p.nblocks, p.G, ra.nb_old, ra.nb_old};
  LRP_LAUNCH_G(K_RHO_REDUCE, k_rho_reduce<RhoReduceArgs>, k_rho_reduce<GroupRef>, dim3(red_blocks), dim3(256), 0, s,
               rg);
  RhoFinalArgs f{};
  f.st = ra.st;
  f.M = p.M;
  f.G = p.G;
  f.nb_new = ra.nb_new;
  f.nb_old = ra.nb_old;
  f.maxiter = ra.maxiter;
  f.trace = ra.trace;
  LRP_LAUNCH_G(K_RHO_FINAL, k_rho_final<RhoFinalArgs>, k_rho_final<GroupRef>, dim3(1), dim3(256), 0, s, f);
  return launch_status();
}

}  // namespace lrp
