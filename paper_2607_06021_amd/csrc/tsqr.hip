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

// Thread layout of a 256-row block: column c = t/16, rows 16 (t%16) .. 16 (t%16)+15, so the
// 16 lanes of a DPP row hold one column. The lanes of column j build reflector j themselves
// (norm and diagonal by row sums), publish it in LDS (double-buffered; element 16 s + i of the
// column is stored at 16 i + s, so that the 16 lanes of a column read 16 consecutive words)
// and one barrier later every trailing column applies it.
__global__ __launch_bounds__(kTsqrThreads) void k_tsqr_factor(FactorArgs a) {
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, c = t >> 4, sub = t & 15;
  const int rbase = sub * kTsqrRowsPerThread;
  __shared__ double vbuf[2][kTsqrRows];

  double x[kTsqrRowsPerThread];
  {
    const int64_t base = row0 + (int64_t)c * a.ldin + rbase;
    const bool colok = c < p;
    if (a.in_f32) {
      const float* X = (const float*)a.in[side];
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; ++i) x[i] = (colok && rbase + i < nr) ? (double)X[base + i] : 0.0;
    } else {
      const double* X = (const double*)a.in[side];
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; ++i) x[i] = (colok && rbase + i < nr) ? X[base + i] : 0.0;
    }
  }
  double* V = a.V[side];
  double* Rb = a.Rout[side] + (int64_t)blockIdx.x * a.pmax;  // this block's R, rows 0..pmax-1
  double* taub = a.tau[side] + (int64_t)blockIdx.x * a.pmax;
  __shared__ double tsh[kPMax];
  // After its own step, column c is final: its registers keep R(0..c-1, c) above the diagonal
  // and the reflector below it, and rdiag = R(c, c). Nothing is written to global memory
  // inside the loop, so the per-step barrier waits on LDS only.
  double rdiag = 0.0;

  for (int j = 0; j < p; ++j) {
    double* vb = vbuf[j & 1];
    if (c == j) {
      // two partial sums shorten the dependent chain of the norm
      double n0 = 0.0, n1 = 0.0, al = 0.0;
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; i += 2) {
        const int r = rbase + i;
        n0 = (r > j) ? fma(x[i], x[i], n0) : n0;
        n1 = (r + 1 > j) ? fma(x[i + 1], x[i + 1], n1) : n1;
        al = (r == j) ? x[i] : al;
        al = (r + 1 == j) ? x[i + 1] : al;
      }
      const double xnorm2 = row16_sum(n0 + n1);
      const double alpha = row16_sum(al);
      double beta, tau, scale;
      const double h2 = fma(alpha, alpha, xnorm2);
      if (xnorm2 == 0.0) {
        tau = 0.0;
        beta = alpha;
        scale = 0.0;
      } else if (h2 > 1e-290 && h2 < 1e290) {  // hardware rsq/rcp refined by Newton steps
        beta = -copysign(h2 * rsq_nr(h2), alpha);
        tau = (beta - alpha) * rcp_nr(beta);
        scale = rcp_nr(alpha - beta);
      } else {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; ++i) {
        const int r = rbase + i;
        const double v = (r > j) ? x[i] * scale : (r == j ? 1.0 : 0.0);
        vb[i * 16 + sub] = v;  // transposed: the 16 lanes of a column read consecutive words
        if (r > j) x[i] = v;
      }
      rdiag = beta;
      if (sub == 0) tsh[j] = tau;
    }
    __syncthreads();
    if (c > j && c < p) {
      const double tau = tsh[j];
      const double* vs = vb + sub;
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; i += 2) {
        d0 = fma(vs[i * 16], x[i], d0);
        d1 = fma(vs[(i + 1) * 16], x[i + 1], d1);
      }
      const double w = row16_sum(d0 + d1) * tau;
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; ++i) x[i] = fma(-w, vs[i * 16], x[i]);
    }
  }
  // write the reflectors, R and tau once
  if (c < p) {
#pragma unroll
    for (int i = 0; i < kTsqrRowsPerThread; ++i) {
      const int r = rbase + i;
      if (r < nr) V[row0 + r + (int64_t)c * a.ldv] = (r > c) ? x[i] : (r == c ? 1.0 : 0.0);
      if (r < a.pmax) Rb[r + (int64_t)c * a.ldr] = (r < c) ? x[i] : (r == c ? rdiag : 0.0);
    }
  }
  if (t < p) taub[t] = tsh[t];
}

// Same thread layout as the factorization: thread (c, sub) keeps rows 16 sub .. 16 sub + 15 of
// output column c and, loaded once at the start, the same rows of reflector c. Reflectors are
// applied in reverse order; at step j the lanes of column j publish v_j in LDS
// (double-buffered) and one barrier later every column applies it.
__global__ __launch_bounds__(kTsqrThreads) void k_tsqr_apply(ApplyArgs a) {
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, c = t >> 4, sub = t & 15;
  const int rbase = sub * kTsqrRowsPerThread;
  __shared__ double vbuf[2][kTsqrRows];
  __shared__ double tsh[kPMax];

  const double* taub = a.tau[side] + (int64_t)blockIdx.x * a.pmax;
  if (t < p) tsh[t] = taub[t];
  double y[kTsqrRowsPerThread], v[kTsqrRowsPerThread];
  const double* T = a.T[side];
  const int64_t toff = (int64_t)blockIdx.x * a.pmax;
  const double* V = a.V[side] + row0 + (int64_t)c * a.ldv + rbase;
#pragma unroll
  for (int i = 0; i < kTsqrRowsPerThread; ++i) {
    const int lr = rbase + i;
    double v0 = 0.0;
    if (c < p && lr < p) v0 = T ? T[toff + lr + (int64_t)c * a.ldt] : (lr == c ? 1.0 : 0.0);
    y[i] = v0;
    v[i] = (c < p && lr < nr) ? V[i] : 0.0;
  }
  for (int j = p - 1; j >= 0; --j) {
    double* vb = vbuf[j & 1];
    if (c == j) {
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; ++i) vb[i * 16 + sub] = v[i];
    }
    __syncthreads();
    const double tj = tsh[j];
    if (c < p && tj != 0.0) {
      const double* vs = vb + sub;
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; i += 2) {
        d0 = fma(vs[i * 16], y[i], d0);
        d1 = fma(vs[(i + 1) * 16], y[i + 1], d1);
      }
      const double w = row16_sum(d0 + d1) * tj;
#pragma unroll
      for (int i = 0; i < kTsqrRowsPerThread; ++i) y[i] = fma(-w, vs[i * 16], y[i]);
    }
  }
  if (c < p) {
    double* Y = a.Y[side] + row0 + (int64_t)c * a.ldy + rbase;
#pragma unroll
    for (int i = 0; i < kTsqrRowsPerThread; ++i)
      if (rbase + i < nr) Y[i] = y[i];
  }
}

// ----------------------------------------------------------------------------------------
int tsqr_plan(TsqrPlan* p, int64_t n, int pmax) {
  if (pmax < 1 || pmax > kPMax) return LRP_EINVAL;
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
    for (int s = 0; s < 2; ++s) {
      size_t vb = sizeof(double) * (size_t)rows * pmax;
      size_t tb = sizeof(double) * (size_t)lv.nblocks * pmax;
      size_t rb = sizeof(double) * (size_t)lv.nblocks * pmax * pmax;
      if (hipMalloc(&lv.V[s], vb) != hipSuccess) return LRP_ENOMEM;
      if (hipMalloc(&lv.tau[s], tb) != hipSuccess) return LRP_ENOMEM;
      if (hipMalloc(&lv.Rout[s], rb) != hipSuccess) return LRP_ENOMEM;
      if (hipMalloc(&lv.Y[s], vb) != hipSuccess) return LRP_ENOMEM;
      // no initialisation: every element of R that is read (columns below the active width,
      // all pmax rows) is written by the factorization first. (A plain memset here would run
      // on the null stream, unordered with the context's non-blocking stream.)
    }
    ++L;
    if (lv.nblocks == 1) break;
    rows = (int64_t)lv.nblocks * pmax;
    br = g * pmax;
  }
  p->nlevels = L;
  return LRP_OK;
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
    prof_mark(s, K_TSQR_FACTOR);
    hipLaunchKernelGGL(k_tsqr_factor, dim3(lv.nblocks, ns), dim3(kTsqrThreads), 0, s, f);
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
    prof_mark(s, K_TSQR_APPLY);
    hipLaunchKernelGGL(k_tsqr_apply, dim3(lv.nblocks, ns), dim3(kTsqrThreads), 0, s, a);
  }
  return launch_status();
}

}  // namespace lrp
