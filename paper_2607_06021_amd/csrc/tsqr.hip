// Tall-skinny Householder QR (the thin QRs C = Q R_C and R^T = Z R_R of Algorithm 1).
//
// The n x p matrix is cut into 256-row blocks. Each block is factored by one workgroup with
// LAPACK's Householder convention (beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta,
// v = x/(alpha - beta), v_0 = 1). The p x p R factors are stacked and factored again, in
// groups of 256/p_max, up a tree until one block is left; its R is the R of the matrix.
// Q is formed top-down: each block applies its reflectors to [T; 0], where T is its p x p
// piece of the parent level's Q.
//
// Register layout of a block: thread t owns column c = t/4 and rows 64 (t%4) .. 64 (t%4)+63,
// so the column dot products of a Householder step reduce over the 4 lanes of a quad. The
// current Householder vector is shared through LDS. Two sides (e.g. C and R^T) are processed
// by the same launch (blockIdx.y).
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

__global__ __launch_bounds__(kTsqrThreads) void k_tsqr_factor(FactorArgs a) {
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, c = t >> 2, sub = t & 3;
  __shared__ double colbuf[kTsqrRows];
  __shared__ double vbuf[kTsqrRows];
  __shared__ double part[4];

  double x[64];
  {
    const int64_t base = row0 + (int64_t)c * a.ldin + sub * 64;
    const bool colok = c < p;
    if (a.in_f32) {
      const float* X = (const float*)a.in[side];
#pragma unroll
      for (int i = 0; i < 64; ++i) x[i] = (colok && sub * 64 + i < nr) ? (double)X[base + i] : 0.0;
    } else {
      const double* X = (const double*)a.in[side];
#pragma unroll
      for (int i = 0; i < 64; ++i) x[i] = (colok && sub * 64 + i < nr) ? X[base + i] : 0.0;
    }
  }
  double* V = a.V[side];
  double* Rb = a.Rout[side] + (int64_t)blockIdx.x * a.pmax;  // this block's R, rows 0..pmax-1
  double* taub = a.tau[side] + (int64_t)blockIdx.x * a.pmax;

  for (int j = 0; j < p; ++j) {
    if (c == j) {
#pragma unroll
      for (int i = 0; i < 64; ++i) colbuf[sub * 64 + i] = x[i];
    }
    __syncthreads();
    const double xv = colbuf[t];
    double nn = (t > j) ? xv * xv : 0.0;
    nn = wave_sum(nn);
    if ((t & 63) == 0) part[t >> 6] = nn;
    __syncthreads();
    const double xnorm2 = (part[0] + part[1]) + (part[2] + part[3]);
    const double alpha = colbuf[j];
    double beta, tau, scale;
    if (xnorm2 == 0.0) {
      tau = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    const double vt = (t > j) ? xv * scale : (t == j ? 1.0 : 0.0);
    vbuf[t] = vt;
    if (t < nr) V[row0 + t + (int64_t)j * a.ldv] = vt;
    if (t < a.pmax) Rb[t + (int64_t)j * a.ldr] = (t < j) ? xv : (t == j ? beta : 0.0);
    if (t == 0) taub[j] = tau;
    __syncthreads();
    if (c > j && c < p) {
      const double* vb = vbuf + sub * 64;
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < 64; i += 2) {
        d0 = fma(vb[i], x[i], d0);
        d1 = fma(vb[i + 1], x[i + 1], d1);
      }
      const double w = quad_sum(d0 + d1) * tau;
#pragma unroll
      for (int i = 0; i < 64; ++i) x[i] = fma(-w, vb[i], x[i]);
    }
  }
}

__global__ __launch_bounds__(kTsqrThreads) void k_tsqr_apply(ApplyArgs a) {
  const int side = blockIdx.y;
  if (a.st && a.st->done) return;
  const int p = side_cols(a.st, a.ncols, side);
  const int64_t row0 = (int64_t)blockIdx.x * a.block_rows;
  const int nr = (int)min((int64_t)a.block_rows, a.rows - row0);
  if (p <= 0 || nr <= 0) return;
  const int t = threadIdx.x, c = t >> 2, sub = t & 3;
  __shared__ double vbuf[2][kTsqrRows];

  double y[64];
  const double* T = a.T[side];
  const int64_t toff = (int64_t)blockIdx.x * a.pmax;
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    const int lr = sub * 64 + i;
    double v0 = 0.0;
    if (c < p && lr < p) v0 = T ? T[toff + lr + (int64_t)c * a.ldt] : (lr == c ? 1.0 : 0.0);
    y[i] = v0;
  }
  const double* V = a.V[side];
  const double* taub = a.tau[side] + (int64_t)blockIdx.x * a.pmax;
  for (int j = p - 1; j >= 0; --j) {
    double* vb = vbuf[j & 1];
    vb[t] = (t < nr) ? V[row0 + t + (int64_t)j * a.ldv] : 0.0;
    const double tj = taub[j];
    __syncthreads();
    if (c < p && tj != 0.0) {
      const double* vs = vb + sub * 64;
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < 64; i += 2) {
        d0 = fma(vs[i], y[i], d0);
        d1 = fma(vs[i + 1], y[i + 1], d1);
      }
      const double w = quad_sum(d0 + d1) * tj;
#pragma unroll
      for (int i = 0; i < 64; ++i) y[i] = fma(-w, vs[i], y[i]);
    }
  }
  if (c < p) {
    double* Y = a.Y[side] + row0 + (int64_t)c * a.ldy + sub * 64;
#pragma unroll
    for (int i = 0; i < 64; ++i)
      if (sub * 64 + i < nr) Y[i] = y[i];
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
      if (hipMemset(lv.Rout[s], 0, rb) != hipSuccess) return LRP_EDEVICE;
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
    hipLaunchKernelGGL(k_tsqr_apply, dim3(lv.nblocks, ns), dim3(kTsqrThreads), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // namespace lrp
