// The small dense steps of one Cross-DEIM pass, on one workgroup (paper, Algorithm 1
// steps after the QRs, and Algorithm 4's pruning and stopping test):
//   * with A = Q(I,:) (|J| <= |I|) or A = Z(J,:) (otherwise), its pseudo-inverse from a
//     one-sided Jacobi SVD, dropping singular values <= max(rows, cols) eps sigma_1;
//   * the |J| x |I| core M = Q(I,:)^+ R_R^T, or M = R_C (Z(J,:)^+)^T, so that the cross
//     approximation is Q M Z^T;
//   * the SVD of M = U^ S V~^T, truncated at max(|I|, |J|) eps sigma_1 (U_k = Q U^ and
//     V_k = Z V~ are formed by the product kernel);
//   * pruning: index l of I (of J) is dropped when |diag R_R| (|diag R_C|) at l is below
//     tau times its largest entry;
//   * eta_1 = 1/sigma_min(U_k(I,:)), eta_2 = 1/sigma_min(V_k(J,:)) on the pruned sets and the
//     indicator min(eta_1 (1 + eta_2), eta_2 (1 + eta_1)) S_min / ||S||_F.
// The warm start uses the same machinery on M = R_u R_v^T, the core of F^ = U^ V^^T.
//
// Jacobi: Hestenes' method, round-robin ordering (k-1 rounds of k/2 disjoint pairs per
// sweep), 8 lanes per column pair, rotation skipped when |a_p . a_q| <= sqrt(m) eps
// ||a_p|| ||a_q||; sweeps end when a whole sweep makes no rotation (at most 60).
#include "lrp_kernels.h"

namespace lrp {

constexpr int LD = kPMax;  // leading dimension of the LDS matrices

__device__ void jacobi_cols(double* A, int m, int k, double* V, int* flag) {
  const int t = threadIdx.x;
  const int pi = t >> 3, li = t & 7;
  const int kk = k + (k & 1);
  const int npairs = kk >> 1;
  const double tol = sqrt((double)m) * kEps;
  if (k < 2) {
    __syncthreads();
    return;
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int rd = 0; rd < kk - 1; ++rd) {
      if (pi < npairs) {
        int p, q;
        if (pi == 0) {
          p = kk - 1;
          q = rd;
        } else {
          p = (rd + pi) % (kk - 1);
          q = (rd - pi + (kk - 1)) % (kk - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q < k) {
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = li; i < m; i += 8) {
            const double ap = A[i + p * LD], aq = A[i + q * LD];
            al = fma(ap, ap, al);
            be = fma(aq, aq, be);
            ga = fma(ap, aq, ga);
          }
          al = oct_sum(al);
          be = oct_sum(be);
          ga = oct_sum(ga);
          if (ga != 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
            const double zeta = (be - al) / (2.0 * ga);
            double tt;
            if (fabs(zeta) > 1e150)
              tt = 0.5 / zeta;
            else
              tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt);
            const double sn = cs * tt;
            for (int i = li; i < m; i += 8) {
              const double ap = A[i + p * LD], aq = A[i + q * LD];
              A[i + p * LD] = cs * ap - sn * aq;
              A[i + q * LD] = sn * ap + cs * aq;
            }
            if (V) {
              for (int i = li; i < k; i += 8) {
                const double vp = V[i + p * LD], vq = V[i + q * LD];
                V[i + p * LD] = cs * vp - sn * vq;
                V[i + q * LD] = sn * vp + cs * vq;
              }
            }
            if (li == 0) *flag = 1;
          }
        }
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) break;
  }
}

// sig[c] = ||A(:, c)||, ord[r] = column of rank r (descending, ties to the smaller index).
__device__ void norms_sorted(const double* A, int m, int k, double* sig, int* ord) {
  const int t = threadIdx.x;
  if (t < k) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(A[i + t * LD], A[i + t * LD], s);
    sig[t] = sqrt(s);
  }
  __syncthreads();
  if (t < k) {
    const double v = sig[t];
    int rk = 0;
    for (int c = 0; c < k; ++c) rk += (sig[c] > v || (sig[c] == v && c < t)) ? 1 : 0;
    ord[rk] = t;
  }
  __syncthreads();
}

__device__ void set_identity(double* V, int k) {
  for (int e = threadIdx.x; e < k * LD; e += blockDim.x) {
    const int i = e % LD, j = e / LD;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
}

// sigma_min over the min(rows, cols) singular values of the rows x cols matrix E in X.
__device__ double sigma_min_of(double* X, double* Xt, int rows, int cols, double* sig, int* ord,
                               int* flag) {
  if (rows == 0 || cols == 0) return 0.0;
  double* A = X;
  int m = rows, k = cols;
  if (rows < cols) {  // work on the transpose so that the matrix is tall
    for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
      const int i = e % rows, j = e / rows;
      Xt[j + i * LD] = X[i + j * LD];
    }
    __syncthreads();
    A = Xt;
    m = cols;
    k = rows;
  }
  jacobi_cols(A, m, k, nullptr, flag);
  norms_sorted(A, m, k, sig, ord);
  return sig[ord[k - 1]];
}

// Singular values of M (nJ x nI, in W) -> U^ (nJ x r) in Ub, V~ (nI x r) in Vb, sorted.
// Returns r; X and Vj are work buffers.
__device__ int svd_core(const double* W, int nJ, int nI, double cut_mult, double* X, double* Vj,
                        double* Ub, double* Vb, double* sig, int* ord, int* flag) {
  const bool tall = nJ >= nI;
  const int m = tall ? nJ : nI, k = tall ? nI : nJ;
  for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
    const int i = e % m, j = e / m;
    X[i + j * LD] = tall ? W[i + j * LD] : W[j + i * LD];
  }
  set_identity(Vj, k);
  __syncthreads();
  jacobi_cols(X, m, k, Vj, flag);
  norms_sorted(X, m, k, sig, ord);
  const double smax = sig[ord[0]];
  int r = 0;
  if (smax > 0.0) {
    const double cut = cut_mult * kEps * smax;
    for (int c = 0; c < k; ++c) r += sig[ord[c]] > cut ? 1 : 0;
  }
  // left factor of the tall orientation: X(:, c)/sig_c; right: Vj(:, c)
  for (int e = threadIdx.x; e < r * LD; e += blockDim.x) {
    const int i = e % LD, rr = e / LD;
    const int c = ord[rr];
    const double inv = 1.0 / sig[c];
    const double lx = i < m ? X[i + c * LD] * inv : 0.0;
    const double rv = i < k ? Vj[i + c * LD] : 0.0;
    if (tall) {
      Ub[i + rr * LD] = lx;
      Vb[i + rr * LD] = rv;
    } else {
      Ub[i + rr * LD] = rv;
      Vb[i + rr * LD] = lx;
    }
  }
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_core(CoreArgs a) {
  DevState* st = a.st;
  if (st->done) return;
  __shared__ double X[LD * LD], Vj[LD * LD], T[LD * LD], W[LD * LD];
  __shared__ double sig[kPMax];
  __shared__ int ord[kPMax];
  __shared__ int flag;
  __shared__ int keepI[kPMax], keepJ[kPMax], posI[kPMax], posJ[kPMax];
  __shared__ double red[8];
  const int t = threadIdx.x;
  const int nI = st->nIpre, nJ = st->nJpre;
  const int pm = a.pmax;
  const double* R_C = a.R0;  // nJ x nJ upper triangular, ld pm
  const double* R_R = a.R1;  // nI x nI
  auto Aq = [&](int i, int c) { return a.Q0[st->Ipre[i] + (int64_t)c * a.ldq]; };  // Q(I,:)
  auto Bq = [&](int j, int c) { return a.Q1[st->Jpre[j] + (int64_t)c * a.ldq]; };  // Z(J,:)
  const double cut_pinv = (double)max(nI, nJ);

  // ---- pseudo-inverse and the core M (into W, nJ x nI)
  const bool branch = nJ <= nI;
  const int m0 = branch ? nI : nJ, k0 = branch ? nJ : nI;
  for (int e = t; e < m0 * k0; e += blockDim.x) {
    const int i = e % m0, c = e / m0;
    X[i + c * LD] = branch ? Aq(i, c) : Bq(i, c);
  }
  set_identity(Vj, k0);
  __syncthreads();
  jacobi_cols(X, m0, k0, Vj, &flag);
  norms_sorted(X, m0, k0, sig, ord);
  {
    const double smax = sig[ord[0]];
    const double cut = cut_pinv * kEps * smax;
    // scaled left factor: X(:, c) / sig_c^2 (= U_c / sig_c), zero where dropped
    for (int e = t; e < m0 * k0; e += blockDim.x) {
      const int i = e % m0, c = e / m0;
      const double s = sig[c];
      X[i + c * LD] = (smax > 0.0 && s > cut) ? X[i + c * LD] / (s * s) : 0.0;
    }
    __syncthreads();
  }
  if (branch) {
    // pinv(A) = Vj diag(1/s) U^T with A = Q(I,:) (nI x nJ); M = pinv(A) R_R^T (nJ x nI)
    // T(c, j) = sum_i Xs(i, c) R_R(j, i)  (c < nJ, j < nI)
    for (int e = t; e < nJ * nI; e += blockDim.x) {
      const int c = e % nJ, j = e / nJ;
      double s = 0.0;
      for (int i = j; i < nI; ++i) s = fma(X[i + c * LD], R_R[j + (int64_t)i * pm], s);
      T[c + j * LD] = s;
    }
    __syncthreads();
    for (int e = t; e < nJ * nI; e += blockDim.x) {
      const int aa = e % nJ, j = e / nJ;
      double s = 0.0;
      for (int c = 0; c < nJ; ++c) s = fma(Vj[aa + c * LD], T[c + j * LD], s);
      W[aa + j * LD] = s;
    }
  } else {
    // pinv(B) = Vj diag(1/s) U^T with B = Z(J,:) (nJ x nI); M = R_C pinv(B)^T = R_C Xs Vj^T
    for (int e = t; e < nJ * nI; e += blockDim.x) {
      const int aa = e % nJ, c = e / nJ;
      double s = 0.0;
      for (int m = aa; m < nJ; ++m) s = fma(R_C[aa + (int64_t)m * pm], X[m + c * LD], s);
      T[aa + c * LD] = s;
    }
    __syncthreads();
    for (int e = t; e < nJ * nI; e += blockDim.x) {
      const int aa = e % nJ, j = e / nJ;
      double s = 0.0;
      for (int c = 0; c < nI; ++c) s = fma(T[aa + c * LD], Vj[j + c * LD], s);
      W[aa + j * LD] = s;
    }
  }
  __syncthreads();

  // ---- truncated SVD of the core: U^ -> T (nJ x r), V~ -> Vj? (use X/Vj as work)
  // svd_core needs X and Vj as work and writes into the two output buffers; W is the input.
  // Outputs go to T (U^) and a second buffer; reuse W after copying M into X inside svd_core.
  const int r = svd_core(W, nJ, nI, cut_pinv, X, Vj, T, W, sig, ord, &flag);
  // now T = U^ (nJ x r), W = V~ (nI x r), singular values sig[ord[0..r)]
  double* Uhat = a.Uhat;
  double* Vtil = a.Vtil;
  for (int e = t; e < r * pm; e += blockDim.x) {
    const int i = e % pm, rr = e / pm;
    Uhat[i + (int64_t)rr * pm] = i < nJ ? T[i + rr * LD] : 0.0;
    Vtil[i + (int64_t)rr * pm] = i < nI ? W[i + rr * LD] : 0.0;
  }
  const int nb = a.nb;
  if (t < kPMax) st->S[nb][t] = t < r ? sig[ord[t]] : 0.0;

  // ---- pruning
  if (t == 0) {
    double mR = 0.0, mC = 0.0;
    for (int l = 0; l < nI; ++l) mR = fmax(mR, fabs(R_R[l + (int64_t)l * pm]));
    for (int l = 0; l < nJ; ++l) mC = fmax(mC, fabs(R_C[l + (int64_t)l * pm]));
    int ci = 0, cj = 0;
    for (int l = 0; l < nI; ++l) {
      keepI[l] = fabs(R_R[l + (int64_t)l * pm]) >= st->tau * mR;
      if (keepI[l]) posI[ci++] = l;
    }
    for (int l = 0; l < nJ; ++l) {
      keepJ[l] = fabs(R_C[l + (int64_t)l * pm]) >= st->tau * mC;
      if (keepJ[l]) posJ[cj++] = l;
    }
    red[0] = ci;
    red[1] = cj;
  }
  __syncthreads();
  const int nIp = (int)red[0], nJp = (int)red[1];

  // ---- eta_1 = 1 / sigma_min(U_k(I,:)) with U_k(I,:) = Q(I,:) U^ on the pruned rows
  double smin1 = 0.0, smin2 = 0.0;
  if (r > 0) {
    for (int e = t; e < nIp * r; e += blockDim.x) {
      const int ii = e % nIp, rr = e / nIp;
      const int i = posI[ii];
      double s = 0.0;
      for (int c = 0; c < nJ; ++c) s = fma(Aq(i, c), T[c + rr * LD], s);
      X[ii + rr * LD] = s;
    }
    __syncthreads();
    smin1 = sigma_min_of(X, Vj, nIp, r, sig, ord, &flag);
    __syncthreads();
    // eta_2 with V_k(J,:) = Z(J,:) V~
    for (int e = t; e < nJp * r; e += blockDim.x) {
      const int jj = e % nJp, rr = e / nJp;
      const int j = posJ[jj];
      double s = 0.0;
      for (int c = 0; c < nI; ++c) s = fma(Bq(j, c), W[c + rr * LD], s);
      X[jj + rr * LD] = s;
    }
    __syncthreads();
    smin2 = sigma_min_of(X, Vj, nJp, r, sig, ord, &flag);
  }
  __syncthreads();

  if (t == 0) {
    const double* S = st->S[nb];
    double nrm2 = 0.0;
    for (int l = 0; l < r; ++l) nrm2 = fma(S[l], S[l], nrm2);
    const double nrm = sqrt(nrm2);
    const double eta1 = smin1 > 0.0 ? 1.0 / smin1 : INFINITY;
    const double eta2 = smin2 > 0.0 ? 1.0 / smin2 : INFINITY;
    double ind = INFINITY;
    if (r > 0 && nrm > 0.0) ind = fmin(eta1 * (1.0 + eta2), eta2 * (1.0 + eta1)) * S[r - 1] / nrm;
    st->nrm = nrm;
    st->eta1 = eta1;
    st->eta2 = eta2;
    st->ind = ind;
    st->r[nb] = r;
    int rs = 0;
    for (int l = 0; l < r; ++l) rs += S[l] > st->eps * S[0] ? 1 : 0;
    st->r_sig = rs;
    for (int ii = 0; ii < nIp; ++ii) st->I[ii] = st->Ipre[posI[ii]];
    for (int jj = 0; jj < nJp; ++jj) st->J[jj] = st->Jpre[posJ[jj]];
    st->nI = nIp;
    st->nJ = nJp;
    for (int ii = 0; ii < nIp; ++ii) st->Ib[nb][ii] = st->I[ii];
    for (int jj = 0; jj < nJp; ++jj) st->Jb[nb][jj] = st->J[jj];
    st->nIb[nb] = nIp;
    st->nJb[nb] = nJp;
    st->indb[nb] = ind;
    if (r == 0) {  // the sampled fibers vanish: nothing to continue from
      st->done = 1;
      st->status = LRP_ENUMERIC;
    }
    const int kp = a.kpass;
    if (kp >= 0 && kp < a.maxiter) {
      a.trace.nI[kp] = nIp;
      a.trace.nJ[kp] = nJp;
      a.trace.rank[kp] = r;
      a.trace.ind[kp] = ind;
    }
  }
}

// Warm start: M = R_u R_v^T (the core of F^ = U^ V^^T) and its SVD.
__global__ __launch_bounds__(256) void k_core_warm(CoreArgs a) {
  DevState* st = a.st;
  if (st->done) return;
  __shared__ double X[LD * LD], Vj[LD * LD], T[LD * LD], W[LD * LD];
  __shared__ double sig[kPMax];
  __shared__ int ord[kPMax];
  __shared__ int flag;
  const int t = threadIdx.x;
  const int rF = st->rF;
  const int pm = a.pmax;
  for (int e = t; e < rF * rF; e += blockDim.x) {
    const int i = e % rF, j = e / rF;
    double s = 0.0;
    for (int m = max(i, j); m < rF; ++m) s = fma(a.R0[i + (int64_t)m * pm], a.R1[j + (int64_t)m * pm], s);
    W[i + j * LD] = s;
  }
  __syncthreads();
  const int r = svd_core(W, rF, rF, (double)rF, X, Vj, T, W, sig, ord, &flag);
  for (int e = t; e < r * pm; e += blockDim.x) {
    const int i = e % pm, rr = e / pm;
    a.Uhat[i + (int64_t)rr * pm] = i < rF ? T[i + rr * LD] : 0.0;
    a.Vtil[i + (int64_t)rr * pm] = i < rF ? W[i + rr * LD] : 0.0;
  }
  if (t < kPMax) st->S[0][t] = t < r ? sig[ord[t]] : 0.0;
  __syncthreads();
  if (t == 0) {
    st->r[0] = r;
    st->nIb[0] = 0;
    st->nJb[0] = 0;
    st->indb[0] = INFINITY;
    if (r == 0) {  // F = 0: the solution is 0
      st->zero = 1;
      st->done = 1;
      st->status = LRP_OK;
      st->r_sig = 0;
    } else {
      int rs = 0;
      for (int l = 0; l < r; ++l) rs += st->S[0][l] > st->eps * st->S[0][0] ? 1 : 0;
      st->r_sig = rs;
    }
  }
}

int core_launch(const CoreArgs& a, bool warm, hipStream_t s) {
  if (warm)
    hipLaunchKernelGGL(k_core_warm, dim3(1), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_core, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

// ----------------------------------------------------------------------------------------
// Set-up, input scan and final truncation
// ----------------------------------------------------------------------------------------
__global__ void k_init_state(DevState* st, int rF, double eps, double tau) {
  if (threadIdx.x != 0) return;
  st->done = 0;
  st->status = LRP_NOT_CONVERGED;
  st->k = 0;
  st->ret = 0;
  st->zero = 0;
  st->rF = rF;
  st->ncols[0] = rF;
  st->ncols[1] = rF;
  st->nI = st->nJ = 0;
  st->nIpre = st->nJpre = 0;
  st->nIprev = st->nJprev = -1;
  st->r_sig = 0;
  st->r_final = 1;
  st->nrm = 0.0;
  st->ind = INFINITY;
  st->rho = INFINITY;
  st->eta1 = st->eta2 = INFINITY;
  st->eps = eps;
  st->tau = tau;
  st->r[0] = st->r[1] = 0;
  st->nIb[0] = st->nIb[1] = st->nJb[0] = st->nJb[1] = 0;
  st->rhob[0] = st->rhob[1] = INFINITY;
  st->indb[0] = st->indb[1] = INFINITY;
}

int init_state_launch(DevState* st, int rF, double eps, double tau, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, rF, eps, tau);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

__global__ void k_scan(DevState* st, const double* U, int64_t ldu, const double* V, int64_t ldv,
                       const double* sig, int64_t n, int rF) {
  const int64_t total = n * rF;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    bad |= !isfinite(U[i + c * ldu]) || !isfinite(V[i + c * ldv]);
  }
  if (blockIdx.x == 0 && threadIdx.x < rF) bad |= !isfinite(sig[threadIdx.x]);
  if (bad) {
    st->status = LRP_ENUMERIC;
    st->done = 1;
  }
}

int scan_inputs_launch(DevState* st, const double* U, int64_t ldu, const double* V, int64_t ldv,
                       const double* sig, int64_t n, int rF, hipStream_t s) {
  const int64_t total = n * rF;
  const int blocks = (int)std::min<int64_t>(1024, (total + 255) / 256);
  hipLaunchKernelGGL(k_scan, dim3(std::max(blocks, 1)), dim3(256), 0, s, st, U, ldu, V, ldv, sig, n, rF);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

// r* = smallest r with sum_{l >= r} S_l^2 < (eps ||S||)^2 ; rank = max(min(r*, r_max), 1).
__global__ void k_finalize(DevState* st, double* S_out, int r_max) {
  if (threadIdx.x != 0) return;
  if (st->status < 0) return;
  int rank = 1;
  const int b = st->ret;
  const double* S = st->S[b];
  if (!st->zero) {
    const int m = st->r[b];
    double nrm2 = 0.0;
    for (int l = 0; l < m; ++l) nrm2 = fma(S[l], S[l], nrm2);
    const double thr = (st->eps * sqrt(nrm2)) * (st->eps * sqrt(nrm2));
    double tail = 0.0;
    int rstar = m;
    for (int rr = m; rr >= 0; --rr) {
      if (rr < m) tail = fma(S[rr], S[rr], tail);
      if (tail < thr)
        rstar = rr;
      else
        break;
    }
    rank = max(min(rstar, r_max), 1);
  }
  st->r_final = rank;
  for (int l = 0; l < r_max; ++l) S_out[l] = (!st->zero && l < rank) ? S[l] : 0.0;
}

int finalize_launch(DevState* st, double* S_out, int r_max, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, st, S_out, r_max);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

// lambda_k = 4 sin^2(pi k / (2(n+1))), k = 1..n (Section 3, eigenvalues of T).
__global__ void k_lambda(double* lam, float* lam32, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = sinpi((double)(i + 1) / (2.0 * (double)(n + 1)));
  const double v = 4.0 * s * s;
  lam[i] = v;
  lam32[i] = (float)v;
}

int lambda_launch(double* lam, float* lam32, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_lambda, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lam, lam32, n);
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // namespace lrp
