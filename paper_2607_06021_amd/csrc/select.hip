// Leverage-score index selection (paper, Algorithm 3) in the deterministic form used here:
//   pi_i = sum_{eta < r_sig} U(i, eta)^2 over the leading r_sig singular vectors;
//   scores <= (64 eps)^2 max_i pi_i are rounding noise and count as 0;
//   the r_sig best indices outside the current (pruned) set are taken, best score first,
//   equal scores to the smaller index; they are appended to the set in ascending order
//   (leverage-score sets carry no order), the set capped at p_max (Algorithm 4's update).
// A pass stops at a fixed point: when both new sets equal the previous pass's sets, the
// cross approximation would repeat, and the previous iterate is the result.
//
// Kernels: k_pi (scores and per-block maxima), k_gmax (global maximum), k_topk_block
// (the best 64 of each 256-row block, ranked by counting), k_topk_merge (16 sorted lists of
// 64 per block merged pairwise, by rank, until one list is left), k_select (set update, fixed-point
// test, trace).
#include "lrp_kernels.h"

namespace lrp {

// Candidate order throughout: a higher key first, then the smaller index. Keys: the floored
// leverage score (>= 0) of a row that may enter the set; with sampling, -1 - u_i (in (-2, -1])
// for a row that was not drawn (the safeguard's random pick is the largest of these); kExcl for
// a row already in the set; kPad for the padding past n.
constexpr double kExcl = -4.0;
constexpr double kPad = -8.0;

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of two 32 x 32 -> 64-bit
// multiplications on the 4 x 32-bit counter, the key bumped by two Weyl constants per round.
// Returns the uniform in [0, 1) made of 53 bits of the first two output words.
__device__ inline double philox_uniform(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  const uint64_t r53 = (((uint64_t)c1 << 32) | c0) >> 11;
  return (double)r53 * 0x1.0p-53;
}

struct PiArgs {
  const DevState* st;
  const double* U[2];
  int64_t ldu;
  int64_t n;
  double* pi[2];
  double* bmax[2];
};

template <class Src>
__global__ __launch_bounds__(256) void k_pi(Src in) {
  const PiArgs& a = kernel_args<PiArgs>(in);
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  const int rs = st->r_sig;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double p = 0.0;
  if (i < a.n) {
    const double* U = a.U[side] + i;
    for (int e = 0; e < rs; ++e) {
      const double u = U[(int64_t)e * a.ldu];
      p = fma(u, u, p);
    }
    a.pi[side][i] = p;
  }
  __shared__ double red[4];
  const double m = block_max256(p, red);
  if (threadIdx.x == 0) a.bmax[side][blockIdx.x] = m;
}

struct GmaxArgs {
  const DevState* st;
  const double* b[2];  // per side: nb block maxima
  int nb;
  double* gmax;        // out: 2
};

template <class Src>
__global__ __launch_bounds__(256) void k_gmax(Src in) {
  const GmaxArgs& a = kernel_args<GmaxArgs>(in);
  if (a.st->done) return;
  const double* b = a.b[blockIdx.x];
  double m = 0.0;
  for (int e = threadIdx.x; e < a.nb; e += blockDim.x) m = fmax(m, b[e]);
  __shared__ double red[4];
  m = block_max256(m, red);
  if (threadIdx.x == 0) a.gmax[blockIdx.x] = m;
}

struct TopkArgs {
  const DevState* st;
  const double* pi[2];
  const double* gmax;
  int64_t n;
  double* cs[2];  // out: nblocks x kPMax scores
  int* ci[2];
  int sampled;    // 1: keep row i with probability min(1, rho score_i) (Algorithm 3)
  double rho;
  uint64_t seed;
};

// Rank of each entry of a 256-row block in the (score desc, index asc) order by counting the
// entries before it; scores sit in their own LDS array and are read two per load (the same
// address on every lane, a broadcast), indices only for a tied score.
template <class Src>
__global__ __launch_bounds__(256) void k_topk_block(Src in) {
  const TopkArgs& a = kernel_args<TopkArgs>(in);
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  __shared__ double2 es2[kSelRows / 2];
  __shared__ int ei[kSelRows];
  __shared__ __align__(16) int excl[kPMax];
  double* es = reinterpret_cast<double*>(es2);
  const int ne = side == 0 ? st->nI : st->nJ;
  const int* set = side == 0 ? st->I : st->J;
  if (threadIdx.x < kPMax) excl[threadIdx.x] = threadIdx.x < ne ? set[threadIdx.x] : -1;
  __syncthreads();
  const double floor_v = kFloorRel * a.gmax[side];
  const int64_t i = (int64_t)blockIdx.x * kSelRows + threadIdx.x;
  double cs;
  int ci;
  if (i < a.n) {
    const double p = a.pi[side][i];
    bool ex = false;
    const int4* ex4 = reinterpret_cast<const int4*>(excl);
#pragma unroll 4
    for (int q = 0; q < kPMax / 4; ++q) {
      const int4 e = ex4[q];
      ex |= (e.x == (int)i) | (e.y == (int)i) | (e.z == (int)i) | (e.w == (int)i);
    }
    const double sc = p <= floor_v ? 0.0 : p;
    cs = ex ? kExcl : sc;
    if (a.sampled && !ex) {
      // uniform of row i for the pass this selection opens (st->k) and this side
      const double u = philox_uniform((uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)st->k, (uint32_t)side,
                                      (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      cs = u < fmin(1.0, a.rho * sc) ? sc : -1.0 - u;
    }
    ci = (int)i;
  } else {  // padding: below every real entry, distinct indices
    cs = kPad;
    ci = 0x40000000 + (int)threadIdx.x;
  }
  es[threadIdx.x] = cs;
  ei[threadIdx.x] = ci;
  __syncthreads();
  int rk = 0;
#pragma unroll 8
  for (int q = 0; q < kSelRows / 2; ++q) {
    const double2 o = es2[q];
    rk += (o.x > cs) + (o.y > cs);
    if (o.x == cs) rk += ei[2 * q] < ci;
    if (o.y == cs) rk += ei[2 * q + 1] < ci;
  }
  if (rk < kPMax) {
    a.cs[side][(int64_t)blockIdx.x * kPMax + rk] = cs;
    a.ci[side][(int64_t)blockIdx.x * kPMax + rk] = ci;
  }
}

struct MergeArgs {
  const DevState* st;
  const double* in_s[2];
  const int* in_i[2];
  int nlists;
  double* out_s[2];
  int* out_i[2];
};

// Each of the kMergeFan input lists is sorted. They are merged pairwise in four rounds
// (16 -> 8 -> 4 -> 2 -> 1 lists), each merged list keeping its first kPMax entries: an entry's
// rank in its pair's order is its position in its own list plus the number of entries of the
// other list that come before it (a 7-step binary search). The order is strict (indices are
// distinct, padding included), so the ranks within a pair are distinct and ranks 0 .. kPMax-1
// are each written once. One thread per entry; scores and indices are kept in separate LDS
// arrays, double-buffered between rounds, and an index is read only on a tied score.
constexpr int kMergeThreads = kMergeFan * kPMax;  // 1024
template <class Src>
__global__ __launch_bounds__(kMergeThreads) void k_topk_merge(Src in) {
  const MergeArgs& a = kernel_args<MergeArgs>(in);
  if (a.st->done) return;
  const int side = blockIdx.y;
  constexpr int NE = kMergeFan * kPMax;
  __shared__ double es[2][NE];
  __shared__ int ei[2][NE];
  const int first = blockIdx.x * kMergeFan;
  const int q = threadIdx.x;
  {
    const int l = first + q / kPMax;
    double cs = kPad;
    int ci = 0x50000000 + q;  // padding entries: distinct indices, below every real entry
    if (l < a.nlists) {
      cs = a.in_s[side][(int64_t)first * kPMax + q];
      ci = a.in_i[side][(int64_t)first * kPMax + q];
      if (cs == kPad) ci = 0x50000000 + q;
    }
    es[0][q] = cs;
    ei[0][q] = ci;
  }
  __syncthreads();
  int cur = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {  // kMergeFan >> r lists of kPMax entries
    if (q < (kMergeFan >> r) * kPMax) {
      const int pr = q / (2 * kPMax), half = (q / kPMax) & 1, pos = q % kPMax;
      const int mine = (2 * pr + half) * kPMax, other = (2 * pr + (half ^ 1)) * kPMax;
      const double cs = es[cur][mine + pos];
      const int ci = ei[cur][mine + pos];
      int lo = 0, hi = kPMax;  // first position of the other list whose entry is not before c
#pragma unroll
      for (int step = 0; step < 7; ++step) {
        if (lo < hi) {
          const int mid = (lo + hi) >> 1;
          const double os = es[cur][other + mid];
          const bool bef = os > cs || (os == cs && ei[cur][other + mid] < ci);
          if (bef)
            lo = mid + 1;
          else
            hi = mid;
        }
      }
      const int rk = pos + lo;
      if (rk < kPMax) {
        es[cur ^ 1][pr * kPMax + rk] = cs;
        ei[cur ^ 1][pr * kPMax + rk] = ci;
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  if (q < kPMax) {
    a.out_s[side][(int64_t)blockIdx.x * kPMax + q] = es[cur][q];
    a.out_i[side][(int64_t)blockIdx.x * kPMax + q] = ei[cur][q];
  }
}

template <class Src>
__global__ __launch_bounds__(64) void k_select(Src in) {
  const SelectArgs& a = kernel_args<SelectArgs>(in);
  DevState* st = a.st;
  if (st->done) return;
  const int t = threadIdx.x;
  __shared__ int oldI[kPMax], oldJ[kPMax], prevI[kPMax], prevJ[kPMax], newv[2][kPMax];
  // (QDEIM reads oldI/oldJ and newv, all written before the first barrier below)
  __shared__ int pre[2][kPMax];
  __shared__ int take_s[2], nold_s[2], nv_s[2];
  __shared__ int same;
  const int nI = st->nI, nJ = st->nJ;
  const int nIprev = st->nIprev, nJprev = st->nJprev;
  const int rsig = st->r_sig;
  oldI[t] = st->I[t];
  oldJ[t] = st->J[t];
  prevI[t] = st->Iprev[t];
  prevJ[t] = st->Jprev[t];
  const double s0 = a.cs[0][t], s1 = a.cs[1][t];
  const double s0h = a.cs[0][0], s1h = a.cs[1][0];  // heads of the lists
  newv[0][t] = a.ci[0][t];
  newv[1][t] = a.ci[1][t];
  // number of valid (score >= 0) candidates: the lists are sorted, so count them
  const unsigned long long b0 = __ballot(s0 >= 0.0), b1 = __ballot(s1 >= 0.0);
  if (t == 0) {
    nv_s[0] = __popcll(b0);
    nv_s[1] = __popcll(b1);
    same = 1;
  }
  __syncthreads();
  const int kp = st->k;  // the pass being computed
  if (kp < st->replay_n) {
    // replay: the given sets are this pass's sets
    const int rn[2] = {a.replay.nI[kp], a.replay.nJ[kp]};
    for (int side = 0; side < 2; ++side) {
      if (t < rn[side]) pre[side][t] = (side == 0 ? a.replay.I : a.replay.J)[kp * kPMax + t];
      if (t == 0) {
        take_s[side] = rn[side];
        nold_s[side] = 0;
      }
    }
  } else if (a.qd) {
    // QDEIM (Algorithm 2 in Algorithm 4's selection and union): the pivots not in the old set are
    // appended in pivot order (capped at pmax); when none is new, or at the first pass, the
    // best leverage-score candidate outside the new set is appended as well (the safeguard)
    for (int side = 0; side < 2; ++side) {
      const int nold = side == 0 ? nI : nJ;
      const int* old = side == 0 ? oldI : oldJ;
      const int p = t < rsig ? a.qd[side].piv[t] : -1;
      bool isnew = t < rsig;
      for (int q = 0; q < nold; ++q) isnew &= old[q] != p;
      const unsigned long long nb = __ballot(isnew);
      const int pos = nold + __popcll(nb & ((1ull << t) - 1));
      if (isnew && pos < a.pmax) pre[side][pos] = p;
      const int cnt = min(a.pmax, nold + (int)__popcll(nb));
      __syncthreads();
      // candidate t of the leverage-score list (best first, old set excluded): usable when valid
      // and not among the new pivots
      const int cand = newv[side][t];
      bool ok = (side == 0 ? s0 : s1) >= 0.0;
      for (int q = nold; q < cnt; ++q) ok &= pre[side][q] != cand;
      const unsigned long long okb = __ballot(ok);
      const bool guard = (cnt == nold || kp == 0) && cnt < a.pmax && cnt < a.n && okb != 0ull;
      if (guard && t == __ffsll((long long)okb) - 1) pre[side][cnt] = cand;
      if (t == 0) {
        take_s[side] = cnt + (guard ? 1 : 0) - nold;
        nold_s[side] = nold;
      }
      if (t < nold) pre[side][t] = old[t];
    }
  } else {
    for (int side = 0; side < 2; ++side) {
      const int nold = side == 0 ? nI : nJ;
      int take;
      if (a.sampled) {
        // every drawn row up to the cap; if none was drawn, the safeguard's random row (the head
        // of the list, when it is a row outside the set)
        const int room = max(0, (int)min((int64_t)a.pmax, a.n) - nold);
        take = min(room, nv_s[side]);
        if (take == 0 && room > 0 && (side == 0 ? s0h : s1h) > -2.0) take = 1;
      } else {
        take = max(0, min(min(rsig, a.pmax - nold), nv_s[side]));
      }
      // the new indices in ascending order: rank among the first `take` candidates
      if (t < take) {
        const int v = newv[side][t];
        int rk = 0;
        for (int q = 0; q < take; ++q) rk += newv[side][q] < v ? 1 : 0;
        pre[side][nold + rk] = v;
      }
      if (t < nold) pre[side][t] = side == 0 ? oldI[t] : oldJ[t];
      if (t == 0) {
        take_s[side] = take;
        nold_s[side] = nold;
      }
    }
  }
  __syncthreads();
  const int nIpre = nold_s[0] + take_s[0], nJpre = nold_s[1] + take_s[1];
  // fixed point: the pass would repeat the previous cross approximation exactly
  const bool sizes_same = nIprev == nIpre && nJprev == nJpre;
  if (sizes_same) {
    if (t < nIpre && prevI[t] != pre[0][t]) same = 0;
    if (t < nJpre && prevJ[t] != pre[1][t]) same = 0;
  }
  __syncthreads();
  if (sizes_same && same) {
    if (t == 0) {
      st->done = 1;
      st->status = LRP_STAGNATED;
    }
    return;
  }
  if (t < nIpre) {
    st->Ipre[t] = pre[0][t];
    st->Iprev[t] = pre[0][t];
  }
  if (t < nJpre) {
    st->Jpre[t] = pre[1][t];
    st->Jprev[t] = pre[1][t];
  }
  a.trace.Ipre[kp * kPMax + t] = t < nIpre ? pre[0][t] : -1;
  a.trace.Jpre[kp * kPMax + t] = t < nJpre ? pre[1][t] : -1;
  if (t == 0) {
    st->nIpre = nIpre;
    st->nJpre = nJpre;
    st->nIprev = nIpre;
    st->nJprev = nJpre;
    st->ncols[0] = nJpre;
    st->ncols[1] = nIpre;
    a.trace.nIpre[kp] = nIpre;
    a.trace.nJpre[kp] = nJpre;
  }
}

// ----------------------------------------------------------------------------------------
// QDEIM: column-pivoted Householder QR of A = U(:, :r_sig)^T (r_sig x n), the first r_sig pivots
// (Algorithm 2). Column i of A is row i of U, so a thread owns one grid row and its r_sig
// entries. Step j (one launch, both sides): every row not yet pivoted applies reflector j - 1
// to its entries j-1 .. r_sig-1 and computes the squared norm of entries j .. r_sig-1 (at or
// below the noise floor: 0); the block maxima go to memory, and the block that finishes last
// picks pivot j -- among the rows within a relative 1e-12 of the largest norm, the smallest
// index, i.e. the first such row of the first block whose maximum reaches that threshold -- and
// builds reflector j from the pivot row (LAPACK convention, as in the column-pivoted QR).
constexpr int kQdRows = 256;
constexpr double kPivotTieRel = 1e-12;

struct QdeimArgs {
  const DevState* st;
  const double* U[2];
  int64_t ldu;
  int64_t n;
  int j;
  double* work[2];
  double* nrm[2];
  double* bmax[2];
  int* flag[2];
  QdeimCtl* ctl;
};

__device__ inline int block_min_int256(int x, int* scratch) {
  for (int m = 32; m >= 1; m >>= 1) x = min(x, __shfl_xor(x, m, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) scratch[w] = x;
  __syncthreads();
  const int r = min(min(scratch[0], scratch[1]), min(scratch[2], scratch[3]));
  __syncthreads();
  return r;
}

template <class Src>
__global__ __launch_bounds__(kQdRows) void k_qdeim_step(Src in) {
  const QdeimArgs& a = kernel_args<QdeimArgs>(in);
  const DevState* st = a.st;
  if (st->done) return;
  const int r = st->r_sig, j = a.j;
  if (j >= r) return;
  const int side = blockIdx.y;
  QdeimCtl* ctl = a.ctl + side;
  double* W = a.work[side];
  const int64_t n = a.n;
  __shared__ double vs[kPMax];
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ int last;
  if (threadIdx.x < kPMax) vs[threadIdx.x] = j > 0 ? ctl->v[threadIdx.x] : 0.0;
  const double tauv = j > 0 ? ctl->tau : 0.0;
  const double floor_v = j > 0 ? ctl->floor : 0.0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kQdRows + threadIdx.x;
  double nrm2 = -1.0;
  if (i < n) {
    if (j == 0) {
      const double* Ui = a.U[side] + i;
      double x[kPMax];
#pragma unroll
      for (int e = 0; e < kPMax; ++e) x[e] = e < r ? Ui[(int64_t)e * a.ldu] : 0.0;
      nrm2 = 0.0;
#pragma unroll
      for (int e = 0; e < kPMax; ++e)
        if (e < r) {
          W[i + (int64_t)e * n] = x[e];
          nrm2 = fma(x[e], x[e], nrm2);
        }
      a.flag[side][i] = 0;
    } else if (!a.flag[side][i]) {
      double x[kPMax];
#pragma unroll
      for (int e = 0; e < kPMax; ++e) x[e] = (e >= j - 1 && e < r) ? W[i + (int64_t)e * n] : 0.0;
      double d = 0.0;
#pragma unroll
      for (int e = 0; e < kPMax; ++e) d = fma(vs[e], x[e], d);
      const double w = tauv * d;
      nrm2 = 0.0;
#pragma unroll
      for (int e = 0; e < kPMax; ++e)
        if (e >= j && e < r) {
          x[e] = fma(-w, vs[e], x[e]);
          W[i + (int64_t)e * n] = x[e];
          nrm2 = fma(x[e], x[e], nrm2);
        }
      if (nrm2 <= floor_v) nrm2 = 0.0;
    }
    a.nrm[side][i] = nrm2;
  }
  const double bm = block_max256(nrm2, red);
  if (threadIdx.x == 0) a.bmax[side][blockIdx.x] = bm;
  // publish this block's results, then count it; the block that completes the count sees every
  // other block's results
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&ctl->count, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const volatile double* bmx = a.bmax[side];
  const int nb = gridDim.x;
  double best = -1.0;
  for (int q = threadIdx.x; q < nb; q += kQdRows) best = fmax(best, bmx[q]);
  best = block_max256(best, red);
  const double fl = j == 0 ? kFloorRel * best : floor_v;
  const double thr = best * (1.0 - kPivotTieRel);
  int fb = 0x7fffffff;
  for (int q = threadIdx.x; q < nb; q += kQdRows)
    if (bmx[q] >= thr) {
      fb = q;
      break;
    }
  fb = block_min_int256(fb, redi);
  const volatile double* nv = a.nrm[side];
  const int64_t row = (int64_t)fb * kQdRows + threadIdx.x;
  const int cand = (row < n && nv[row] >= thr) ? (int)threadIdx.x : 0x7fffffff;
  const int pl = block_min_int256(cand, redi);
  const int p = fb * kQdRows + pl;
  // reflector j from entries j .. r-1 of row p (wave 0, one entry per lane)
  if (threadIdx.x < 64) {
    const int e = threadIdx.x;
    const volatile double* Wp = W + p;
    const double x = (j + e < r) ? Wp[(int64_t)(j + e) * n] : 0.0;
    const double xn = sqrt(wave_sum(x * x));
    const double alpha = __shfl(x, 0, 64);
    double v = 0.0, tau = 0.0;
    if (xn != 0.0) {
      const double beta = -copysign(xn, alpha);
      v = e == 0 ? 1.0 : x / (alpha - beta);
      tau = (beta - alpha) / beta;
    }
    for (int q = e; q < kPMax; q += 64) ctl->v[q] = 0.0;
    if (j + e < r) ctl->v[j + e] = v;
    if (e == 0) {
      ctl->tau = tau;
      ctl->piv[j] = p;
      if (j == 0) ctl->floor = fl;
      a.flag[side][p] = 1;
      a.nrm[side][p] = -1.0;
      ctl->count = 0;
    }
  }
}

int qdeim_plan(QdeimPlan* p, int64_t n, hipStream_t s) {
  *p = QdeimPlan{};
  p->n = n;
  p->nblocks = (int)((n + kQdRows - 1) / kQdRows);
  for (int q = 0; q < 2; ++q) {
    if (hipMalloc(&p->work[q], sizeof(double) * (size_t)n * kPMax) != hipSuccess) return LRP_ENOMEM;
    if (hipMalloc(&p->nrm[q], sizeof(double) * (size_t)n) != hipSuccess) return LRP_ENOMEM;
    if (hipMalloc(&p->bmax[q], sizeof(double) * (size_t)p->nblocks) != hipSuccess) return LRP_ENOMEM;
    if (hipMalloc(&p->flag[q], sizeof(int) * (size_t)n) != hipSuccess) return LRP_ENOMEM;
  }
  if (hipMalloc(&p->ctl, sizeof(QdeimCtl) * 2) != hipSuccess) return LRP_ENOMEM;
  // the block counters start at 0 (on the context's stream, which is synchronized after set-up)
  return hipMemsetAsync(p->ctl, 0, sizeof(QdeimCtl) * 2, s) == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

void qdeim_free(QdeimPlan* p) {
  for (int q = 0; q < 2; ++q) {
    if (p->work[q]) (void)hipFree(p->work[q]);
    if (p->nrm[q]) (void)hipFree(p->nrm[q]);
    if (p->bmax[q]) (void)hipFree(p->bmax[q]);
    if (p->flag[q]) (void)hipFree(p->flag[q]);
  }
  if (p->ctl) (void)hipFree(p->ctl);
  *p = QdeimPlan{};
}

int qdeim_launch(const QdeimPlan& p, const DevState* st, const double* U[2], int64_t ldu, int pmax, hipStream_t s) {
  QdeimArgs a{};
  a.st = st;
  a.U[0] = U[0];
  a.U[1] = U[1];
  a.ldu = ldu;
  a.n = p.n;
  for (int q = 0; q < 2; ++q) {
    a.work[q] = p.work[q];
    a.nrm[q] = p.nrm[q];
    a.bmax[q] = p.bmax[q];
    a.flag[q] = p.flag[q];
  }
  a.ctl = p.ctl;
  for (int j = 0; j < pmax; ++j) {
    a.j = j;
    LRP_LAUNCH_G(K_QDEIM, k_qdeim_step<QdeimArgs>, k_qdeim_step<GroupRef>, dim3(p.nblocks, 2), dim3(kQdRows), 0, s, a);
  }
  return launch_status();
}

// ----------------------------------------------------------------------------------------
int select_plan(SelectPlan* p, int64_t n) {
  p->n = n;
  p->nblocks = (int)((n + kSelRows - 1) / kSelRows);
  int lists = p->nblocks;
  int L = 0;
  while (lists > 1) {
    if (L >= 8) return LRP_EINVAL;
    p->lists[L] = lists;
    lists = (lists + kMergeFan - 1) / kMergeFan;
    ++L;
  }
  p->nlevels = L;
  for (int s = 0; s < 2; ++s) {
    if (hipMalloc(&p->pi[s], sizeof(double) * n) != hipSuccess) return LRP_ENOMEM;
    if (hipMalloc(&p->bmax[s], sizeof(double) * p->nblocks) != hipSuccess) return LRP_ENOMEM;
    for (int b = 0; b < 2; ++b) {
      if (hipMalloc(&p->cand_s[b][s], sizeof(double) * p->nblocks * kPMax) != hipSuccess) return LRP_ENOMEM;
      if (hipMalloc(&p->cand_i[b][s], sizeof(int) * p->nblocks * kPMax) != hipSuccess) return LRP_ENOMEM;
    }
  }
  if (hipMalloc(&p->gmax, sizeof(double) * 2) != hipSuccess) return LRP_ENOMEM;
  return LRP_OK;
}

// Writes the final candidate lists (side 0 then 1) into cand_s/cand_i[*final_list_slot].
// The final list of side s starts at element 0 of cand_*[slot][s].
int select_candidates(const SelectPlan& p, const DevState* st, const double* U[2], int64_t ldu,
                      hipStream_t s, int* final_list_slot, SampleOpts so) {
  PiArgs pa{};
  pa.st = st;
  pa.U[0] = U[0];
  pa.U[1] = U[1];
  pa.ldu = ldu;
  pa.n = p.n;
  for (int q = 0; q < 2; ++q) {
    pa.pi[q] = p.pi[q];
    pa.bmax[q] = p.bmax[q];
  }
  LRP_LAUNCH_G(K_PI, k_pi<PiArgs>, k_pi<GroupRef>, dim3(p.nblocks, 2), dim3(256), 0, s, pa);
  GmaxArgs ga{};
  ga.st = st;
  ga.b[0] = p.bmax[0];
  ga.b[1] = p.bmax[1];
  ga.nb = p.nblocks;
  ga.gmax = p.gmax;
  LRP_LAUNCH_G(K_GMAX, k_gmax<GmaxArgs>, k_gmax<GroupRef>, dim3(2), dim3(256), 0, s, ga);
  TopkArgs ta{};
  ta.st = st;
  ta.pi[0] = p.pi[0];
  ta.pi[1] = p.pi[1];
  ta.gmax = p.gmax;
  ta.n = p.n;
  ta.sampled = so.sampled;
  ta.rho = so.rho;
  ta.seed = so.seed;
  for (int q = 0; q < 2; ++q) {
    ta.cs[q] = p.cand_s[0][q];
    ta.ci[q] = p.cand_i[0][q];
  }
  LRP_LAUNCH_G(K_TOPK_BLOCK, k_topk_block<TopkArgs>, k_topk_block<GroupRef>, dim3(p.nblocks, 2), dim3(256), 0, s, ta);
  int slot = 0;
  for (int L = 0; L < p.nlevels; ++L) {
    const int lists = p.lists[L];
    const int outl = (lists + kMergeFan - 1) / kMergeFan;
    MergeArgs ma{};
    ma.st = st;
    ma.nlists = lists;
    for (int q = 0; q < 2; ++q) {
      ma.in_s[q] = p.cand_s[slot][q];
      ma.in_i[q] = p.cand_i[slot][q];
      ma.out_s[q] = p.cand_s[slot ^ 1][q];
      ma.out_i[q] = p.cand_i[slot ^ 1][q];
    }
    LRP_LAUNCH_G(K_TOPK_MERGE, k_topk_merge<MergeArgs>, k_topk_merge<GroupRef>, dim3(outl, 2), dim3(kMergeThreads), 0, s, ma);
    slot ^= 1;
  }
  *final_list_slot = slot;
  return launch_status();
}

int select_update(const SelectArgs& a, hipStream_t s) {
  LRP_LAUNCH_G(K_SELECT, k_select<SelectArgs>, k_select<GroupRef>, dim3(1), dim3(kPMax), 0, s, a);
  return launch_status();
}

}  // namespace lrp
