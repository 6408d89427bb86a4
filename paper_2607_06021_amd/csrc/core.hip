// The small dense steps of one Cross-DEIM pass, on one workgroup (paper, Algorithm 1
// after the QRs, and Algorithm 4's pruning and stopping test):
//   * with A = Q(I,:) (|J| <= |I|) or A = Z(J,:) (otherwise), the least-squares solve of
//     Algorithm 1 through A's pseudo-inverse. A Householder QR A = Q2 R gives
//     A^+ = R^{-1} Q2^T whenever no singular value of A can fall at or below the cutoff
//     max(rows, cols) eps sigma_1 -- guaranteed when 4 cutoff ||R||_F ||R^{-1}||_F < 1, since
//     sigma_min >= 1/||R^{-1}||_F and sigma_1 <= ||R||_F. Otherwise A^+ comes from a one-sided
//     Jacobi SVD with that cutoff;
//   * the |J| x |I| core M = Q(I,:)^+ R_R^T, or M = R_C (Z(J,:)^+)^T, so that the cross
//     approximation is Q M Z^T;
//   * the SVD of M = U^ S V~^T by one-sided Jacobi, truncated at max(|I|, |J|) eps sigma_1
//     (U_k = Q U^ and V_k = Z V~ are formed by the product kernel);
//   * pruning: index l of I (of J) is dropped when |diag R_R| (|diag R_C|) at l is below
//     tau times its largest entry;
//   * the cheap bound 2 S_min / ||S||_F < eps that the indicator
//     min(eta_1 (1 + eta_2), eta_2 (1 + eta_1)) S_min / ||S||_F must pass for a stop; the
//     indicator itself (eta_1 = 1/sigma_min(U_k(I,:)), eta_2 = 1/sigma_min(V_k(J,:)) on the
//     pruned sets, two Jacobi problems solved side by side) and the stop decision are made by
//     k_eta once rho is known, and only when a stop is possible.
// The warm start uses the same SVD on M = R_u R_v^T, the core of F^ = U^ V^^T.
//
// Jacobi: Hestenes' one-sided method; a pair is rotated unless
// |a_p . a_q| <= sqrt(m) eps ||a_p|| ||a_q||, and the sweeps end after one whose rotations all
// had |a_p . a_q| <= 1e-8 ||a_p|| ||a_q|| (at most 60): convergence is quadratic by then, so the
// next sweep would find the pairs at about 1e-16, at the rotation threshold, and change nothing
// beyond rounding. Every sweep visits each column pair once, in an order built for wavefronts (see
// jacobi_waves): each wave keeps 8 columns in registers for 4 rounds at a time.
#include "lrp_kernels.h"

namespace lrp {

constexpr int LDP = kPMax + 1;        // padded leading dimension of the LDS matrices
constexpr int kCoreThreads = 512;
constexpr int kEtaThreads = 512;  // one Jacobi problem of up to 8 waves per workgroup
constexpr int kBuf = kPMax * LDP;

// ---------------------------------------------------------------- lane-group sums (DPP)
__device__ inline double dpp_d(double x, int ctrl) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  switch (ctrl) {  // the control word must be a compile-time constant
    case 0xB1:
      lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
      break;
    case 0x4E:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
      break;
    case 0x141:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
      break;
  }
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G lanes (G = 4, 8 or 16); every lane gets its group's total.
template <int G>
__device__ inline double group_sum(double x) {
  x += dpp_d(x, 0xB1);    // quad_perm [1,0,3,2]
  x += dpp_d(x, 0x4E);    // quad_perm [2,3,0,1]
  if (G >= 8) x += dpp_d(x, 0x141);   // row_half_mirror: the other quad of the octet
  if (G >= 16) x += dpp_d(x, 0x140);  // row_mirror: the other octet of the row
  return x;
}

// ---------------------------------------------------------------- one-sided Jacobi
struct JacProb {
  double* A;  // m x k, column-major, ld LDP (LDS)
  int m, k;
  double* V;  // k x k accumulated rotations (holding the identity on entry), or null
};

// Rotation (c, s) that makes columns p, q orthogonal: with al = |a_p|^2, be = |a_q|^2,
// ga = a_p . a_q, d = be - al, h = sqrt(d^2 + 4ga^2) and u = h + |d|, Rutishauser's smaller
// root t = sign(d) 2ga / u gives c = 1/sqrt(1 + t^2) = u / sqrt(2hu) and
// s = c t = sign(d) 2ga / sqrt(2hu) (u^2 + 4ga^2 = 2hu), so c^2 + s^2 = 1 holds by construction
// and no quotient has to be formed.
__device__ inline void jacobi_rotation(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, g2 = 2.0 * ga;
  const double h2 = fma(d, d, g2 * g2);
  if (h2 > 1e-290 && h2 < 1e290) {
    const double h = h2 * rsq_nr(h2);
    const double u = h + fabs(d);
    const double r = rsq_nr(2.0 * h * u);
    c = u * r;
    s = copysign(1.0, d) * g2 * r;
  } else {  // extreme magnitudes: the correctly rounded library operations
    const double zeta = d / g2;
    const double t =
        fabs(zeta) > 1e150 ? 0.5 / zeta : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    c = 1.0 / sqrt(1.0 + t * t);
    s = c * t;
  }
}

// Column pair of pair slot pi in round rd of the round-robin ordering of kk (even) columns:
// slot 0 pairs the fixed column kk-1 with rd, slot pi > 0 pairs rd+pi and rd-pi (mod kk-1).
__device__ inline void rr_pair(int kk, int pi, int rd, int& p, int& q) {
  const int n1 = kk - 1;
  if (pi == 0) {
    p = n1;
    q = rd;
  } else {
    p = rd + pi;
    if (p >= n1) p -= n1;
    q = rd - pi;
    if (q < 0) q += n1;
  }
  if (p > q) {
    const int tmp = p;
    p = q;
    q = tmp;
  }
}

// Value of x held by lane src of the wave (ds_bpermute moves 32 bits per lane).
__device__ inline double lane_fetch(double x, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Column groups of 4 for a k-column problem: an even count >= 2 (columns past k are empty).
__device__ inline int jac_groups(int k) {
  int g = (k + 3) >> 2;
  g += g & 1;
  return g < 2 ? 2 : g;
}

// One Jacobi pair step on the 16 lanes of a pair slot: lane li holds rows li + 16u (u < 4)
// of the two columns (a, b) and of their V columns; rows past m (or k for V) are zero, and so is
// an empty column, which is never rotated (its dot products vanish).
constexpr double kJacQuiet2 = 1e-16;  // (1e-8)^2: a rotation below this leaves the next sweep idle

template <bool WV>
__device__ inline bool jac_pair(double (&a)[4], double (&b)[4], double (&va)[4], double (&vb)[4], double tol2,
                                bool& loud) {
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    al = fma(a[u], a[u], al);
    be = fma(b[u], b[u], be);
    ga = fma(a[u], b[u], ga);
  }
  al = group_sum<16>(al);
  be = group_sum<16>(be);
  ga = group_sum<16>(ga);
  const bool rot = ga != 0.0 && ga * ga > tol2 * al * be;
  loud |= rot && ga * ga > kJacQuiet2 * al * be;
  // Straight-line rotation for every slot (slots that do not rotate take c = 1, s = 0, which
  // leaves the values of their columns unchanged); the extreme-range formula is a rare branch.
  const double d = be - al, g2 = 2.0 * ga;
  const double h2 = fma(d, d, g2 * g2);
  const double h = h2 * rsq_nr(h2);
  const double uu = h + fabs(d);
  const double rr = rsq_nr(2.0 * h * uu);
  double c = uu * rr, sn = copysign(1.0, d) * g2 * rr;
  if (rot && !(h2 > 1e-290 && h2 < 1e290)) jacobi_rotation(al, be, ga, c, sn);
  c = rot ? c : 1.0;
  sn = rot ? sn : 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double x = a[u], y = b[u];
    a[u] = c * x - sn * y;
    b[u] = sn * x + c * y;
  }
  if (WV) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double x = va[u], y = vb[u];
      va[u] = c * x - sn * y;
      vb[u] = sn * x + c * y;
    }
  }
  return rot;
}

// The second columns of every slot (and their V columns) move to the slot of lane ^ xmask.
template <bool WV>
__device__ inline void jac_move_b(double (&b)[4], double (&vb)[4], int src) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    b[u] = lane_fetch(b[u], src);
    if (WV) vb[u] = lane_fetch(vb[u], src);
  }
}

// Column col (into x, vx) from LDS, zero past the problem. Every address lies in the 64 x LDP
// buffer (col < 64, rows < 64), so all loads are issued unconditionally and the entries outside
// the problem are replaced afterwards; the empty asm statements keep the selects from being
// turned back into branches around single loads.
template <bool WV>
__device__ inline void jac_load(const JacProb& pr, int col, int li, double (&x)[4], double (&vx)[4]) {
  const bool ok = col < pr.k;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    x[u] = pr.A[li + 16 * u + col * LDP];
    if (WV) vx[u] = pr.V[li + 16 * u + col * LDP];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = li + 16 * u;
    asm volatile("" : "+v"(x[u]));
    x[u] = (ok && i < pr.m) ? x[u] : 0.0;
    if (WV) {
      asm volatile("" : "+v"(vx[u]));
      vx[u] = (ok && i < pr.k) ? vx[u] : 0.0;
    }
  }
}

template <bool WV>
__device__ inline void jac_store(const JacProb& pr, int col, int li, const double (&x)[4], const double (&vx)[4]) {
  if (col >= pr.k) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = li + 16 * u;
    if (i < pr.m) pr.A[i + col * LDP] = x[u];
    if (WV && i < pr.k) pr.V[i + col * LDP] = vx[u];
  }
}

// Solve one or two independent Jacobi problems (A: m x k in LDS, m, k <= 64; V: the k x k
// accumulated rotations, holding the identity on entry, or null for none) with the workgroup:
// problem q runs on waves 8q .. 8q+7 (blockDim.x >= 512 nprob). flags: 2 ints of LDS.
//
// The k columns are split into NG groups of 4 (NG even, columns past k empty). A sweep is
//   * NG - 1 group rounds: the round-robin (circle) schedule over the groups gives wave w the
//     group pair (g, h); the wave loads the 8 columns into registers -- pair slot i (lanes
//     16i .. 16i+15) takes columns 4g + i and 4h + i -- and runs 4 rounds pairing 4g + i with
//     4h + (i ^ s), s = 0, 1, 3, 2, the second columns moving between slots by lane permutes,
//     then stores them back (one workgroup barrier per group round);
//   * an intra-group phase: wave w takes groups 2w and 2w+1 and pairs the 4 columns of each in 3
//     rounds ((0,1)(2,3), (0,2)(1,3), (0,3)(1,2)).
// Every column pair is visited once per sweep, no two pairs of a round share a column, and no
// barrier is needed inside a group round.
template <bool WV>
__device__ int jacobi_waves(JacProb* P, int nprob, int* flags) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int q = (nprob == 2 && wv >= 8) ? 1 : 0;
  const int lw = wv - 8 * q;
  const JacProb pr = P[q];
  const int slot = lane >> 4, li = lane & 15;
  int ngmax = 0, kmax = 0;
  for (int x = 0; x < nprob; ++x) {
    kmax = max(kmax, P[x].k);
    ngmax = max(ngmax, jac_groups(P[x].k));
  }
  if (kmax < 2) {
    __syncthreads();
    return 0;
  }
  const int ng = jac_groups(pr.k);
  const bool mine = pr.k >= 2 && lw < (ng >> 1) && (nprob == 2 || wv < 8);
  const double tol = sqrt((double)max(pr.m, 1)) * kEps;
  const double tol2 = tol * tol;
  double a[4], b[4], va[4], vb[4];
  bool active = true;  // this problem's last sweep made a rotation above the quiet level
  int sweeps = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    sweeps = sweep + 1;
    if (t < 2) flags[t] = 0;
    __syncthreads();
    bool loud = false;
    for (int gr = 0; gr < ngmax - 1; ++gr) {
      if (active && mine && gr < ng - 1) {
        int g, h;
        rr_pair(ng, lw, gr, g, h);
        jac_load<WV>(pr, 4 * g + slot, li, a, va);
        jac_load<WV>(pr, 4 * h + slot, li, b, vb);
        jac_pair<WV>(a, b, va, vb, tol2, loud);  // s = 0
        jac_move_b<WV>(b, vb, lane ^ 16);
        jac_pair<WV>(a, b, va, vb, tol2, loud);  // s = 1
        jac_move_b<WV>(b, vb, lane ^ 32);
        jac_pair<WV>(a, b, va, vb, tol2, loud);  // s = 3
        jac_move_b<WV>(b, vb, lane ^ 16);
        jac_pair<WV>(a, b, va, vb, tol2, loud);  // s = 2
        jac_store<WV>(pr, 4 * g + slot, li, a, va);
        jac_store<WV>(pr, 4 * h + (slot ^ 2), li, b, vb);
      }
      __syncthreads();
    }
    if (active && mine) {
      const int c0 = 4 * (2 * lw + (slot >> 1));
      const bool odd = slot & 1;
      jac_load<WV>(pr, c0 + (odd ? 2 : 0), li, a, va);
      jac_load<WV>(pr, c0 + (odd ? 3 : 1), li, b, vb);
      jac_pair<WV>(a, b, va, vb, tol2, loud);  // (0,1) (2,3)
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // even slot: b <- partner's a; odd slot: a <- partner's b
        const double ta = lane_fetch(a[u], lane ^ 16), tb = lane_fetch(b[u], lane ^ 16);
        if (odd)
          a[u] = tb;
        else
          b[u] = ta;
        if (WV) {
          const double tva = lane_fetch(va[u], lane ^ 16), tvb = lane_fetch(vb[u], lane ^ 16);
          if (odd)
            va[u] = tvb;
          else
            vb[u] = tva;
        }
      }
      jac_pair<WV>(a, b, va, vb, tol2, loud);  // (0,2) (1,3)
      jac_move_b<WV>(b, vb, lane ^ 16);
      jac_pair<WV>(a, b, va, vb, tol2, loud);  // (0,3) (1,2)
      jac_store<WV>(pr, c0 + (odd ? 1 : 0), li, a, va);
      jac_store<WV>(pr, c0 + (odd ? 2 : 3), li, b, vb);
    }
    if (loud) flags[q] = 1;
    __syncthreads();
    const bool any0 = flags[0] != 0, any1 = flags[1] != 0;
    active = q == 0 ? any0 : any1;
    const bool more = any0 || (nprob == 2 && any1);
    __syncthreads();
    if (!more) break;
  }
  return sweeps;
}

// Returns the number of sweeps made (the last one made no rotation above the quiet level).
__device__ int jacobi(JacProb* P, int nprob, int* flags) {
  bool wv = false;
  for (int x = 0; x < nprob; ++x) wv |= P[x].V != nullptr;
  if (wv) return jacobi_waves<true>(P, nprob, flags);
  return jacobi_waves<false>(P, nprob, flags);
}

// sig[c] = ||A(:, c)||, ord[r] = column of rank r (descending, ties to the smaller index).
__device__ void norms_sorted(const double* A, int m, int k, double* sig, int* ord) {
  const int t = threadIdx.x;
  if (t < k) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(A[i + t * LDP], A[i + t * LDP], s);
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
  for (int e = threadIdx.x; e < k * LDP; e += blockDim.x) {
    const int i = e % LDP, j = e / LDP;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// An empty asm statement taking a loaded value as input and output: the load completes before
// it unconditionally, so a following select cannot become a branch around the load.
__device__ inline void pin(double& v) { asm volatile("" : "+v"(v)); }

// C = A B for 64 x 64 matrices in LDS (column-major, ld LDP, zero outside the used m x k and
// k x n parts) on the FP64 matrix cores (v_mfma_f64_16x16x4: operand A lane l = A(l%16, l/16),
// B lane l = B(l/16, l%16), result item v = C(l/16 + 4v, l%16)): the 16 tiles of 16 x 16 go
// round the waves of the workgroup. C(i, j), i < m, j < n, is stored at C[i + j LDP], or at
// C[j + i LDP] when trans. C must not overlap A or B.
__device__ void lds_gemm(const double* A, const double* B, double* C, int m, int n, bool trans) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  for (int q = wave; q < 16; q += nw) {
    const int I = q >> 2, J = q & 3;
    if (16 * I >= m || 16 * J >= n) continue;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[16 * I + lr + (4 * ks + lk) * LDP],
                                                  B[4 * ks + lk + (16 * J + lr) * LDP], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * I + lk + 4 * v, j = 16 * J + lr;
      if (i < m && j < n) C[trans ? j + i * LDP : i + j * LDP] = acc[v];
    }
  }
}

// Q(idx[i], c) for i < m, c < k into S (64 x 64, ld LDP, zero elsewhere); Q column-major with
// leading dimension ldq. Every load reads a valid element and the loads of a thread are in
// flight together.
__device__ void gather_rows(const double* Q, int64_t ldq, const int* idx, int m, int k, double* S) {
  for (int base = threadIdx.x; base < kPMax * kPMax; base += blockDim.x * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * blockDim.x, i = e % kPMax, c = e / kPMax;
      const int ii = min(i, max(m - 1, 0)), cc = min(c, max(k - 1, 0));
      v[u] = (e < kPMax * kPMax && m > 0 && k > 0) ? Q[idx[ii] + (int64_t)cc * ldq] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * blockDim.x, i = e % kPMax, c = e / kPMax;
      pin(v[u]);
      if (e < kPMax * kPMax) S[i + c * LDP] = (i < m && c < k) ? v[u] : 0.0;
    }
  }
}

// B(r, c) = F[r + c ldf] for r < m, c < k into S (64 x 64, ld LDP, zero elsewhere).
__device__ void load_block(const double* F, int64_t ldf, int m, int k, double* S) {
  for (int base = threadIdx.x; base < kPMax * kPMax; base += blockDim.x * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * blockDim.x, i = e % kPMax, c = e / kPMax;
      const int ii = min(i, max(m - 1, 0)), cc = min(c, max(k - 1, 0));
      v[u] = (e < kPMax * kPMax && m > 0 && k > 0) ? F[ii + (int64_t)cc * ldf] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * blockDim.x, i = e % kPMax, c = e / kPMax;
      pin(v[u]);
      if (e < kPMax * kPMax) S[i + c * LDP] = (i < m && c < k) ? v[u] : 0.0;
    }
  }
}

// ---------------------------------------------------------------- small Householder QR
// The small dense routines below keep one column per 8 lanes (rows li + 8u, u < 8, in
// registers; with 512 threads the 64 columns are covered in one pass).

// x[u] for a u that is the same on every active lane (a scalar branch, not a select chain).
__device__ inline double pick8(const double (&x)[8], int u) {
  switch (u & 7) {
    case 0: return x[0];
    case 1: return x[1];
    case 2: return x[2];
    case 3: return x[3];
    case 4: return x[4];
    case 5: return x[5];
    case 6: return x[6];
    default: return x[7];
  }
}

// In place on A (m x k, m >= k, ld LDP): R in the upper triangle, the reflectors' tails below
// (LAPACK convention: beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta, v = x/(alpha - beta),
// v_j = 1 implicit), tau[j] in LDS. Column j builds its reflector from its registers (tau =
// 1 + |alpha|/h and 1/(alpha - beta) = sign(alpha)/(|alpha| + h) with h = ||x||, one rsq and one
// rcp), publishes it in LDS (vb: 2 x 64 doubles, double-buffered) and after one barrier every
// trailing column applies it. blockDim.x >= 512.
__device__ void small_qr(double* A, int m, int k, double* tau, double* vb) {
  const int t = threadIdx.x, c = t >> 3, li = t & 7;
  const bool col = c < k;
  double x[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = li + 8 * u;
    x[u] = (col && i < m) ? A[i + c * LDP] : 0.0;
  }
  double rdiag = 0.0, vscale = 0.0;
  for (int j = 0; j < k; ++j) {
    double* vj = vb + (j & 1) * kPMax;
    if (c == j) {
      double y[8], n[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        y[u] = li + 8 * u > j ? x[u] : 0.0;
        n[u & 3] = fma(y[u], y[u], n[u & 3]);
      }
      const double xnorm2 = oct_sum((n[0] + n[1]) + (n[2] + n[3]));
      const double xj = pick8(x, j >> 3);
      const int src = ((j & 7) << 3) + (j & 7);  // lane of row j within column j's octet
      const double alpha = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(xj), src),
                                            __builtin_amdgcn_readlane(__double2loint(xj), src)) +
                           0.0;
      const double h2 = fma(alpha, alpha, xnorm2);
      const double rh = rsq_nr(h2);
      const double h = h2 * rh;
      double beta = -copysign(h, alpha);
      double tj = fma(fabs(alpha), rh, 1.0);
      double scale = copysign(rcp_nr(fabs(alpha) + h), alpha);
      if (xnorm2 == 0.0) {
        tj = 0.0;
        beta = alpha;
        scale = 0.0;
      } else if (!(h2 > 1e-290 && h2 < 1e290)) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) vj[li + 8 * u] = y[u] * scale;
      if (li == (j & 7)) vj[j] = 1.0;  // same lane, after its zero: in order
      rdiag = beta;
      vscale = scale;
      if (li == 0) tau[j] = tj;
    }
    __syncthreads();
    if (c > j && col) {
      double v[8], d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = vj[li + 8 * u];
        d[u & 3] = fma(v[u], x[u], d[u & 3]);
      }
      const double w = oct_sum((d[0] + d[1]) + (d[2] + d[3])) * tau[j];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = fma(-w, v[u], x[u]);
    }
  }
  if (col) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = li + 8 * u;
      if (i < m) A[i + c * LDP] = i < c ? x[u] : (i == c ? rdiag : x[u] * vscale);
    }
  }
  __syncthreads();
}

// B (m x ncols, ld LDP) <- H_{k-1} .. H_0 B (Q2-full^T B) if transpose, else H_0 .. H_{k-1} B,
// with V holding the reflectors explicitly (unit diagonal, zeros above and below row m - 1: see
// explicit_reflectors). Every column runs through the k reflectors on its own lanes.
__device__ void apply_reflectors(const double* V, const double* tau, int m, int k, double* B, int ncols,
                                 bool transpose) {
  const int t = threadIdx.x, li = t & 7;
  for (int c = t >> 3; c < ncols; c += blockDim.x >> 3) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = li + 8 * u;
      x[u] = i < m ? B[i + c * LDP] : 0.0;
    }
    for (int s = 0; s < k; ++s) {
      const int j = transpose ? s : k - 1 - s;
      const double* vj = V + j * LDP + li;
      double v[8], d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = vj[8 * u];
        d[u & 3] = fma(v[u], x[u], d[u & 3]);
      }
      const double w = oct_sum((d[0] + d[1]) + (d[2] + d[3])) * tau[j];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = fma(-w, v[u], x[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = li + 8 * u;
      if (i < m) B[i + c * LDP] = x[u];
    }
  }
  __syncthreads();
}

// Overwrites the R part of a small_qr result with the explicit reflectors: 1 on the diagonal,
// 0 above it and below row m - 1 (all 64 x 64 entries written).
__device__ void explicit_reflectors(double* QR, int m, int k) {
  for (int e = threadIdx.x; e < kPMax * kPMax; e += blockDim.x) {
    const int i = e % kPMax, j = e / kPMax;
    if (i <= j || i >= m || j >= k) QR[i + j * LDP] = (i == j && j < k) ? 1.0 : 0.0;
  }
  __syncthreads();
}

// Ri <- R^{-1} for the k x k upper triangle of QR, zero elsewhere in 64 x 64, by back
// substitution on R X = I in 16-row blocks from the bottom (dinv: kPMax doubles of LDS, the
// diagonal reciprocals). In block b, wave 0 solves the block's triangle with a lane per column
// (the 16 rows in registers, updated right-looking after each row: one multiply and one fma per
// row on the dependent chain); then the waves update the rows above the block,
// X(0:16b, :) -= R(0:16b, block) X(block, :), as 16 x 16 MFMA tiles. Only the strict upper
// triangle of QR is read (the reflector tails below it are not), and QR is zero past column k.
__device__ __forceinline__ void tri_inverse(const double* QR, int k, double* Ri, double* dinv) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (t < kPMax) dinv[t] = t < k ? 1.0 / QR[t + t * LDP] : 0.0;
  for (int e = t; e < kPMax * kPMax; e += blockDim.x) {
    const int i = e % kPMax, j = e / kPMax;
    Ri[i + j * LDP] = (i == j && i < k) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int pt = (k + 15) >> 4;
  for (int b = pt - 1; b >= 0; --b) {  // uniform
    const int r0 = 16 * b;
    if (wave == 0) {
      double x[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) x[w] = Ri[(r0 + w) + lane * LDP];
#pragma unroll
      for (int w = 15; w >= 0; --w) {
        const double z = dinv[r0 + w] * x[w];  // zero past k
        Ri[(r0 + w) + lane * LDP] = z;
#pragma unroll
        for (int w2 = 0; w2 < w; ++w2) x[w2] = fma(-QR[(r0 + w2) + (r0 + w) * LDP], z, x[w2]);
      }
    }
    __syncthreads();
    if (b == 0) break;
    for (int q = wave; q < b * pt; q += nw) {  // tile (I, J): rows 16 I of X, columns 16 J
      const int I = q / pt, J = q % pt;
      f64x4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = Ri[(16 * I + lk + 4 * v) + (16 * J + lr) * LDP];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-QR[(16 * I + lr) + (r0 + 4 * kk + lk) * LDP],
                                                   Ri[(r0 + 4 * kk + lk) + (16 * J + lr) * LDP], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) Ri[(16 * I + lk + 4 * v) + (16 * J + lr) * LDP] = acc[v];
    }
    __syncthreads();
  }
}

// Frobenius norms of the upper triangle of QR (k x k) and of Ri: into out[0], out[1].
__device__ void tri_norms(const double* QR, const double* Ri, int k, double* red, double* out) {
  double a = 0.0, b = 0.0;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    if (i <= j) {
      a = fma(QR[i + j * LDP], QR[i + j * LDP], a);
      b = fma(Ri[i + j * LDP], Ri[i + j * LDP], b);
    }
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[8 + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < kCoreThreads / 64; ++q) {
      sa += red[q];
      sb += red[8 + q];
    }
    out[0] = sqrt(sa);
    out[1] = sqrt(sb);
  }
  __syncthreads();
}

// Truncated SVD of M (nJ x nI, ld LDP, in Mb), QR-preconditioned one-sided Jacobi: with X = M
// (nJ >= nI) or M^T, m x k, X = Q R (small_qr) and Jacobi on R^T (R^T V = W, orthogonal columns
// W_c = sigma_c w_c) gives X = (Q V) Sigma W'^T, W' = W Sigma^{-1}: the left singular vectors of X
// are Q V (reflectors applied to [V; 0]) and the right ones the normalized columns of W. Jacobi on
// the triangular factor of a graded matrix needs far fewer sweeps than on the matrix itself.
// Columns are sorted by singular value (ties to the smaller index) and truncated at
// cut_mult eps sigma_1. Outputs: U^ (nJ x r) in Cb, V~ (nI x r) in Xb; returns r and the Jacobi
// sweeps in *sweeps. Mb, Xb, Vq, Cb are distinct 64 x 64 LDS buffers (Mb, Vq are overwritten);
// tau: kPMax, vbq: 2 kPMax doubles.
__device__ __forceinline__ int svd_qr(double* Mb, int nJ, int nI, double cut_mult, double* Xb, double* Vq, double* Cb,
                      double* tau, double* vbq, double* sig, int* ord, int* flags, int* sweeps) {
  const int t = threadIdx.x;
  const bool tall = nJ >= nI;
  const int m = tall ? nJ : nI, k = tall ? nI : nJ;
  for (int e = t; e < kPMax * kPMax; e += blockDim.x) {  // X, zero-padded
    const int i = e % kPMax, j = e / kPMax;
    Xb[i + j * LDP] = (i < m && j < k) ? (tall ? Mb[i + j * LDP] : Mb[j + i * LDP]) : 0.0;
  }
  __syncthreads();
  small_qr(Xb, m, k, tau, vbq);
  for (int e = t; e < kPMax * kPMax; e += blockDim.x) {  // R^T into Mb, identity into Vq
    const int i = e % kPMax, j = e / kPMax;
    Mb[i + j * LDP] = (i < k && j <= i) ? Xb[j + i * LDP] : 0.0;
    Vq[i + j * LDP] = (i == j && i < k) ? 1.0 : 0.0;
  }
  __syncthreads();
  JacProb pr{Mb, k, k, Vq};
  *sweeps = jacobi(&pr, 1, flags);
  norms_sorted(Mb, k, k, sig, ord);
  const double smax = k > 0 ? sig[ord[0]] : 0.0;
  int r = 0;
  if (smax > 0.0) {
    const double cut = cut_mult * kEps * smax;
    for (int c = 0; c < k; ++c) r += sig[ord[c]] > cut ? 1 : 0;
  }
  explicit_reflectors(Xb, m, k);
  apply_reflectors(Xb, tau, m, k, Vq, k, false);  // Vq <- Q [V; 0]
  for (int e = t; e < r * kPMax; e += blockDim.x) {
    const int i = e % kPMax, rr = e / kPMax;
    const int c = ord[rr];
    const double inv = 1.0 / sig[c];
    const double left = i < m ? Vq[i + c * LDP] : 0.0;
    const double right = i < k ? Mb[i + c * LDP] * inv : 0.0;
    Cb[i + rr * LDP] = tall ? left : right;
    Xb[i + rr * LDP] = tall ? right : left;
  }
  __syncthreads();
  return r;
}

template <class Src>
__global__ __launch_bounds__(kCoreThreads) void k_core(Src in) {
  const CoreArgs& a = kernel_args<CoreArgs>(in);
  DevState* st = a.st;
  if (st->done) return;
  __shared__ double B0[kBuf], B1[kBuf], B2[kBuf], B3[kBuf];
  __shared__ double sig[kPMax], tau[kPMax], red[16], nrm2[2], vbq[2 * kPMax], dinv[kPMax];
  __shared__ int ord[kPMax], flags[2], posI[kPMax], posJ[kPMax], cnt[2], idxI[kPMax], idxJ[kPMax];
  const int t = threadIdx.x;
  const int nI = st->nIpre, nJ = st->nJpre;
  const int pm = a.pmax;
  const double* R_C = a.R0;  // nJ x nJ upper triangular, ld pm
  const double* R_R = a.R1;  // nI x nI
  const double cut_pinv = (double)max(nI, nJ);
  if (t < kPMax) {
    idxI[t] = t < nI ? st->Ipre[t] : 0;
    idxJ[t] = t < nJ ? st->Jpre[t] : 0;
  }
  __syncthreads();

  // ---- the core M = A^+ R_R^T (|J| <= |I|, A = Q(I,:)) or R_C (A^+)^T (A = Z(J,:))
  const bool branch = nJ <= nI;
  const int m0 = branch ? nI : nJ, k0 = branch ? nJ : nI;
  gather_rows(branch ? a.Q0 : a.Q1, a.ldq, branch ? idxI : idxJ, m0, k0, B0);  // zero-padded
  __syncthreads();
  small_qr(B0, m0, k0, tau, vbq);
  tri_inverse(B0, k0, B1, dinv);  // B1 = R^{-1}, zero-padded
  tri_norms(B0, B1, k0, red, nrm2);
  const double bound = nrm2[0] * nrm2[1] * cut_pinv * kEps * 4.0;
  double* M;
  const bool qr_route = bound < 1.0;
  if (qr_route) {
    // With A = Q(I,:) and R_m = R_R (|J| <= |I|) the core is M = A^+ R_m^T; with A = Z(J,:) and
    // R_m = R_C it is M = R_C (A^+)^T, i.e. M^T = A^+ R_m^T: the same product, stored
    // transposed. A^+ R_m^T = R^{-1} (H^T R_m^T)(0:k0, :), H the QR's reflectors.
    const double* Rm = branch ? R_R : R_C;  // m0 x m0 upper triangular, ld pm
    explicit_reflectors(B0, m0, k0);
    load_block(Rm, pm, m0, m0, B3);
    __syncthreads();
    for (int e = t; e < kPMax * kPMax; e += blockDim.x) {  // B2 = R_m^T, zero-padded
      const int i = e % kPMax, j = e / kPMax;
      B2[i + j * LDP] = (j <= i) ? B3[j + i * LDP] : 0.0;
    }
    __syncthreads();
    apply_reflectors(B0, tau, m0, k0, B2, m0, true);
    lds_gemm(B1, B2, B3, k0, m0, !branch);  // k0 x m0 product: M, or M^T stored transposed
    __syncthreads();
    M = B3;
  } else {
    // A may have singular values at or below the cutoff: Jacobi pseudo-inverse.
    gather_rows(branch ? a.Q0 : a.Q1, a.ldq, branch ? idxI : idxJ, m0, k0, B0);
    set_identity(B1, k0);
    __syncthreads();
    JacProb pr{B0, m0, k0, B1};
    jacobi(&pr, 1, flags);
    norms_sorted(B0, m0, k0, sig, ord);
    const double smax = sig[ord[0]];
    const double cut = cut_pinv * kEps * smax;
    for (int e = t; e < m0 * k0; e += blockDim.x) {  // U_c / s_c = X_c / s_c^2, dropped -> 0
      const int i = e % m0, c = e / m0;
      const double s = sig[c];
      B0[i + c * LDP] = (smax > 0.0 && s > cut) ? B0[i + c * LDP] / (s * s) : 0.0;
    }
    __syncthreads();
    if (branch) {
      // A^+ = B1 Xs^T; M = B1 (Xs^T R_R^T): B2(c, j) = sum_i Xs(i, c) R_R(j, i)
      for (int e = t; e < nJ * nI; e += blockDim.x) {
        const int c = e % nJ, j = e / nJ;
        double s = 0.0;
        for (int i = j; i < nI; ++i) s = fma(B0[i + c * LDP], R_R[j + (int64_t)i * pm], s);
        B2[c + j * LDP] = s;
      }
      __syncthreads();
      for (int e = t; e < nJ * nI; e += blockDim.x) {
        const int aa = e % nJ, j = e / nJ;
        double s = 0.0;
        for (int c = 0; c < nJ; ++c) s = fma(B1[aa + c * LDP], B2[c + j * LDP], s);
        B3[aa + j * LDP] = s;
      }
    } else {
      // (A^+)^T = Xs B1^T; M = R_C Xs B1^T
      for (int e = t; e < nJ * nI; e += blockDim.x) {
        const int aa = e % nJ, c = e / nJ;
        double s = 0.0;
        for (int l = aa; l < nJ; ++l) s = fma(R_C[aa + (int64_t)l * pm], B0[l + c * LDP], s);
        B2[aa + c * LDP] = s;
      }
      __syncthreads();
      for (int e = t; e < nJ * nI; e += blockDim.x) {
        const int aa = e % nJ, j = e / nJ;
        double s = 0.0;
        for (int c = 0; c < nI; ++c) s = fma(B2[aa + c * LDP], B1[j + c * LDP], s);
        B3[aa + j * LDP] = s;
      }
    }
    __syncthreads();
    M = B3;
  }

  // ---- truncated SVD of the core (M is B3): U^ -> B2, V~ -> B0
  double* Ub = B2;
  double* Vb = B0;
  int sweeps = 0;
  const int r = svd_qr(M, nJ, nI, cut_pinv, B0, B1, B2, tau, vbq, sig, ord, flags, &sweeps);
  // now Ub = U^ (nJ x r), Vb = V~ (nI x r), singular values sig[ord[0..r)]
  for (int e = t; e < r * pm; e += blockDim.x) {
    const int i = e % pm, rr = e / pm;
    a.Uhat[i + (int64_t)rr * pm] = i < nJ ? Ub[i + rr * LDP] : 0.0;
    a.Vtil[i + (int64_t)rr * pm] = i < nI ? Vb[i + rr * LDP] : 0.0;
  }
  const int nb = a.nb;
  if (t < kPMax) st->S[nb][t] = t < r ? sig[ord[t]] : 0.0;

  // ---- pruning: wave 0 takes the diagonal of R_R, wave 1 that of R_C, one lane per index; the
  // kept indices are compacted in order through a ballot
  if (t < 2 * 64) {
    const int w = t >> 6, l = t & 63;
    const int nn = w == 0 ? nI : nJ;
    const double* Rm = w == 0 ? R_R : R_C;
    const double d = l < nn ? fabs(Rm[l + (int64_t)l * pm]) : 0.0;
    const double mx = wave_max(d);
    const bool keep = l < nn && d >= st->tau * mx;
    const unsigned long long bal = __ballot(keep);
    if (keep) (w == 0 ? posI : posJ)[__popcll(bal & ((1ull << l) - 1))] = l;
    if (l == 0) cnt[w] = __popcll(bal);
  }
  __syncthreads();
  const int nIp = cnt[0], nJp = cnt[1];

  // ---- the indicator min(eta_1 (1 + eta_2), eta_2 (1 + eta_1)) S_min / ||S||_F is evaluated by
  // k_eta after rho, and only when it can matter: rows of an orthonormal basis have singular
  // values <= 1, so eta_1, eta_2 >= 1 and the indicator is at least 2 S_min / ||S||_F; when that
  // bound already fails the test (or at pass 0, where no stop is allowed) no stop is possible.
  bool need_eta;
  {
    double n2 = 0.0;
    for (int l = 0; l < r; ++l) n2 = fma(sig[ord[l]], sig[ord[l]], n2);
    need_eta = r > 0 && st->k >= 1 && nIp > 0 && nJp > 0 && 1.9 * sig[ord[r - 1]] < st->eps * sqrt(n2);
  }
  __syncthreads();

  // index sets of the new iterate, one thread per index
  if (t < nIp) {
    const int v = idxI[posI[t]];
    st->I[t] = v;
    st->Ib[nb][t] = v;
  }
  if (t >= kPMax && t - kPMax < nJp) {
    const int v = idxJ[posJ[t - kPMax]];
    st->J[t - kPMax] = v;
    st->Jb[nb][t - kPMax] = v;
  }
  if (t == 0) {
    double n2 = 0.0;
    for (int l = 0; l < r; ++l) n2 = fma(sig[ord[l]], sig[ord[l]], n2);
    const double nrm = sqrt(n2);
    st->nrm = nrm;
    st->eta1 = INFINITY;
    st->eta2 = INFINITY;
    st->ind = INFINITY;
    st->eta_need = need_eta ? 1 : 0;
    st->r[nb] = r;
    int rs = 0;
    for (int l = 0; l < r; ++l) rs += sig[ord[l]] > st->eps * sig[ord[0]] ? 1 : 0;
    st->r_sig = rs;
    st->nI = nIp;
    st->nJ = nJp;
    st->nIb[nb] = nIp;
    st->nJb[nb] = nJp;
    st->indb[nb] = INFINITY;
    if (r == 0) {  // the sampled fibers vanish: nothing to continue from
      st->done = 1;
      st->status = LRP_ENUMERIC;
    }
    const int kp = st->k;  // the pass being computed (passes completed so far)
    if (kp >= 0 && kp < a.maxiter) {
      a.trace.nI[kp] = nIp;
      a.trace.nJ[kp] = nJp;
      a.trace.rank[kp] = r;
      a.trace.ind[kp] = INFINITY;
      a.trace.branch[kp] = branch ? 1 : 0;
      a.trace.route[kp] = qr_route ? 0 : 1;
      a.trace.sweeps[kp] = sweeps;
    }
  }
}

// Indicator and stop decision of a pass (Algorithm 4, after rho): when a stop is possible
// (cheap bound passed, rho < eps), eta_1 = 1/sigma_min(U_k(I,:)) and eta_2 =
// 1/sigma_min(V_k(J,:)) on the pruned sets, with U_k(I,:) = Q(I,:) U^ and V_k(J,:) = Z(J,:) V~
// each stored tall (rows >= cols) so that Jacobi gives its min(rows, cols) singular values.
// Workgroup q solves problem q (two CUs; a problem's sweeps do not depend on the other's), and
// the second workgroup to finish makes the decision: the pass is accepted as the new iterate and
// the solve stops when max(rho, indicator) < eps, or after maxiter passes.
template <class Src>
__global__ __launch_bounds__(kEtaThreads) void k_eta(Src in) {
  const EtaArgs& a = kernel_args<EtaArgs>(in);
  DevState* st = a.st;
  if (st->done) return;
  __shared__ double E[kBuf], Qs[kBuf], Us[kBuf];
  __shared__ double red[1];
  __shared__ int flags[2], idx[kPMax], last;
  const int t = threadIdx.x, q = blockIdx.x;
  const int nb = a.nb;
  const int r = st->r[nb];
  const bool need = st->k >= 1 && st->eta_need && st->rho < st->eps;
  if (need) {
    // side 0: rows I of Q (ncols[0] columns) times U^; side 1: rows J of Z (ncols[1]) times V~
    const int ns = q == 0 ? st->nI : st->nJ;
    const int kc = st->ncols[q];
    const bool tall = ns >= r;
    if (t < kPMax) idx[t] = t < ns ? (q == 0 ? st->I[t] : st->J[t]) : 0;
    __syncthreads();
    gather_rows(q == 0 ? a.Q0 : a.Q1, a.ldq, idx, ns, kc, Qs);
    load_block(q == 0 ? a.Uhat : a.Vtil, a.pmax, kc, r, Us);
    __syncthreads();
    lds_gemm(Qs, Us, E, ns, r, !tall);
    __syncthreads();
    JacProb pp[1] = {{E, tall ? ns : r, tall ? r : ns, nullptr}};
    jacobi(pp, 1, flags);
    if (t < 64) {  // smallest column norm
      double v = INFINITY;
      if (t < pp[0].k) {
        double s = 0.0;
        for (int i = 0; i < pp[0].m; ++i) s = fma(E[i + t * LDP], E[i + t * LDP], s);
        v = sqrt(s);
      }
      for (int msk = 32; msk >= 1; msk >>= 1) v = fmin(v, shfl_xor_d(v, msk));
      if (t == 0) red[0] = v;
    }
    __syncthreads();
    if (t == 0) st->smin[q] = red[0];
  }
  // publish this workgroup's result, then count it; the second to arrive sees both
  __threadfence();
  __syncthreads();
  if (t == 0) last = atomicAdd(&st->eta_count, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (t == 0) {
    const volatile double* sm = st->smin;
    const double smin1 = need ? sm[0] : 0.0, smin2 = need ? sm[1] : 0.0;
    st->eta_count = 0;
    const int kp = st->k;
    double ind = INFINITY;
    if (need) {
      const double eta1 = smin1 > 0.0 ? 1.0 / smin1 : INFINITY;
      const double eta2 = smin2 > 0.0 ? 1.0 / smin2 : INFINITY;
      st->eta1 = eta1;
      st->eta2 = eta2;
      if (st->nrm > 0.0) ind = fmin(eta1 * (1.0 + eta2), eta2 * (1.0 + eta1)) * st->S[nb][r - 1] / st->nrm;
    }
    st->ind = ind;
    st->indb[nb] = ind;
    if (kp < a.maxiter) a.trace.ind[kp] = ind;
    st->ret = nb;
    st->k = kp + 1;
    if (kp >= 1 && fmax(st->rho, ind) < st->eps) {
      st->done = 1;
      st->status = LRP_OK;
    } else if (kp == a.maxiter - 1) {
      st->done = 1;
      st->status = LRP_NOT_CONVERGED;
    }
  }
}

int eta_launch(const EtaArgs& a, hipStream_t s) {
  LRP_LAUNCH_G(K_ETA, k_eta<EtaArgs>, k_eta<GroupRef>, dim3(2), dim3(kEtaThreads), 0, s, a);
  return launch_status();
}

// Warm start: M = R_u R_v^T (the core of F^ = U^ V^^T) and its SVD.
__global__ __launch_bounds__(kCoreThreads) void k_core_warm(CoreArgs a) {
  DevState* st = a.st;
  if (st->done) return;
  __shared__ double B0[kBuf], B1[kBuf], B2[kBuf], B3[kBuf];
  __shared__ double sig[kPMax], tau[kPMax], vbq[2 * kPMax];
  __shared__ int ord[kPMax], flags[2];
  const int t = threadIdx.x;
  // the width of the start: the right-hand side's rank, or the guess's columns
  const int rF = a.guess ? st->ncols[0] : st->rF;
  const int pm = a.pmax;
  // M = R_u R_v^T from the two triangular factors, staged in LDS first (B0 and B1 are free
  // until the SVD), so that no thread waits on a chain of memory loads
  load_block(a.R0, pm, rF, rF, B0);
  load_block(a.R1, pm, rF, rF, B1);
  __syncthreads();
  for (int e = t; e < rF * rF; e += blockDim.x) {
    const int i = e % rF, j = e / rF;
    double s = 0.0;
    for (int m = max(i, j); m < rF; ++m) s = fma(B0[i + m * LDP], B1[j + m * LDP], s);
    B3[i + j * LDP] = s;
  }
  __syncthreads();
  int sweeps = 0;
  const int r = svd_qr(B3, rF, rF, (double)rF, B0, B1, B2, tau, vbq, sig, ord, flags, &sweeps);
  // a zero guess leaves the start from the right-hand side in place
  if (a.guess && r == 0) {
    if (t == 0) st->guess_ok = 0;
    return;
  }
  for (int e = t; e < r * pm; e += blockDim.x) {
    const int i = e % pm, rr = e / pm;
    a.Uhat[i + (int64_t)rr * pm] = i < rF ? B2[i + rr * LDP] : 0.0;
    a.Vtil[i + (int64_t)rr * pm] = i < rF ? B0[i + rr * LDP] : 0.0;
  }
  if (t < kPMax) st->S[0][t] = t < r ? sig[ord[t]] : 0.0;
  __syncthreads();
  if (t == 0 && a.guess) st->guess_ok = 1;
  if (t == 0) {
    st->r[0] = r;
    st->nIb[0] = 0;
    st->nJb[0] = 0;
    st->indb[0] = INFINITY;
    if (r == 0 && a.zero_is_error) {  // a zero starting guess: nothing to start from
      st->done = 1;
      st->status = LRP_ENUMERIC;
      st->r_sig = 0;
    } else if (r == 0) {  // F = 0: the solution is 0
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
  if (warm) {
    LRP_LAUNCH(K_CORE_WARM, k_core_warm, dim3(1), dim3(kCoreThreads), 0, s, a);
  } else {
    LRP_LAUNCH_G(K_CORE, k_core<CoreArgs>, k_core<GroupRef>, dim3(1), dim3(kCoreThreads), 0, s, a);
  }
  return launch_status();
}


// ----------------------------------------------------------------------------------------
// Set-up, input scan and final truncation
// ----------------------------------------------------------------------------------------
__global__ void k_init_state(DevState* st, int rF, double eps, double tau, int replay_n) {
  if (threadIdx.x != 0) return;
  st->replay_n = replay_n;
  st->guess_ok = 0;
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
  st->eta_need = 0;
  st->eta_count = 0;
  st->eps = eps;
  st->tau = tau;
  st->r[0] = st->r[1] = 0;
  st->nIb[0] = st->nIb[1] = st->nJb[0] = st->nJb[1] = 0;
  st->rhob[0] = st->rhob[1] = INFINITY;
  st->indb[0] = st->indb[1] = INFINITY;
}

int init_state_launch(DevState* st, int rF, double eps, double tau, int replay_n, hipStream_t s) {
  LRP_LAUNCH(K_INIT, k_init_state, dim3(1), dim3(64), 0, s, st, rF, eps, tau, replay_n);
  return launch_status();
}

__global__ void k_guess_begin(DevState* st, int r0) {
  if (threadIdx.x != 0 || st->done) return;
  st->ncols[0] = r0;
  st->ncols[1] = r0;
  st->guess_ok = 0;
}

int guess_begin_launch(DevState* st, int r0, hipStream_t s) {
  LRP_LAUNCH(K_INIT, k_guess_begin, dim3(1), dim3(64), 0, s, st, r0);
  return launch_status();
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
  if (sig && blockIdx.x == 0 && threadIdx.x < rF) bad |= !isfinite(sig[threadIdx.x]);
  if (bad) {
    st->status = LRP_ENUMERIC;
    st->done = 1;
  }
}

int scan_inputs_launch(DevState* st, const double* U, int64_t ldu, const double* V, int64_t ldv,
                       const double* sig, int64_t n, int rF, hipStream_t s) {
  const int64_t total = n * rF;
  const int blocks = (int)std::min<int64_t>(1024, (total + 255) / 256);
  LRP_LAUNCH(K_SCAN, k_scan, dim3(std::max(blocks, 1)), dim3(256), 0, s, st, U, ldu, V, ldv, sig, n, rF);
  return launch_status();
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
  LRP_LAUNCH(K_FINALIZE, k_finalize, dim3(1), dim3(64), 0, s, st, S_out, r_max);
  return launch_status();
}

__global__ void k_copy_cols(const DevState* st, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t n,
                            int cols, int cols_out) {
  if (st && st->status < 0) return;
  const int64_t total = n * cols_out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    Y[i + c * ldy] = c < cols ? X[i + c * ldx] : 0.0;
  }
}

int copy_cols_launch(const DevState* st, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t n, int cols,
                     int cols_out, hipStream_t s, int) {
  const int64_t total = n * cols_out;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (total + 255) / 256));
  LRP_LAUNCH(K_FINALIZE, k_copy_cols, dim3(blocks), dim3(256), 0, s, st, X, ldx, Y, ldy, n, cols, cols_out);
  return launch_status();
}

__global__ void k_copy_ret(const DevState* st, const double* X0, const double* X1, int64_t n, double* Y, int64_t ldy,
                           int r_max) {
  if (st->status < 0) return;
  const double* X = st->ret ? X1 : X0;
  const int cols = st->zero ? 0 : st->r_final;
  const int64_t total = n * r_max;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    Y[i + c * ldy] = c < cols ? X[i + c * n] : 0.0;
  }
}

int copy_ret_launch(const DevState* st, const double* X0, const double* X1, int64_t n, double* Y, int64_t ldy,
                    int r_max, hipStream_t s) {
  const int64_t total = n * r_max;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (total + 255) / 256));
  LRP_LAUNCH(K_FINALIZE, k_copy_ret, dim3(blocks), dim3(256), 0, s, st, X0, X1, n, Y, ldy, r_max);
  return launch_status();
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
  return launch_status();
}

}  // namespace lrp
