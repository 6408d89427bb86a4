// Internal definitions shared by the HIP sources of the low-rank Poisson library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrp.h"

namespace lrp {

constexpr int kPMax = 64;          // largest index set / rank the kernels are built for
constexpr int kTsqrRows = 256;     // rows of one block QR
constexpr int kTsqrThreads = 1024;  // 16 waves, four columns each
constexpr int kSelRows = 256;      // rows per leverage-score block
constexpr int kMergeFan = 16;      // candidate lists merged per block
constexpr int kCUs = 256;          // compute units of the MI355X
constexpr int kMaxLevels = 12;     // TSQR tree levels (n <= 2^23 needs 7 at p_max = 64)
constexpr double kEps = 2.220446049250313e-16;
// leverage scores at or below (64 eps)^2 * max(pi) are rounding noise and count as 0
constexpr double kFloorRel = (64.0 * kEps) * (64.0 * kEps);

// Device-resident control state of one solve. Sizes and index sets live here so that the
// whole pass can be enqueued without reading anything back to the host.
struct DevState {
  int done;     // 1: stop -- every later kernel of the solve returns at once
  int status;   // lrp_status of the solve so far
  int k;        // cross approximations computed
  int ret;      // iterate buffer (0/1) holding the result
  int zero;     // right-hand side is exactly zero
  int rF;       // rank of the right-hand side
  int ncols[2]; // columns of the QR inputs: side 0 = C = W^(:,J) (|J|), side 1 = R^T (|I|)
  int nI, nJ;   // pruned sets of the newest iterate
  int nIpre, nJpre;
  int nIprev, nJprev;  // pre-prune sets of the previous pass (fixed-point test)
  int r_sig;    // leading singular vectors used by the next selection
  int r_final;  // rank of the returned solution
  int eta_need;  // 1: the last core passed the cheap bound on the indicator (a stop is possible)
  int replay_n;  // passes 0 .. replay_n-1 take their index sets from the replay buffers
  int guess_ok;  // 1: the initial guess was nonzero and replaced the start from the right-hand side
  double nrm, ind, rho, eta1, eta2;
  double smin[2];  // sigma_min of U_k(I,:) and V_k(J,:) from the indicator's two workgroups
  int eta_count;   // indicator workgroups done with the current pass (the second one decides)
  double eps;   // effective tolerance
  double tau;   // prune threshold
  int I[kPMax], J[kPMax];
  int Ipre[kPMax], Jpre[kPMax];
  int Iprev[kPMax], Jprev[kPMax];
  // per iterate buffer
  double S[2][kPMax];
  int r[2];
  int nIb[2], nJb[2];
  int Ib[2][kPMax], Jb[2][kPMax];
  double indb[2], rhob[2];
};

struct TraceBuf {
  int* Ipre;   // maxiter x kPMax
  int* Jpre;
  int* nIpre;  // maxiter
  int* nJpre;
  int* nI;
  int* nJ;
  int* rank;
  double* ind;
  double* rho;
  int* branch;  // 1: |J| <= |I| (the core solves with Q(I,:)); 0: with Z(J,:)
  int* route;   // pseudo-inverse of the core: 0 Householder QR (left inverse), 1 Jacobi SVD with cutoff
  int* sweeps;  // one-sided Jacobi sweeps of the core's SVD
};

// Index sets given for the first passes of a solve (replay): maxiter x kPMax entries per side.
struct ReplayBuf {
  int* I;
  int* J;
  int* nI;  // maxiter
  int* nJ;
};

// One level of the TSQR tree, two independent sides per launch.
struct TsqrLevel {
  int64_t rows;      // rows of this level's input
  int block_rows;    // rows per block (<= kTsqrRows)
  int nblocks;
  double* V[2];      // Householder vectors, rows x p_max (ld = rows), 1 on the diagonal
  double* tau[2];    // nblocks x p_max
  double* Rout[2];   // R factors stacked for the next level: (nblocks p_max) x p_max
  double* Y[2];      // top-down output of this level: rows x p_max (ld = rows)
};

// ----------------------------------------------------------------------------------------
// Wavefront helpers (64 lanes)
// ----------------------------------------------------------------------------------------
// 1/x and 1/sqrt(x) from the hardware approximations refined by two Newton steps (each
// step squares the relative error), for normal positive x (rcp_nr: normal nonzero x).
// Status of the launches just made on this thread. hipErrorNotReady (the answer of a
// non-blocking hipEventQuery on unfinished work) is never a launch failure.
inline int launch_status() {
  const hipError_t e = hipGetLastError();
  return (e == hipSuccess || e == hipErrorNotReady) ? LRP_OK : LRP_EDEVICE;
}

__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ inline double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

__device__ inline double shfl_xor_d(double x, int mask) {
  int lo = __double2loint(x);
  int hi = __double2hiint(x);
  lo = __shfl_xor(lo, mask, 64);
  hi = __shfl_xor(hi, mask, 64);
  return __hiloint2double(hi, lo);
}

// Sum over the 4 lanes of a quad (lanes 4q .. 4q+3) using DPP quad permutes.
__device__ inline double quad_sum(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  int lo1 = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  int hi1 = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  x += __hiloint2double(hi1, lo1);
  lo = __double2loint(x);
  hi = __double2hiint(x);
  int lo2 = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  int hi2 = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  return x + __hiloint2double(hi2, lo2);
}

__device__ inline float quad_sum_f(float x) {
  int v = __float_as_int(x);
  x += __int_as_float(__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
  v = __float_as_int(x);
  return x + __int_as_float(__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
}

__device__ inline double wave_sum(double x) {
  for (int m = 32; m >= 1; m >>= 1) x += shfl_xor_d(x, m);
  return x;
}

__device__ inline double wave_max(double x) {
  for (int m = 32; m >= 1; m >>= 1) x = fmax(x, shfl_xor_d(x, m));
  return x;
}

// Sum over aligned groups of 8 consecutive lanes (DPP: lane ^ 1, lane ^ 2, then the other quad
// of the octet); every lane gets its group's total.
__device__ inline double oct_sum(double x) {
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
  return x;
}

// Block-wide sum for blockDim.x == 256; `scratch` holds >= 4 doubles of LDS. Ends with every
// thread holding the total; contains two barriers.
__device__ inline double block_sum256(double x, double* scratch) {
  x = wave_sum(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) scratch[w] = x;
  __syncthreads();
  double t = scratch[0] + scratch[1] + scratch[2] + scratch[3];
  __syncthreads();
  return t;
}

__device__ inline double block_max256(double x, double* scratch) {
  x = wave_max(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) scratch[w] = x;
  __syncthreads();
  double t = fmax(fmax(scratch[0], scratch[1]), fmax(scratch[2], scratch[3]));
  __syncthreads();
  return t;
}

}  // namespace lrp

#define LRP_HIP_CHECK(expr)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return LRP_EDEVICE;        \
  } while (0)
