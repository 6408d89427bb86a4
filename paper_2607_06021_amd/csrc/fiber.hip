// Fibers of the spectrally divided solution (paper, Section 3.1, eq. g_for_p):
//   W^(i, j) = sum_t U^(i, t) V^(j, t) / (lambda_i + lambda_j),
// with h^2 sigma folded into U^. One launch writes both C = W^(:, J) (side 0) and
// R^T = W^(I, :)^T (side 1): out(i, c) = sum_t A(i, t) b_c(t) / (lambda_i + lambda_{idx_c}),
// A = U^, b_c = V^(J_c, :) for side 0 and A = V^, b_c = U^(I_c, :) for side 1.
// The gathered b_c rows and lambda_{idx_c} sit in LDS. Reads of A and writes of out are
// coalesced (column-major, one row per lane). The mixed-precision path runs this kernel in
// FP32 with FP32 accumulation.
#include "lrp_kernels.h"

namespace lrp {

// q / d for d > 0 normal: reciprocal from the hardware approximation, two Newton steps on the
// reciprocal and one correction of the quotient (FP64); FP32 uses the plain division.
__device__ inline double div_pos(double q, double d) {
  const double r = rcp_nr(d);
  const double x = q * r;
  return fma(r, fma(-d, x, q), x);
}
__device__ inline float div_pos(float q, float d) { return q / d; }

// Each thread owns one grid row i: A(i, 0..rF-1) in registers (the loops over t are unrolled
// to RT >= rF with a uniform bound test, so the row never leaves registers); the outputs of 8
// columns are accumulated at once (two partial sums each, so 16 independent FMA chains hide
// the FP latency), with b_c(t) read from LDS as broadcasts. RT = 32 serves rF <= 32 with half
// the registers of RT = 64: the FP64 build runs four waves per SIMD instead of two (113 VGPRs
// against 177), so the loads, sums and stores of different blocks overlap (n = 2^20 - 1, rF = 30:
// 0.45 -> 0.30 ms per launch). Both builds make the same operations for such rF, so their
// results are bitwise equal.
template <typename T, int RT, class Src>
__global__ __launch_bounds__(256) void k_fiber(Src in) {
  const FiberArgs& a = kernel_args<FiberArgs>(in);
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  const int rF = st->rF;
  const int nc = side == 0 ? st->nJpre : st->nIpre;
  const int* idx = side == 0 ? st->Jpre : st->Ipre;
  const T* A = (const T*)(side == 0 ? a.Uh : a.Vh);
  const T* Bsrc = (const T*)(side == 0 ? a.Vh : a.Uh);
  const T* lam = (const T*)a.lam;
  T* out = (T*)(side == 0 ? a.C : a.Rt);

  constexpr int G = 8;
  __shared__ T b[kPMax + G][RT];  // rows beyond nc stay zero
  __shared__ T lb[kPMax + G];
  for (int e = threadIdx.x; e < (kPMax + G) * RT; e += blockDim.x) {
    const int cc = e / RT, tt = e % RT;
    b[cc][tt] = (cc < nc && tt < rF) ? Bsrc[idx[cc] + (int64_t)tt * a.ldh] : T(0);
  }
  for (int cc = threadIdx.x; cc < kPMax + G; cc += blockDim.x) lb[cc] = cc < nc ? lam[idx[cc]] : T(1);
  __syncthreads();

  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  T ar[RT];
#pragma unroll
  for (int tt = 0; tt < RT; ++tt) ar[tt] = tt < rF ? A[i + (int64_t)tt * a.ldh] : T(0);
  const T li = lam[i];
  for (int c0 = 0; c0 < nc; c0 += G) {
    T s0[G], s1[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s0[g] = s1[g] = T(0);
#pragma unroll
    for (int tt = 0; tt < RT; tt += 2) {
      if (tt < rF) {  // uniform
#pragma unroll
        for (int g = 0; g < G; ++g) {
          s0[g] = fma(ar[tt], b[c0 + g][tt], s0[g]);
          s1[g] = fma(ar[tt + 1], b[c0 + g][tt + 1], s1[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c0 + g < nc) out[i + (int64_t)(c0 + g) * a.ldc] = div_pos(s0[g] + s1[g], li + lb[c0 + g]);
  }
}

// Fibers of the test matrices of Section 4.2 (square, 0-based indices), from their formulas in
// FP64 (rounded to FP32 for the mixed-precision path):
//   H(i, j) = 1/(1 + i + j) (the Hilbert matrix);
//   K(i, j) = (|x_i + x_j| / 2)^5, x_i = -1 + 2 i/(n - 1), the fifth power as ((t t)(t t)) t.
// Side 0 writes C(i, c) = G(i, J_c), side 1 R^T(j, c) = G(I_c, j). One thread per grid row,
// coalesced column-major stores.
__device__ inline double matrix_entry(int kind, int64_t i, int64_t j, int64_t n) {
  if (kind == LRP_MAT_HILBERT) return 1.0 / ((1.0 + (double)i) + (double)j);
  const double x = -1.0 + (2.0 * (double)i) / (double)(n - 1);
  const double y = -1.0 + (2.0 * (double)j) / (double)(n - 1);
  const double t = fabs(x + y) / 2.0;
  const double t2 = t * t;
  return (t2 * t2) * t;
}

template <typename T, class Src>
__global__ __launch_bounds__(256) void k_fiber_matrix(Src in) {
  const FiberArgs& a = kernel_args<FiberArgs>(in);
  const DevState* st = a.st;
  if (st->done) return;
  const int side = blockIdx.y;
  const int nc = side == 0 ? st->nJpre : st->nIpre;
  const int* idx = side == 0 ? st->Jpre : st->Ipre;
  T* out = (T*)(side == 0 ? a.C : a.Rt);
  __shared__ int ix[kPMax];
  if (threadIdx.x < kPMax) ix[threadIdx.x] = threadIdx.x < nc ? idx[threadIdx.x] : 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  for (int c = 0; c < nc; ++c) {
    // side 0: G(i, J_c); side 1: G(I_c, i)
    const double g = side == 0 ? matrix_entry(a.matrix, i, ix[c], a.n) : matrix_entry(a.matrix, ix[c], i, a.n);
    out[i + (int64_t)c * a.ldc] = (T)g;
  }
}

int fiber_launch(const FiberArgs& a, bool fp32, hipStream_t s) {
  dim3 grid((unsigned)((a.n + 255) / 256), 2);
  if (a.matrix != LRP_MAT_POISSON) {
    if (fp32)
      LRP_LAUNCH_G(K_FIBER, (k_fiber_matrix<float, FiberArgs>), (k_fiber_matrix<float, GroupRef>), grid, dim3(256), 0, s, a);
    else
      LRP_LAUNCH_G(K_FIBER, (k_fiber_matrix<double, FiberArgs>), (k_fiber_matrix<double, GroupRef>), grid, dim3(256), 0, s, a);
    return launch_status();
  }
  if (fp32 && a.narrow)
    LRP_LAUNCH_G(K_FIBER, (k_fiber<float, 32, FiberArgs>), (k_fiber<float, 32, GroupRef>), grid, dim3(256), 0, s, a);
  else if (fp32)
    LRP_LAUNCH_G(K_FIBER, (k_fiber<float, 64, FiberArgs>), (k_fiber<float, 64, GroupRef>), grid, dim3(256), 0, s, a);
  else if (a.narrow)
    LRP_LAUNCH_G(K_FIBER, (k_fiber<double, 32, FiberArgs>), (k_fiber<double, 32, GroupRef>), grid, dim3(256), 0, s,
                 a);
  else
    LRP_LAUNCH_G(K_FIBER, (k_fiber<double, 64, FiberArgs>), (k_fiber<double, 64, GroupRef>), grid, dim3(256), 0, s,
                 a);
  return launch_status();
}

}  // namespace lrp
