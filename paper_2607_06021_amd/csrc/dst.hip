// Orthonormal DST-I of the columns of an n x c matrix, n + 1 = N a power of two.
//
// (Z x)_i = sqrt(2/N) sum_k x_k sin(pi i k / N) (paper, Section 3: the eigenvectors of T).
// Two real columns a, b share one complex FFT of length L = 2N of the odd extensions:
// z = ext(a) + i ext(b), ext(x) = [0, x_1..x_{N-1}, 0, -x_{N-1}..-x_1]. Its DFT is
// Z_k = 2 y_b(k) - 2 i y_a(k) with y(k) = sum_j x_j sin(pi j k / N), so
// (Z a)_k = -Im Z_k / sqrt(2N) and (Z b)_k = Re Z_k / sqrt(2N), k = 1..N-1.
// L <= 4096: one workgroup per column pair, the whole FFT in LDS.
// L  > 4096: four-step FFT, L = L1 L2; pass 1 does L1 FFTs of length L2 over the strided
// subsequences and applies the twiddles W_L^{j1 k2}; pass 2 does L2 FFTs of length L1.
// Twiddles come from tables built on the device from sincospi (exact arguments 2k/M).
#include "lrp_kernels.h"

namespace lrp {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ inline unsigned bitrev(unsigned j, int logL) {
  return logL == 0 ? 0u : (__brev(j) >> (32 - logL));
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

// Radix-2 decimation-in-time stages on `nb` sequences of length 2^logL stored contiguously
// in LDS in bit-reversed order; tw[k] = W_L^k, k < L/2. Natural-order output.
template <typename T>
__device__ void fft_stages(cplx<T>* buf, int logL, int nb, const cplx<T>* __restrict__ tw) {
  const int L = 1 << logL;
  const int halfL = L >> 1;
  const int total = nb * halfL;
  for (int s = 1; s <= logL; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = L >> s;  // W_{2 half}^k = W_L^{k L/(2 half)}
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int b = idx >> (logL - 1);
      const int q = idx & (halfL - 1);
      const int k = q & (half - 1);
      const int j0 = b * L + ((q >> (s - 1)) << s) + k;
      const int j1 = j0 + half;
      const cplx<T> w = tw[k * tstride];
      const cplx<T> t = cmul(w, buf[j1]);
      const cplx<T> u = buf[j0];
      buf[j0] = {u.x + t.x, u.y + t.y};
      buf[j1] = {u.x - t.x, u.y - t.y};
    }
    __syncthreads();
  }
}

// Column pair (ca, cb) of the source, with the odd extension, element j of z.
template <typename T>
__device__ inline cplx<T> ext_pair(const double* __restrict__ X, int64_t ldx, int ca, int cb,
                                   int ncols, int N, int j) {
  int src;
  T sg;
  if (j >= 1 && j < N) {
    src = j - 1;
    sg = T(1);
  } else if (j > N) {
    src = 2 * N - j - 1;
    sg = T(-1);
  } else {
    return {T(0), T(0)};
  }
  T a = ca < ncols ? (T)X[src + (int64_t)ca * ldx] * sg : T(0);
  T b = cb < ncols ? (T)X[src + (int64_t)cb * ldx] * sg : T(0);
  return {a, b};
}

// Store output k (1..N-1) of a pair; columns >= ncols (but < ncols_out) are written as 0.
template <typename T>
__device__ inline void put_pair(const DstArgs& a, int ca, int cb, int ncols, int k, cplx<T> Z,
                                double sa, double sb) {
  const double va = ca < ncols ? -(double)Z.y * sa : 0.0;
  const double vb = cb < ncols ? (double)Z.x * sb : 0.0;
  if (a.Yf) {  // FP32 destination (spectral factors of the mixed-precision path)
    if (ca < a.ncols_out) a.Yf[(k - 1) + (int64_t)ca * a.ldy] = (float)va;
    if (cb < a.ncols_out) a.Yf[(k - 1) + (int64_t)cb * a.ldy] = (float)vb;
  } else {
    if (ca < a.ncols_out) a.Y[(k - 1) + (int64_t)ca * a.ldy] = va;
    if (cb < a.ncols_out) a.Y[(k - 1) + (int64_t)cb * a.ldy] = vb;
  }
}

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

__device__ inline void col_scales(const DstArgs& a, int ca, int cb, int ncols, double& sa,
                                  double& sb) {
  sa = a.outscale;
  sb = a.outscale;
  if (a.scale) {
    if (ca < ncols) sa *= a.scale[ca];
    if (cb < ncols) sb *= a.scale[cb];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dst_small(DstArgs a) {
  __shared__ cplx<T> buf[4096];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int ca = 2 * blockIdx.x, cb = ca + 1;
  if (ca >= a.ncols_out) return;
  const int L = 1 << a.logL;
  const int N = L >> 1;
  for (int j = threadIdx.x; j < L; j += blockDim.x)
    buf[bitrev(j, a.logL)] = ext_pair<T>(X, a.ldx, ca, cb, ncols, N, j);
  __syncthreads();
  fft_stages<T>(buf, a.logL, 1, reinterpret_cast<const cplx<T>*>(a.t1));
  double sa, sb;
  col_scales(a, ca, cb, ncols, sa, sb);
  for (int k = 1 + threadIdx.x; k < N; k += blockDim.x) put_pair<T>(a, ca, cb, ncols, k, buf[k], sa, sb);
}

// Pass 1: for j1 in a tile, FFT over j2 of z[j1 + L1 j2] (length L2), times W_L^{j1 k2},
// stored transposed as Tb[pair][k2 L1 + j1].
template <typename T>
__global__ __launch_bounds__(256) void k_dst_pass1(DstArgs a) {
  __shared__ cplx<T> buf[4096];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int pair = blockIdx.y;
  const int ca = 2 * pair, cb = ca + 1;
  if (ca >= a.ncols_out) return;
  const int L1 = 1 << a.logL1, L2 = 1 << a.logL2;
  const int L = L1 * L2, N = L >> 1;
  const int TJ = a.tile1;
  const int j1_0 = blockIdx.x * TJ;
  for (int e = threadIdx.x; e < TJ * L2; e += blockDim.x) {
    const int jj = e % TJ, j2 = e / TJ;
    const int j = j1_0 + jj + L1 * j2;
    buf[jj * L2 + bitrev(j2, a.logL2)] = ext_pair<T>(X, a.ldx, ca, cb, ncols, N, j);
  }
  __syncthreads();
  fft_stages<T>(buf, a.logL2, TJ, reinterpret_cast<const cplx<T>*>(a.t2));
  const cplx<T>* thi = reinterpret_cast<const cplx<T>*>(a.t1);  // W_L^{a L2} = W_L1^a
  const cplx<T>* tlo = reinterpret_cast<const cplx<T>*>(a.tl);  // W_L^b, b < L2
  cplx<T>* Tb = reinterpret_cast<cplx<T>*>(a.work) + (int64_t)pair * L;
  for (int e = threadIdx.x; e < TJ * L2; e += blockDim.x) {
    const int jj = e % TJ, k2 = e / TJ;
    const int j1 = j1_0 + jj;
    const int m = j1 * k2;  // < L
    const cplx<T> w = cmul(thi[m >> a.logL2], tlo[m & (L2 - 1)]);
    Tb[(int64_t)k2 * L1 + j1] = cmul(w, buf[jj * L2 + k2]);
  }
}

// Pass 2: for k2 in a tile, FFT over j1 (length L1); output index k = k2 + L2 k1.
template <typename T>
__global__ __launch_bounds__(256) void k_dst_pass2(DstArgs a) {
  __shared__ cplx<T> buf[4096];
  const double* X;
  int ncols;
  if (!dst_resolve(a, X, ncols)) return;
  const int pair = blockIdx.y;
  const int ca = 2 * pair, cb = ca + 1;
  if (ca >= a.ncols_out) return;
  const int L1 = 1 << a.logL1, L2 = 1 << a.logL2;
  const int L = L1 * L2, N = L >> 1;
  const int TK = a.tile2;
  const int k2_0 = blockIdx.x * TK;
  const cplx<T>* Tb = reinterpret_cast<const cplx<T>*>(a.work) + (int64_t)pair * L;
  for (int e = threadIdx.x; e < TK * L1; e += blockDim.x) {
    const int kk = e / L1, j1 = e % L1;
    buf[kk * L1 + bitrev(j1, a.logL1)] = Tb[(int64_t)(k2_0 + kk) * L1 + j1];
  }
  __syncthreads();
  fft_stages<T>(buf, a.logL1, TK, reinterpret_cast<const cplx<T>*>(a.t1));
  double sa, sb;
  col_scales(a, ca, cb, ncols, sa, sb);
  for (int e = threadIdx.x; e < TK * L1; e += blockDim.x) {
    const int kk = e % TK, k1 = e / TK;
    const int k = k2_0 + kk + L2 * k1;
    if (k >= 1 && k < N) put_pair<T>(a, ca, cb, ncols, k, buf[kk * L1 + k1], sa, sb);
  }
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
  const int64_t N = n + 1;
  const int logL = ilog2(2 * N);
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
    if (p->logL1 > 12) return LRP_EINVAL;
  }
  const int L1 = 1 << p->logL1, L2 = 1 << p->logL2;
  p->tile1 = p->four_step ? std::min(16, std::max(1, 4096 / L2)) : 0;
  p->tile2 = p->four_step ? std::min(16, std::max(1, 4096 / L1)) : 0;
  if (p->four_step && (L1 % p->tile1 != 0 || L2 % p->tile2 != 0)) return LRP_EINVAL;
  p->t1_count = L1;
  p->t2_count = p->four_step ? L2 : 0;
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
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

int dst_launch(const DstPlan& p, DstArgs a, bool fp32, hipStream_t s) {
  const int npairs = (a.ncols_out + 1) / 2;
  if (npairs <= 0) return LRP_OK;
  if (npairs > p.max_pairs) return LRP_EINVAL;
  a.logL = p.logL;
  a.logL1 = p.logL1;
  a.logL2 = p.logL2;
  a.tile1 = p.tile1;
  a.tile2 = p.tile2;
  a.t1 = fp32 ? (const void*)p.t1_32 : (const void*)p.t1_64;
  a.t2 = fp32 ? (const void*)p.t2_32 : (const void*)p.t2_64;
  a.tl = fp32 ? (const void*)p.tl_32 : (const void*)p.tl_64;
  a.outscale *= 1.0 / std::sqrt(2.0 * (double)(p.n + 1));
  if (!p.four_step) {
    if (fp32)
      hipLaunchKernelGGL(k_dst_small<float>, dim3(npairs), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(k_dst_small<double>, dim3(npairs), dim3(256), 0, s, a);
  } else {
    a.work = p.work;
    const int L1 = 1 << p.logL1, L2 = 1 << p.logL2;
    dim3 g1(L1 / p.tile1, npairs), g2(L2 / p.tile2, npairs);
    if (fp32) {
      hipLaunchKernelGGL(k_dst_pass1<float>, g1, dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_dst_pass2<float>, g2, dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_dst_pass1<double>, g1, dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_dst_pass2<double>, g2, dim3(256), 0, s, a);
    }
  }
  return hipGetLastError() == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // namespace lrp
