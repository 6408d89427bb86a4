// Kernel argument blocks and host-side launchers of the low-rank Poisson library.
#pragma once

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lrp_internal.h"

namespace lrp {

// ---------------------------------------------------------------- DST-I (dst.hip)
// ---------------------------------------------------------------- launch profile
// Kernel classes for the optional per-kernel timing of a solve (api.hip).
enum KernelId {
  K_INIT, K_SCAN, K_DST_SINGLE, K_DST_PASS1, K_DST_PASS2, K_FIBER, K_TSQR_FACTOR, K_TSQR_APPLY,
  K_CORE_WARM, K_CORE, K_PROD, K_PI, K_GMAX, K_TOPK_BLOCK, K_TOPK_MERGE, K_SELECT, K_RHO_A,
  K_RHO_B, K_RHO_REDUCE, K_RHO_FINAL, K_ETA, K_FINALIZE, K_COPY, K_EMPTY, K_QDEIM, K_COUNT
};
// Called right before a launch (or copy) on stream s: when this thread is recording a
// profile on s, records an event that ends the previous entry and starts this one.
// Profile mode: the start/stop events of a launch of kernel class id on stream s, attached to the
// dispatch itself (hipExtLaunchKernelGGL), or nulls when no profile is being recorded there.
struct ProfEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
ProfEvents prof_launch(hipStream_t s, int id);
// Events around a non-kernel operation (a copy) of class id: begin before it, end after it.
void prof_begin(hipStream_t s, int id);
void prof_end(hipStream_t s);

// ---------------------------------------------------------------- grouped launches
// A pass of several requests of one shape runs as one launch per stage (the serving loop):
// each request keeps the argument blocks of its pass's launches in device memory, at the same
// offsets as every other request of that shape, and workgroup z of a grouped launch runs the
// stage's kernel body on request z's block. The grid's x and y and the body are those of the
// solo launch, so a request's result does not depend on the group it ran in.
struct GroupRef {
  const char* const* bases;  // per request z: its argument area (device)
  uint32_t off;              // offset of this launch's block in every area
};
// The blocks are read through the constant address space: they do not change while a launch
// runs, so uniform reads of them (dynamic indexing included) become scalar loads, as reads of
// the kernel argument segment are.
typedef const __attribute__((address_space(4))) char* lrp_const_ptr;
template <class A>
__device__ __forceinline__ const A& group_args(const GroupRef& g) {
  const lrp_const_ptr* tab = (const lrp_const_ptr*)(const __attribute__((address_space(4))) void*)g.bases;
  return *(const A*)(const __attribute__((address_space(4))) A*)(tab[blockIdx.z] + g.off);
}
// A stage kernel is a template over where its argument block comes from: the block itself (a
// solo launch) or a GroupRef (a grouped launch); the kernel body binds `const Args& a` to
// kernel_args<Args>(src) and is otherwise the same code for both.
template <class A>
__device__ __forceinline__ const A& kernel_args(const A& a) {
  return a;
}
template <class A>
__device__ __forceinline__ const A& kernel_args(const GroupRef& g) {
  return group_args<A>(g);
}

// One launch of a recorded pass: the grouped kernel, the solo grid and block, and where the
// argument block sits in the request's argument area.
struct LaunchRec {
  const void* fn;
  unsigned gx, gy, bx;
  uint32_t shm, off, size;
  bool operator==(const LaunchRec& o) const {
    return fn == o.fn && gx == o.gx && gy == o.gy && bx == o.bx && shm == o.shm && off == o.off && size == o.size;
  }
};
// While a recorder is set on this thread, the launchers of a pass record instead of launching;
// a launch without a grouped form marks the record unusable.
struct PassRecord {
  std::vector<LaunchRec> recs;
  std::vector<unsigned char> blob;  // the argument blocks, 16-byte aligned
  bool bad = false;
};
PassRecord*& pass_recorder();
void record_launch(PassRecord* r, const void* fn, dim3 grid, dim3 block, size_t shm, const void* args, size_t size);

// Launch of a stage with a grouped form KERNEL_G (one argument block ARGS).
#define LRP_LAUNCH_G(ID, KERNEL, KERNEL_G, GRID, BLOCK, SHM, STREAM, ARGS)                             \
  do {                                                                                                \
    if (::lrp::PassRecord* rec_ = ::lrp::pass_recorder()) {                                           \
      ::lrp::record_launch(rec_, reinterpret_cast<const void*>(KERNEL_G), GRID, BLOCK, SHM, &(ARGS),     \
                           sizeof(ARGS));                                                             \
      break;                                                                                          \
    }                                                                                                 \
    LRP_LAUNCH(ID, KERNEL, GRID, BLOCK, SHM, STREAM, ARGS);                                           \
  } while (0)

#define LRP_LAUNCH(ID, KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                        \
  do {                                                                                              \
    if (::lrp::PassRecord* rec_any_ = ::lrp::pass_recorder()) {                                     \
      rec_any_->bad = true;                                                                         \
      break;                                                                                        \
    }                                                                                               \
    const ::lrp::ProfEvents pe_ = ::lrp::prof_launch((STREAM), (ID));                               \
    if (pe_.start)                                                                                  \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, pe_.start, pe_.stop, 0, __VA_ARGS__);  \
    else                                                                                            \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                            \
  } while (0)

struct DstPlan {
  int64_t n;
  int logL, logL1, logL2;  // L = 2(n+1); four-step: L = L1 L2 (pass 2 length L1, pass 1 length L2)
  int four_step;
  int max_pairs;
  int t1_count, t2_count;
  int64_t s1;              // row stride (complex elements) of the four-step intermediate
  int64_t work_bytes;      // bytes of the intermediate for max_pairs column pairs (FP64)
  double2 *t1_64, *t2_64, *tl_64;
  float2 *t1_32, *t2_32, *tl_32;
  void* work;
  // n + 1 not a power of two: the length-2(n+1) DFT by Bluestein's chirp-z method on
  // power-of-two FFTs of length M = 2^logM >= 4(n+1) - 1 (M = M1 M2 above 4096 points)
  int bluestein;
  int logM;
  int batch_pairs;         // column pairs per round of launches (bounds the work buffers)
  double2* chirp_64;       // L entries exp(-pi i (j^2 mod 2L)/L)
  float2* chirp_32;
  double2* bhat_64;        // M entries: DFT_M of the circular chirp b_m = conj(chirp_|m|)
  float2* bhat_32;
  void* work2;             // batch_pairs x M complex: the data between the two FFTs (FP64 size)
};

struct DstArgs {
  const double* X;   // source columns (ld ldx)
  const double* X1;  // second candidate source (pick_ret)
  int64_t ldx;
  double* Y;         // FP64 destination (ld ldy), or
  float* Yf;         // FP32 destination
  int64_t ldy;
  int ncols;         // columns to transform
  int ncols_out;     // columns written (extra ones are zero-filled)
  const double* scale;  // per-column factor or null
  double outscale;      // global factor (the launcher folds in 1/sqrt(2N))
  const DevState* st;   // optional: skip after an error; pick_ret selects source/rank
  int pick_ret;
  // filled by the launcher
  int pair0;  // first column pair of this launch (pairs are transformed in batches)
  int logL, logL1, logL2;
  int64_t s1;
  const void *t1, *t2, *tl;
  void* work;
};

int dst_plan(DstPlan* p, int64_t n, int max_cols);
int dst_alloc(DstPlan* p);  // tables and work buffers of a plan
void dst_free(DstPlan* p);
int dst_tables(DstPlan* p, hipStream_t s);
// device bytes dst_alloc takes for this plan
int64_t dst_bytes(const DstPlan& p);
int dst_launch(const DstPlan& p, DstArgs a, bool fp32, hipStream_t s);

// ---------------------------------------------------------------- TSQR (tsqr.hip)
struct TsqrPlan {
  int64_t n;
  int pmax;
  int nlevels;
  TsqrLevel lev[kMaxLevels];
};

// Level-0 input and output of one two-sided TSQR.
struct TsqrIO {
  const DevState* st;  // if set: ncols per side from st->ncols[side]; skip when st->done
  int ncols[2];        // used when st is null
  int nsides;
  const void* X[2];    // level-0 inputs (n rows), FP64 or FP32
  int x_f32;
  int64_t ldx;
  double* Q[2];        // level-0 apply output (n rows), ld ldq; null -> internal Y
  int64_t ldq;
};

int tsqr_plan(TsqrPlan* p, int64_t n, int pmax);
int tsqr_run(const TsqrPlan& p, const TsqrIO& io, hipStream_t s);
// Final R of side `side` (pmax x pmax, ld pmax, upper triangular).
inline const double* tsqr_R(const TsqrPlan& p, int side) { return p.lev[p.nlevels - 1].Rout[side]; }

// ---------------------------------------------------------------- fibers (fiber.hip)
struct FiberArgs {
  const DevState* st;
  const void* Uh;  // n x rF spectral factors (U side carries h^2 sigma), FP64 or FP32
  const void* Vh;
  int64_t ldh;
  const void* lam;  // eigenvalues, same type
  void* C;          // n x pmax: C = W^(:, Jpre)
  void* Rt;         // n x pmax: R^T = W^(Ipre, :)^T
  int64_t ldc;
  int64_t n;
  int matrix;       // enum lrp_matrix: LRP_MAT_POISSON uses Uh, Vh, lam; the test matrices are
                    // evaluated from their formulas
  int narrow;       // 1: the right-hand side's rank is at most 32 (a build with half the registers)
};
int fiber_launch(const FiberArgs& a, bool fp32, hipStream_t s);

// ---------------------------------------------------------------- core (core.hip)
struct CoreArgs {
  DevState* st;
  const double* Q0;  // explicit Q of side 0 (C), n x ncols[0]
  const double* Q1;  // explicit Q of side 1 (R^T), n x ncols[1]
  int64_t ldq;
  const double* R0;  // pmax x pmax
  const double* R1;
  int pmax;
  double* Uhat;      // out: pmax x pmax (ld pmax): coefficients of U_k in Q
  double* Vtil;      // out: coefficients of V_k in Z
  int nb;            // iterate buffer written by this pass
  TraceBuf trace;    // row = the device pass counter
  int maxiter;
  int guess;         // warm start only: 1 = from the initial guess (width st->ncols[0]; a zero
                     // guess leaves the start from the right-hand side in place)
  int zero_is_error; // warm start only: a zero start is an error (LRP_ENUMERIC), not F = 0
};
int core_launch(const CoreArgs& a, bool warm, hipStream_t s);

// ---------------------------------------------------------------- products (prod.hip)
struct ProdArgs {
  const DevState* st;
  const double* Q[2];
  int64_t ldq;
  const double* B[2];  // pmax x pmax coefficient matrices (Uhat / Vtil)
  int pmax;
  double* out[2];      // n x pmax (ld ldo)
  int64_t ldo;
  int64_t n;
  int nb;              // buffer index whose rank st->r[nb] gives the columns
  int gate_guess;      // 1: run only if st->guess_ok (the product of a warm start from a guess)
  int tiles;           // set by prod_launch: 16-row tiles per wave (even)
};
int prod_launch(const ProdArgs& a, hipStream_t s);

struct EtaArgs {
  DevState* st;
  const double* Q0;  // Q of side 0 (ncols[0] columns), ld ldq
  const double* Q1;  // Z of side 1 (ncols[1] columns)
  int64_t ldq;
  const double* Uhat;  // pmax x pmax coefficients (U_k = Q U^), ld pmax
  const double* Vtil;
  int pmax;
  int nb;              // iterate buffer of this pass
  int maxiter;
  TraceBuf trace;
};
int eta_launch(const EtaArgs& a, hipStream_t s);

// ---------------------------------------------------------------- selection (select.hip)
struct SelectPlan {
  int64_t n;
  int nblocks;            // ceil(n / kSelRows)
  int nlevels;            // merge levels after the block level
  int lists[8];           // lists at each merge level input
  double* pi[2];          // n
  double* bmax[2];        // nblocks
  double* gmax;           // 2
  double* cand_s[2][2];   // ping-pong candidate scores
  int* cand_i[2][2];
};
int select_plan(SelectPlan* p, int64_t n);
// Leverage scores of the iterate in buffers U0/U1 and top candidates outside the pruned sets.
// sampled: rows are drawn with probability min(1, rho score) first (Philox4x32-10, key seed).
struct SampleOpts {
  int sampled;
  double rho;
  uint64_t seed;
};
int select_candidates(const SelectPlan& p, const DevState* st, const double* U[2], int64_t ldu,
                      hipStream_t s, int* final_list_slot, SampleOpts so = SampleOpts{});
// ---------------------------------------------------------------- QDEIM (select.hip)
// Control block of the column-pivoted QR of U(:, :r_sig)^T, one per side (device memory).
struct QdeimCtl {
  double v[kPMax];  // reflector of the last step at its absolute positions (zero elsewhere), v_j = 1
  double tau;
  double floor;     // squared norms at or below it count as 0 (set by the first step)
  int piv[kPMax];   // pivots in the order chosen
  int count;        // blocks of the current step that have finished (0 between launches)
  int pad;
};
struct QdeimPlan {
  int64_t n;
  int nblocks;
  double* work[2];  // n x kPMax: the rows of U(:, :r_sig) as the reflectors transform them
  double* nrm[2];   // n: trailing squared norm of each row (-1 once pivoted)
  double* bmax[2];  // nblocks: block maxima of nrm
  int* flag[2];     // n: 1 once the row is a pivot
  QdeimCtl* ctl;    // 2
};
int qdeim_plan(QdeimPlan* p, int64_t n, hipStream_t s);
void qdeim_free(QdeimPlan* p);
// r_sig pivots per side of the iterate U[side] (ld ldu); pmax launches, those past r_sig return at once.
int qdeim_launch(const QdeimPlan& p, const DevState* st, const double* U[2], int64_t ldu, int pmax, hipStream_t s);

struct SelectArgs {
  DevState* st;
  const double* cs[2];  // final candidate list per side (kPMax entries, best first)
  const int* ci[2];
  int pmax;
  int64_t n;
  TraceBuf trace;
  ReplayBuf replay;     // sets of passes k < st->replay_n
  const QdeimCtl* qd;   // QDEIM pivots (null: leverage-score selection)
  int sampled;          // sampled leverage scores: take every drawn candidate (up to the cap)
};
int select_update(const SelectArgs& a, hipStream_t s);

// ---------------------------------------------------------------- rho / stop (rho.hip)
struct RhoPlan {
  int64_t n;
  int nblocks;
  double* part;  // nblocks x 2 x kPMax x kPMax
  double* M;     // 2 x kPMax x kPMax : M_u, N_v
  double* G;     // 2 x kPMax x kPMax : Y^T Y, Y'^T Y'
};
int rho_plan(RhoPlan* p, int64_t n);
struct RhoArgs {
  DevState* st;
  const double* Unew[2];  // U_k, V_k
  const double* Uold[2];  // U_{k-1}, V_{k-1}
  int64_t ldu;
  int nb_new, nb_old;
  int maxiter;
  TraceBuf trace;
};
int rho_launch(const RhoPlan& p, const RhoArgs& a, hipStream_t s);

// ---------------------------------------------------------------- misc (core.hip)
int scan_inputs_launch(DevState* st, const double* U, int64_t ldu, const double* V, int64_t ldv,
                       const double* sig, int64_t n, int rF, hipStream_t s);
int finalize_launch(DevState* st, double* S_out, int r_max, hipStream_t s);
int init_state_launch(DevState* st, int rF, double eps, double tau, int replay_n, hipStream_t s);
// Warm start from a guess of r0 columns: QR widths r0, guess_ok cleared.
int guess_begin_launch(DevState* st, int r0, hipStream_t s);
// Y(:, 0:cols) = X(:, 0:cols) for n rows, columns cols..cols_out-1 of Y set to 0 (skipped after an
// error in st, if given).
int copy_cols_launch(const DevState* st, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t n, int cols,
                     int cols_out, hipStream_t s, int unused);
// The returned iterate (X0 or X1 by st->ret, st->r_final columns, 0 for a zero result) into Y,
// r_max columns (zeros past the rank).
int copy_ret_launch(const DevState* st, const double* X0, const double* X1, int64_t n, double* Y, int64_t ldy,
                    int r_max, hipStream_t s);
int lambda_launch(double* lam, float* lam32, int64_t n, hipStream_t s);

}  // namespace lrp
