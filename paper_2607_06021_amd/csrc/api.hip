// C-ABI of the low-rank Poisson library: context, workspace and the solve pipeline.
//
// One solve (paper, Section 3.2 with Algorithm 4):
//   DST-I of the factors (U side scaled by h^2 sigma)          -> U^, V^
//   warm start: thin QRs of U^, V^ and the SVD of R_u R_v^T      -> U_{-1}, S_{-1}, V_{-1}
//   pass k = 0 .. maxiter-1:
//     leverage-score selection from U_{k-1}, V_{k-1}             -> I_k, J_k (fixed-point test)
//     fibers C = W^(:, J_k), R^T = W^(I_k, :)^T
//     thin QRs C = Q R_C, R^T = Z R_R (Householder TSQR)
//     core: pseudo-inverse, |J| x |I| core, its SVD, pruning, indicator
//     U_k = Q U^, V_k = Z V~
//     rho (only if the indicator passes) and the stopping decision
//   final truncation of the returned iterate and DST-I back to physical space.
// Every size, index set and flag stays in device memory; each kernel of a pass reads them
// there and returns at once after the solve has stopped, so a pass is enqueued without any
// read-back. The stop flag of a pass is copied right after its decision; the host reads it
// while the device runs that pass's candidate selection (the serving loop reads it one pass
// behind).
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include <hip/hip_ext.h>

#include "ctx.h"

using namespace lrp;

namespace lrp {

template <typename T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, sizeof(T) * count) == hipSuccess ? LRP_OK : LRP_ENOMEM;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// [p, p + bytes) of a column-major n x cols matrix with leading dimension ld
struct Range {
  uintptr_t lo, hi;
};
Range span(const void* p, int64_t n, int64_t ld, int64_t cols, size_t w) {
  uintptr_t lo = (uintptr_t)p;
  uintptr_t hi = lo + (uintptr_t)(((cols - 1) * ld + n) * (int64_t)w);
  return {lo, hi};
}
bool overlap(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; }

void free_ctx(lrp_ctx* c) {
  if (!c) return;
  dfree(c->st);
  if (c->st_host) (void)hipHostFree(c->st_host);
  if (c->done_host) (void)hipHostFree(c->done_host);
  dfree(c->lam);
  dfree(c->lam32);
  dfree(c->Uh);
  dfree(c->Vh);
  dfree(c->Uh32);
  dfree(c->Vh32);
  dfree(c->C);
  dfree(c->Rt);
  dfree(c->C32);
  dfree(c->Rt32);
  for (int s = 0; s < 2; ++s) {
    dfree(c->Q[s]);
    dfree(c->Uit[s]);
    dfree(c->Vit[s]);
  }
  dfree(c->Uhat);
  dfree(c->Vtil);
  dfree(c->trace.Ipre);
  dfree(c->trace.Jpre);
  dfree(c->trace.nIpre);
  dfree(c->trace.nJpre);
  dfree(c->trace.nI);
  dfree(c->trace.nJ);
  dfree(c->trace.rank);
  dfree(c->trace.ind);
  dfree(c->trace.rho);
  dfree(c->trace.branch);
  dfree(c->trace.route);
  dfree(c->trace.sweeps);
  dfree(c->replay.I);
  dfree(c->replay.J);
  dfree(c->replay.nI);
  dfree(c->replay.nJ);
  dst_free(&c->dst);
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  c->prof_ev.clear();

  for (int L = 0; L < c->tsqr.nlevels; ++L)
    for (int s = 0; s < 2; ++s) {
      dfree(c->tsqr.lev[L].V[s]);
      dfree(c->tsqr.lev[L].tau[s]);
      dfree(c->tsqr.lev[L].Rout[s]);
      dfree(c->tsqr.lev[L].Y[s]);
    }
  for (int s = 0; s < 2; ++s) {
    dfree(c->sel.pi[s]);
    dfree(c->sel.bmax[s]);
    for (int b = 0; b < 2; ++b) {
      dfree(c->sel.cand_s[b][s]);
      dfree(c->sel.cand_i[b][s]);
    }
  }
  dfree(c->sel.gmax);
  qdeim_free(&c->qd);
  dfree(c->rho.part);
  dfree(c->rho.M);
  dfree(c->rho.G);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->evfin) (void)hipEventDestroy(c->evfin);
  for (int s = 0; s < 2; ++s)
    if (c->evit[s]) (void)hipEventDestroy(c->evit[s]);
  for (int s = 0; s < 4; ++s) {
    if (c->gexec[s]) (void)hipGraphExecDestroy(c->gexec[s]);
    if (c->gexec_upd[s]) (void)hipGraphExecDestroy(c->gexec_upd[s]);
  }
  for (int s = 0; s < 2; ++s)
    if (c->gexec_sel[s]) (void)hipGraphExecDestroy(c->gexec_sel[s]);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

#define TRY(expr)                 \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != LRP_OK) return rc_; \
  } while (0)

int create_impl(lrp_ctx* c) {
  const int64_t n = c->n;
  const int pm = c->r_max;
  const bool mixed = c->precision == LRP_MIXED;
  const size_t np = (size_t)n * pm;
  if (hipGetDevice(&c->device) != hipSuccess) return LRP_EDEVICE;
  TRY(dalloc(&c->st, 1));
  if (hipHostMalloc((void**)&c->st_host, sizeof(DevState)) != hipSuccess) return LRP_ENOMEM;
  if (hipHostMalloc((void**)&c->done_host, 2 * sizeof(int)) != hipSuccess) return LRP_ENOMEM;
  const bool poisson = c->matrix == LRP_MAT_POISSON;
  if (poisson) {
    TRY(dalloc(&c->lam, n));
    TRY(dalloc(&c->lam32, n));
  }
  if (mixed) {
    if (poisson) {
      TRY(dalloc(&c->Uh32, np));
      TRY(dalloc(&c->Vh32, np));
    }
    TRY(dalloc(&c->C32, np));
    TRY(dalloc(&c->Rt32, np));
  } else {
    if (poisson) {
      TRY(dalloc(&c->Uh, np));
      TRY(dalloc(&c->Vh, np));
    }
    TRY(dalloc(&c->C, np));
    TRY(dalloc(&c->Rt, np));
  }
  for (int s = 0; s < 2; ++s) {
    TRY(dalloc(&c->Q[s], np));
    TRY(dalloc(&c->Uit[s], np));
    TRY(dalloc(&c->Vit[s], np));
  }
  TRY(dalloc(&c->Uhat, (size_t)pm * pm));
  TRY(dalloc(&c->Vtil, (size_t)pm * pm));
  const size_t mi = (size_t)std::max(c->maxiter, 1);
  TRY(dalloc(&c->trace.Ipre, mi * kPMax));
  TRY(dalloc(&c->trace.Jpre, mi * kPMax));
  TRY(dalloc(&c->trace.nIpre, mi));
  TRY(dalloc(&c->trace.nJpre, mi));
  TRY(dalloc(&c->trace.nI, mi));
  TRY(dalloc(&c->trace.nJ, mi));
  TRY(dalloc(&c->trace.rank, mi));
  TRY(dalloc(&c->trace.ind, mi));
  TRY(dalloc(&c->trace.rho, mi));
  TRY(dalloc(&c->trace.branch, mi));
  TRY(dalloc(&c->trace.route, mi));
  TRY(dalloc(&c->trace.sweeps, mi));
  TRY(dalloc(&c->replay.I, mi * kPMax));
  TRY(dalloc(&c->replay.J, mi * kPMax));
  TRY(dalloc(&c->replay.nI, mi));
  TRY(dalloc(&c->replay.nJ, mi));
  // DST tables and work (the Poisson solve only)
  if (poisson) {
    TRY(dst_plan(&c->dst, n, 2 * pm));
    TRY(dst_alloc(&c->dst));
  }
  TRY(tsqr_plan(&c->tsqr, n, pm));
  TRY(select_plan(&c->sel, n));
  if (c->selector == LRP_SEL_QDEIM) TRY(qdeim_plan(&c->qd, n, c->stream));
  TRY(rho_plan(&c->rho, n));
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&c->evfin, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->evit[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->evit[1], hipEventDisableTiming) != hipSuccess)
    return LRP_EDEVICE;
  if (poisson) {
    TRY(lambda_launch(c->lam, c->lam32, n, c->stream));
    TRY(dst_tables(&c->dst, c->stream));
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LRP_EDEVICE;
  return LRP_OK;
}

// ---------------------------------------------------------------- pass records
static thread_local PassRecord* g_rec = nullptr;  // record being filled on this thread

PassRecord*& pass_recorder() { return g_rec; }

void record_launch(PassRecord* r, const void* fn, dim3 grid, dim3 block, size_t shm, const void* args, size_t size) {
  if (grid.z != 1 || block.y != 1 || block.z != 1 || shm > UINT32_MAX || size > 65536) {
    r->bad = true;
    return;
  }
  const size_t off = (r->blob.size() + 15) & ~(size_t)15;
  r->blob.resize(off + size);
  memcpy(r->blob.data() + off, args, size);
  r->recs.push_back(LaunchRec{fn, grid.x, grid.y, block.x, (uint32_t)shm, (uint32_t)off, (uint32_t)size});
}

int enqueue_pass_kernels(lrp_ctx* c, int k);

int record_pass(lrp_ctx* c, int k, PassRecord* out) {
  *out = PassRecord{};
  if (c->profile) return LRP_EINVAL;
  // the general fiber build, valid for every rank (its results equal the narrow build's)
  const bool narrow = c->fiber_narrow;
  c->fiber_narrow = false;
  g_rec = out;
  const int rc = enqueue_pass_kernels(c, k);
  g_rec = nullptr;
  c->fiber_narrow = narrow;
  return (rc == LRP_OK && !out->bad && !out->recs.empty()) ? LRP_OK : LRP_EINVAL;
}

// ---------------------------------------------------------------- launch profile
static thread_local lrp_ctx* g_prof = nullptr;  // context recording a profile on this thread

ProfEvents prof_launch(hipStream_t s, int id) {
  lrp_ctx* c = g_prof;
  if (!c || c->stream != s) return {};
  while (c->prof_ev.size() < 2 * (c->prof_used + 1)) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return {};
    c->prof_ev.push_back(e);
  }
  if (c->prof_id.size() < c->prof_used + 1) c->prof_id.resize(c->prof_used + 1, -1);
  ProfEvents pe{c->prof_ev[2 * c->prof_used], c->prof_ev[2 * c->prof_used + 1]};
  c->prof_id[c->prof_used] = id;
  ++c->prof_used;
  return pe;
}

void prof_begin(hipStream_t s, int id) {
  lrp_ctx* c = g_prof;
  const ProfEvents pe = prof_launch(s, id);
  if (!pe.start) return;
  if (hipEventRecord(pe.start, s) != hipSuccess) return;
  c->prof_open = pe.stop;
}

void prof_end(hipStream_t s) {
  lrp_ctx* c = g_prof;
  if (!c || c->stream != s || !c->prof_open) return;
  (void)hipEventRecord(c->prof_open, s);
  c->prof_open = nullptr;
}

// Holds the stream for a bounded time (about 0.5 ms) so that the host enqueues the first
// stages before the device reaches them; launch gaps then do not enter the profile.
__global__ void k_hold(int iters) {
  for (int i = 0; i < iters; ++i) __builtin_amdgcn_s_sleep(127);
}

// Per-class time: every kernel launch carries start/stop events attached to its own dispatch
// (hipExtLaunchKernelGGL), so each record is the kernel's duration from the start to the end of
// its dispatch; copies are bracketed by events recorded around them.
static void prof_reduce(lrp_ctx* c) {
  for (int q = 0; q < K_COUNT; ++q) {
    c->prof_ms[q] = 0.0;
    c->prof_n[q] = 0;
  }
  for (size_t i = 0; i < c->prof_used; ++i) {
    const int id = c->prof_id[i];
    if (id < 0 || id >= K_COUNT) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]) != hipSuccess) continue;
    c->prof_ms[id] += ms;
    c->prof_n[id] += 1;
  }
}

// Pass k up to the stop decision: the set update from the previous candidates, fibers, the
// two thin QRs, the core, the factor products, rho and the indicator.
int enqueue_pass_update(lrp_ctx* c, int k) {
  const bool mixed = c->precision == LRP_MIXED;
  const int nb_new = (k + 1) & 1, nb_old = k & 1;
  const int64_t n = c->n;
  const int pm = c->r_max;
  hipStream_t s = c->stream;
  // selection from the previous iterate (candidates were computed right after it)
  SelectArgs sa{};
  sa.st = c->st;
  sa.pmax = pm;
  sa.trace = c->trace;
  sa.replay = c->replay;
  sa.n = n;
  sa.qd = c->selector == LRP_SEL_QDEIM ? c->qd.ctl : nullptr;
  sa.sampled = c->selector == LRP_SEL_LEVERAGE_SAMPLED;
  // the candidate slot depends only on the merge depth, which is fixed per context
  const int slot = c->sel.nlevels & 1;
  sa.cs[0] = c->sel.cand_s[slot][0];
  sa.cs[1] = c->sel.cand_s[slot][1];
  sa.ci[0] = c->sel.cand_i[slot][0];
  sa.ci[1] = c->sel.cand_i[slot][1];
  TRY(select_update(sa, s));
  FiberArgs fa{};
  fa.st = c->st;
  fa.Uh = mixed ? (const void*)c->Uh32 : (const void*)c->Uh;
  fa.Vh = mixed ? (const void*)c->Vh32 : (const void*)c->Vh;
  fa.ldh = n;
  fa.lam = mixed ? (const void*)c->lam32 : (const void*)c->lam;
  fa.C = mixed ? (void*)c->C32 : (void*)c->C;
  fa.Rt = mixed ? (void*)c->Rt32 : (void*)c->Rt;
  fa.ldc = n;
  fa.n = n;
  fa.matrix = c->matrix;
  fa.narrow = c->fiber_narrow ? 1 : 0;
  TRY(fiber_launch(fa, mixed, s));
  TsqrIO io{};
  io.st = c->st;
  io.nsides = 2;
  io.X[0] = fa.C;
  io.X[1] = fa.Rt;
  io.x_f32 = mixed;
  io.ldx = n;
  io.Q[0] = c->Q[0];
  io.Q[1] = c->Q[1];
  io.ldq = n;
  TRY(tsqr_run(c->tsqr, io, s));
  CoreArgs ca{};
  ca.st = c->st;
  ca.Q0 = c->Q[0];
  ca.Q1 = c->Q[1];
  ca.ldq = n;
  ca.R0 = tsqr_R(c->tsqr, 0);
  ca.R1 = tsqr_R(c->tsqr, 1);
  ca.pmax = pm;
  ca.Uhat = c->Uhat;
  ca.Vtil = c->Vtil;
  ca.nb = nb_new;
  ca.trace = c->trace;
  ca.maxiter = c->maxiter;
  TRY(core_launch(ca, false, s));
  ProdArgs pa{};
  pa.st = c->st;
  pa.Q[0] = c->Q[0];
  pa.Q[1] = c->Q[1];
  pa.ldq = n;
  pa.B[0] = c->Uhat;
  pa.B[1] = c->Vtil;
  pa.pmax = pm;
  pa.out[0] = c->Uit[nb_new];
  pa.out[1] = c->Vit[nb_new];
  pa.ldo = n;
  pa.n = n;
  pa.nb = nb_new;
  TRY(prod_launch(pa, s));
  RhoArgs ra{};
  ra.st = c->st;
  ra.Unew[0] = c->Uit[nb_new];
  ra.Unew[1] = c->Vit[nb_new];
  ra.Uold[0] = c->Uit[nb_old];
  ra.Uold[1] = c->Vit[nb_old];
  ra.ldu = n;
  ra.nb_new = nb_new;
  ra.nb_old = nb_old;
  ra.maxiter = c->maxiter;
  ra.trace = c->trace;
  TRY(rho_launch(c->rho, ra, s));
  EtaArgs ea{};
  ea.st = c->st;
  ea.Q0 = c->Q[0];
  ea.Q1 = c->Q[1];
  ea.ldq = n;
  ea.Uhat = c->Uhat;
  ea.Vtil = c->Vtil;
  ea.pmax = pm;
  ea.nb = nb_new;
  ea.maxiter = c->maxiter;
  ea.trace = c->trace;
  TRY(eta_launch(ea, s));
  return LRP_OK;
}

// Candidates of the next selection from the iterate U[0], U[1]: the leverage-score lists, and
// with QDEIM also the pivots of the column-pivoted QR (the leverage lists then give the
// safeguard index).
int enqueue_selection(lrp_ctx* c, const double* U[2]) {
  int fslot = 0;
  SampleOpts so{};
  so.sampled = c->selector == LRP_SEL_LEVERAGE_SAMPLED;
  so.rho = c->ls_rho;
  so.seed = c->seed;
  TRY(select_candidates(c->sel, c->st, U, c->n, c->stream, &fslot, so));
  if (c->selector == LRP_SEL_QDEIM) TRY(qdeim_launch(c->qd, c->st, U, c->n, c->r_max, c->stream));
  return LRP_OK;
}

// The tail of pass k: the selection candidates of the new iterate, for the selection that
// opens pass k+1 (every kernel returns at once once the stop flag is set).
int enqueue_pass_select(lrp_ctx* c, int k) {
  const int nb_new = (k + 1) & 1;
  const double* U[2] = {c->Uit[nb_new], c->Vit[nb_new]};
  return enqueue_selection(c, U);
}

int enqueue_pass_kernels(lrp_ctx* c, int k) {
  TRY(enqueue_pass_update(c, k));
  return enqueue_pass_select(c, k);
}

// Warm start from the initial guess U0, S0, V0 of Algorithm 4 (physical space, like the output):
// the truncated SVD of DST(U0) diag(S0) DST(V0)^T replaces the start from the right-hand side,
// computed in FP64 in both precisions through the iterate buffers of pass 0's new side (free
// until pass 0 writes them). A zero guess leaves the start from the right-hand side in place; the
// right-hand side is still factored first, which also detects a zero right-hand side.
int enqueue_guess(lrp_ctx* c) {
  const int64_t n = c->n;
  const int r0 = c->guess_r0;
  hipStream_t s = c->stream;
  TRY(scan_inputs_launch(c->st, c->guess_U, c->guess_ldu, c->guess_V, c->guess_ldv, c->guess_S, n, r0, s));
  TRY(guess_begin_launch(c->st, r0, s));
  DstArgs da{};
  da.st = c->st;
  da.X = c->guess_U;
  da.ldx = c->guess_ldu;
  da.ncols = r0;
  da.ncols_out = r0;
  da.Y = c->Uit[1];
  da.ldy = n;
  da.scale = c->guess_S;
  da.outscale = 1.0;
  TRY(dst_launch(c->dst, da, false, s));
  da.X = c->guess_V;
  da.ldx = c->guess_ldv;
  da.Y = c->Vit[1];
  da.scale = nullptr;
  TRY(dst_launch(c->dst, da, false, s));
  TsqrIO io{};
  io.st = c->st;
  io.nsides = 2;
  io.X[0] = c->Uit[1];
  io.X[1] = c->Vit[1];
  io.x_f32 = 0;
  io.ldx = n;
  io.Q[0] = c->Q[0];
  io.Q[1] = c->Q[1];
  io.ldq = n;
  TRY(tsqr_run(c->tsqr, io, s));
  CoreArgs ca{};
  ca.st = c->st;
  ca.R0 = tsqr_R(c->tsqr, 0);
  ca.R1 = tsqr_R(c->tsqr, 1);
  ca.pmax = c->r_max;
  ca.Uhat = c->Uhat;
  ca.Vtil = c->Vtil;
  ca.nb = 0;
  ca.trace = c->trace;
  ca.maxiter = c->maxiter;
  ca.guess = 1;
  TRY(core_launch(ca, true, s));
  ProdArgs pa{};
  pa.st = c->st;
  pa.Q[0] = c->Q[0];
  pa.Q[1] = c->Q[1];
  pa.ldq = n;
  pa.B[0] = c->Uhat;
  pa.B[1] = c->Vtil;
  pa.pmax = c->r_max;
  pa.out[0] = c->Uit[0];
  pa.out[1] = c->Vit[0];
  pa.ldo = n;
  pa.n = n;
  pa.nb = 0;
  pa.gate_guess = 1;
  return prod_launch(pa, s);
}

// Stage 1 of a solve: state reset, input scan, DST of the factors, warm start (from the
// right-hand side, then from the guess if one is set) and the candidates of the first selection.
// Asynchronous on the context's stream.
int enqueue_start(lrp_ctx* c, int rF, const double* U_F, int64_t ldu, const double* sigma_F,
                  const double* V_F, int64_t ldv) {
  const bool mixed = c->precision == LRP_MIXED;
  const int64_t n = c->n;
  const int pm = c->r_max;
  hipStream_t s = c->stream;
  const double eps = mixed ? std::max(c->tol, 1e-7) : c->tol;
  const double h = 1.0 / (double)(n + 1);
  c->fiber_narrow = rF <= 32;  // this solve's passes use the fiber build for its rank
  if (hipEventRecord(c->ev0, s) != hipSuccess) return LRP_EDEVICE;
  TRY(init_state_launch(c->st, rF, eps, c->tau, c->replay_n, s));
  TRY(scan_inputs_launch(c->st, U_F, ldu, V_F, ldv, sigma_F, n, rF, s));
  // spectral factors U^ = DST(U_F) diag(h^2 sigma), V^ = DST(V_F)
  DstArgs da{};
  da.X = U_F;
  da.ldx = ldu;
  da.ncols = rF;
  da.ncols_out = rF;
  da.ldy = n;
  da.st = c->st;
  da.scale = sigma_F;
  da.outscale = h * h;
  if (mixed)
    da.Yf = c->Uh32;
  else
    da.Y = c->Uh;
  TRY(dst_launch(c->dst, da, mixed, s));
  da.X = V_F;
  da.ldx = ldv;
  da.scale = nullptr;
  da.outscale = 1.0;
  da.Y = nullptr;
  da.Yf = nullptr;
  if (mixed)
    da.Yf = c->Vh32;
  else
    da.Y = c->Vh;
  TRY(dst_launch(c->dst, da, mixed, s));
  // warm start
  TsqrIO io{};
  io.st = c->st;
  io.nsides = 2;
  io.X[0] = mixed ? (const void*)c->Uh32 : (const void*)c->Uh;
  io.X[1] = mixed ? (const void*)c->Vh32 : (const void*)c->Vh;
  io.x_f32 = mixed;
  io.ldx = n;
  io.Q[0] = c->Q[0];
  io.Q[1] = c->Q[1];
  io.ldq = n;
  TRY(tsqr_run(c->tsqr, io, s));
  CoreArgs ca{};
  ca.st = c->st;
  ca.R0 = tsqr_R(c->tsqr, 0);
  ca.R1 = tsqr_R(c->tsqr, 1);
  ca.pmax = pm;
  ca.Uhat = c->Uhat;
  ca.Vtil = c->Vtil;
  ca.nb = 0;
  ca.trace = c->trace;
  ca.maxiter = c->maxiter;
  TRY(core_launch(ca, true, s));
  ProdArgs pa{};
  pa.st = c->st;
  pa.Q[0] = c->Q[0];
  pa.Q[1] = c->Q[1];
  pa.ldq = n;
  pa.B[0] = c->Uhat;
  pa.B[1] = c->Vtil;
  pa.pmax = pm;
  pa.out[0] = c->Uit[0];
  pa.out[1] = c->Vit[0];
  pa.ldo = n;
  pa.n = n;
  pa.nb = 0;
  TRY(prod_launch(pa, s));
  if (c->guess_r0 > 0) TRY(enqueue_guess(c));
  const double* U[2] = {c->Uit[0], c->Vit[0]};
  return enqueue_selection(c, U);
}

// Stage 1 of a Cross-DEIM run on a test matrix (Section 4.2): state reset, input scan, the
// guess copied into the iterate buffers of pass 0's new side, its truncated SVD (thin QRs of U0
// and V0, SVD of R_u R_v^T, truncated at r0 eps sigma_1) as the starting iterate, and the
// candidates of the first selection.
int enqueue_start_matrix(lrp_ctx* c, int r0, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0) {
  const int64_t n = c->n;
  hipStream_t s = c->stream;
  const double eps = c->precision == LRP_MIXED ? std::max(c->tol, 1e-7) : c->tol;
  if (hipEventRecord(c->ev0, s) != hipSuccess) return LRP_EDEVICE;
  TRY(init_state_launch(c->st, r0, eps, c->tau, c->replay_n, s));
  TRY(scan_inputs_launch(c->st, U0, ldu0, V0, ldv0, nullptr, n, r0, s));
  TRY(copy_cols_launch(c->st, U0, ldu0, c->Uit[1], n, n, r0, r0, s, 0));
  TRY(copy_cols_launch(c->st, V0, ldv0, c->Vit[1], n, n, r0, r0, s, 0));
  TsqrIO io{};
  io.st = c->st;
  io.nsides = 2;
  io.X[0] = c->Uit[1];
  io.X[1] = c->Vit[1];
  io.x_f32 = 0;
  io.ldx = n;
  io.Q[0] = c->Q[0];
  io.Q[1] = c->Q[1];
  io.ldq = n;
  TRY(tsqr_run(c->tsqr, io, s));
  CoreArgs ca{};
  ca.st = c->st;
  ca.R0 = tsqr_R(c->tsqr, 0);
  ca.R1 = tsqr_R(c->tsqr, 1);
  ca.pmax = c->r_max;
  ca.Uhat = c->Uhat;
  ca.Vtil = c->Vtil;
  ca.nb = 0;
  ca.trace = c->trace;
  ca.maxiter = c->maxiter;
  ca.zero_is_error = 1;
  TRY(core_launch(ca, true, s));
  ProdArgs pa{};
  pa.st = c->st;
  pa.Q[0] = c->Q[0];
  pa.Q[1] = c->Q[1];
  pa.ldq = n;
  pa.B[0] = c->Uhat;
  pa.B[1] = c->Vtil;
  pa.pmax = c->r_max;
  pa.out[0] = c->Uit[0];
  pa.out[1] = c->Vit[0];
  pa.ldo = n;
  pa.n = n;
  pa.nb = 0;
  TRY(prod_launch(pa, s));
  const double* U[2] = {c->Uit[0], c->Vit[0]};
  return enqueue_selection(c, U);
}

// Stage 3 of a test-matrix run: final truncation and the returned iterate copied into the
// caller's buffers (there is no transform back), state read-back.
int enqueue_finish_matrix(lrp_ctx* c, double* U_out, int64_t ldou, double* S_out, double* V_out, int64_t ldov) {
  const int64_t n = c->n;
  const int pm = c->r_max;
  hipStream_t s = c->stream;
  TRY(finalize_launch(c->st, S_out, pm, s));
  TRY(copy_ret_launch(c->st, c->Uit[0], c->Uit[1], n, U_out, ldou, pm, s));
  TRY(copy_ret_launch(c->st, c->Vit[0], c->Vit[1], n, V_out, ldov, pm, s));
  if (hipEventRecord(c->ev1, s) != hipSuccess) return LRP_EDEVICE;
  prof_begin(s, K_COPY);
  if (hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess)
    return LRP_EDEVICE;
  prof_end(s);
  return hipEventRecord(c->evfin, s) == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

// Pass k: the launch sequence depends only on the parity of k (which iterate buffer is
// new), so each parity is captured once into a hipGraph and replayed; if capture is not
// possible the kernels are launched directly.
static int enqueue_captured(lrp_ctx* c, int k, hipGraphExec_t* slot, int (*fn)(lrp_ctx*, int)) {
  if (c->use_graphs && !c->profile && !*slot) {
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    const int rc = ok ? fn(c, k) : LRP_EDEVICE;
    ok = (hipStreamEndCapture(c->stream, &g) == hipSuccess) && ok && rc == LRP_OK;
    if (ok) ok = hipGraphInstantiate(slot, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
      *slot = nullptr;
      c->use_graphs = false;
      (void)hipGetLastError();
    }
  }
  if (c->use_graphs && !c->profile && *slot)
    return hipGraphLaunch(*slot, c->stream) == hipSuccess ? LRP_OK : LRP_EDEVICE;
  return fn(c, k);
}

// The captured pass for the fiber build of the current solve and the parity of k.
static int graph_slot(const lrp_ctx* c, int k) { return (c->fiber_narrow ? 2 : 0) | (k & 1); }

int enqueue_pass(lrp_ctx* c, int k) {
  return enqueue_captured(c, k, &c->gexec[graph_slot(c, k)], enqueue_pass_kernels);
}

// Pass k with the stop flag read between its two parts: the update part (captured per parity),
// the flag copy and its event, then the candidate selection (captured per parity).
int enqueue_pass_polled(lrp_ctx* c, int k) {
  TRY(enqueue_captured(c, k, &c->gexec_upd[graph_slot(c, k)], enqueue_pass_update));
  TRY(enqueue_poll(c, k));
  return enqueue_captured(c, k, &c->gexec_sel[k & 1], enqueue_pass_select);
}

// After pass k: copy the stop flag to pinned memory and mark the point with an event.
// The stop flag into its pinned host slot. A one-thread kernel rather than a copy, so that the
// pass boundary stays on the compute queue (a copy may go to a DMA engine, and the next pass
// would wait for the hand-over between the two).
__global__ void k_flag_copy(const int* src, int* dst) {
  if (threadIdx.x == 0) {
    *dst = *src;
    __threadfence_system();
  }
}

int enqueue_poll(lrp_ctx* c, int k) {
  const int slot = k & 1;
  LRP_LAUNCH(K_COPY, k_flag_copy, dim3(1), dim3(64), 0, c->stream, &c->st->done, &c->done_host[slot]);
  TRY(launch_status());
  return hipEventRecord(c->evit[slot], c->stream) == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

// Stage 3: final truncation, DST back into the caller's buffers, state read-back.
int enqueue_finish(lrp_ctx* c, double* U_out, int64_t ldou, double* S_out, double* V_out, int64_t ldov) {
  const bool mixed = c->precision == LRP_MIXED;
  const int64_t n = c->n;
  const int pm = c->r_max;
  hipStream_t s = c->stream;
  TRY(finalize_launch(c->st, S_out, pm, s));
  DstArgs db{};
  db.st = c->st;
  db.pick_ret = 1;
  db.X = c->Uit[0];
  db.X1 = c->Uit[1];
  db.ldx = n;
  db.Y = U_out;
  db.ldy = ldou;
  db.ncols = 0;
  db.ncols_out = pm;
  db.outscale = 1.0;
  TRY(dst_launch(c->dst, db, mixed, s));
  db.X = c->Vit[0];
  db.X1 = c->Vit[1];
  db.Y = V_out;
  db.ldy = ldov;
  TRY(dst_launch(c->dst, db, mixed, s));
  if (hipEventRecord(c->ev1, s) != hipSuccess) return LRP_EDEVICE;
  prof_begin(s, K_COPY);
  if (hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess)
    return LRP_EDEVICE;
  prof_end(s);
  return hipEventRecord(c->evfin, s) == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

// Stage 4 (host, after evfin completed): the report.
int collect(lrp_ctx* c, int32_t* r_out, lrp_info* info) {
  const DevState& h_st = *c->st_host;
  c->solved = true;
  const int status = h_st.status;
  if (status < 0) {  // no result; report how far the solve got
    if (info) {
      *info = lrp_info{};
      info->status = status;
      info->iters = h_st.k;
    }
    return status;
  }
  if (r_out) *r_out = h_st.r_final;
  if (info) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    info->status = status;
    info->iters = h_st.k;
    info->rank = h_st.r_final;
    info->nI = h_st.nIb[h_st.ret];
    info->nJ = h_st.nJb[h_st.ret];
    info->rho = h_st.rhob[h_st.ret];
    info->indicator = h_st.indb[h_st.ret];
    info->ms = ms;
  }
  return status;
}

int check_solve_args(int64_t n, int r_max, int32_t r_F, const double* U_F, int64_t ldu, const double* sigma_F,
                     const double* V_F, int64_t ldv, const double* U_out, int64_t ldou, const double* S_out,
                     const double* V_out, int64_t ldov) {
  if (!U_F || !V_F || !U_out || !S_out || !V_out) return LRP_EINVAL;
  if (r_F < 1 || r_F > r_max) return LRP_EINVAL;
  if (ldu < n || ldv < n || ldou < n || ldov < n) return LRP_EINVAL;
  // sigma_F may be null (a guess without weights): it then overlaps nothing
  const Range in[3] = {span(U_F, n, ldu, r_F, 8), span(V_F, n, ldv, r_F, 8),
                       sigma_F ? span(sigma_F, r_F, r_F, 1, 8) : Range{0, 0}};
  const Range out[3] = {span(U_out, n, ldou, r_max, 8), span(V_out, n, ldov, r_max, 8), span(S_out, r_max, r_max, 1, 8)};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      if (overlap(out[a], in[b])) return LRP_EINVAL;
    for (int b = a + 1; b < 3; ++b)
      if (overlap(out[a], out[b])) return LRP_EINVAL;
  }
  return LRP_OK;
}

// Device bytes of a context, mirroring create_impl and the plans (up to allocation rounding).
int64_t context_bytes(int64_t n, int pm, int maxiter, bool mixed) {
  const int64_t np = n * pm;
  int64_t b = (int64_t)sizeof(DevState) + 12 * n;                  // state, lambda (FP64 + FP32)
  b += mixed ? 4 * 4 * np : 4 * 8 * np;                            // U^, V^, C, R^T
  b += 6 * 8 * np;                                                 // Q, Z, two iterates per side
  b += 2 * 8 * (int64_t)pm * pm;                                   // U^, V~ coefficients
  b += (int64_t)maxiter * (2 * kPMax * 4 + 8 * 4 + 2 * 8);         // trace
  b += (int64_t)maxiter * (2 * kPMax * 4 + 2 * 4);                 // replay sets
  DstPlan dp{};
  if (dst_plan(&dp, n, 2 * pm) == LRP_OK) b += dst_bytes(dp);
  int64_t rows = n, br = kTsqrRows;                                // TSQR tree, two sides
  const int g = kTsqrRows / pm;
  for (int L = 0; L < kMaxLevels; ++L) {
    const int64_t nb = (rows + br - 1) / br;
    b += 2 * (2 * rows * pm * 8 + nb * pm * 8 + nb * pm * pm * 8);
    if (nb == 1) break;
    rows = nb * pm;
    br = (int64_t)g * pm;
  }
  const int64_t nsel = (n + kSelRows - 1) / kSelRows;              // selection
  b += 2 * (8 * n + 8 * nsel + 2 * nsel * kPMax * 12) + 16;
  const int64_t chunks = (n + 255) / 256, per = (chunks + 511) / 512;  // rho
  b += ((chunks + per - 1) / per) * 2 * kPMax * kPMax * 8 + 4 * kPMax * kPMax * 8;
  return b;
}

int solve_impl(lrp_ctx* c, int rF, const double* U_F, int64_t ldu, const double* sigma_F,
               const double* V_F, int64_t ldv, double* U_out, int64_t ldou, double* S_out,
               double* V_out, int64_t ldov, int32_t* r_out, lrp_info* info) {
  struct ProfScope {  // ends the recording on every return path
    lrp_ctx* c;
    ~ProfScope() {
      if (c) g_prof = nullptr;
    }
  } scope{c->profile ? c : nullptr};
  if (c->profile) {
    c->prof_used = 0;
    hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, c->stream, 150);
    if (launch_status() != LRP_OK) return LRP_EDEVICE;
    g_prof = c;
    for (int q = 0; q < 16; ++q)  // empty launches: the floor of a kernel's dispatch duration
      LRP_LAUNCH(K_EMPTY, k_hold, dim3(1), dim3(64), 0, c->stream, 0);
    if (launch_status() != LRP_OK) return LRP_EDEVICE;
  }
  struct GuessScope {  // the guess applies to this solve only
    lrp_ctx* c;
    ~GuessScope() { c->guess_r0 = 0; }
  } gscope{c};
  if (c->matrix == LRP_MAT_POISSON)
    TRY(enqueue_start(c, rF, U_F, ldu, sigma_F, V_F, ldv));
  else
    TRY(enqueue_start_matrix(c, rF, U_F, ldu, V_F, ldv));
  // passes; the stop flag of pass k is copied right after its decision, and the host reads it
  // while the device runs pass k's candidate selection, so no pass is enqueued after the stop
  // (only the selection of the last pass, whose kernels return at once)
  for (int k = 0; k < c->maxiter; ++k) {
    TRY(enqueue_pass_polled(c, k));
    if (hipEventSynchronize(c->evit[k & 1]) != hipSuccess) return LRP_EDEVICE;
    if (c->done_host[k & 1]) break;
  }
  if (c->matrix == LRP_MAT_POISSON)
    TRY(enqueue_finish(c, U_out, ldou, S_out, V_out, ldov));
  else
    TRY(enqueue_finish_matrix(c, U_out, ldou, S_out, V_out, ldov));
  if (hipEventSynchronize(c->evfin) != hipSuccess) return LRP_EDEVICE;
  if (c->profile) {
    g_prof = nullptr;
    prof_reduce(c);
  }
  return collect(c, r_out, info);
}

}  // namespace lrp

extern "C" {

const char* lrp_strerror(int code) {
  switch (code) {
    case LRP_OK: return "converged";
    case LRP_NOT_CONVERGED: return "maxiter passes made without meeting the tolerance";
    case LRP_STAGNATED: return "index sets repeated (fixed point); last distinct iterate returned";
    case LRP_EINVAL: return "invalid argument";
    case LRP_ENOMEM: return "device allocation failed";
    case LRP_EDEVICE: return "HIP runtime error";
    case LRP_ENUMERIC: return "non-finite input or degenerate fibers";
    case LRP_ESIZE: return "problem larger than the fixed workspace of the allocation-free entry point";
    default: return "unknown status";
  }
}

int lrp_create(lrp_ctx** ctx, int64_t n, int32_t r_max, double tol, const lrp_opts* opts) {
  if (!ctx) return LRP_EINVAL;
  *ctx = nullptr;
  lrp_opts o{};
  if (opts) o = *opts;
  if (o.matrix != LRP_MAT_POISSON && o.matrix != LRP_MAT_HILBERT && o.matrix != LRP_MAT_K) return LRP_EINVAL;
  if (o.matrix == LRP_MAT_POISSON) {
    // n + 1 a power of two up to 2^23, or any other n up to 2^22 - 1 (Bluestein DST)
    if (n < 2 || n + 1 > (int64_t(1) << 23) || (!pow2(n + 1) && n + 1 > (int64_t(1) << 22))) return LRP_EINVAL;
  } else if (n < 2 || n > (int64_t(1) << 23)) {
    return LRP_EINVAL;
  }
  if (r_max < 1 || r_max > kPMax || r_max > n) return LRP_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return LRP_EINVAL;
  if (o.maxiter < 0 || o.maxiter > 1000) return LRP_EINVAL;
  if (o.precision != LRP_FP64 && o.precision != LRP_MIXED) return LRP_EINVAL;
  if (!(o.prune_tau >= 0.0) || o.prune_tau >= 1.0) return LRP_EINVAL;
  if ((o.flags & ~LRP_FLAG_PROFILE) ||
      (o.selector != LRP_SEL_LEVERAGE && o.selector != LRP_SEL_QDEIM && o.selector != LRP_SEL_LEVERAGE_SAMPLED))
    return LRP_EINVAL;
  if (!(o.ls_oversampling >= 0.0) || !std::isfinite(o.ls_oversampling)) return LRP_EINVAL;
  if (o.reserved != 0) return LRP_EINVAL;
  lrp_ctx* c = new (std::nothrow) lrp_ctx();
  if (!c) return LRP_ENOMEM;
  c->n = n;
  c->r_max = r_max;
  c->tol = tol;
  c->maxiter = o.maxiter == 0 ? 20 : o.maxiter;
  c->precision = o.precision;
  c->tau = o.prune_tau > 0.0 ? o.prune_tau : (o.precision == LRP_MIXED ? 1e-7 : 1e-12);
  c->profile = (o.flags & LRP_FLAG_PROFILE) != 0;
  c->selector = o.selector;
  c->matrix = o.matrix;
  c->ls_rho = o.ls_oversampling > 0.0 ? o.ls_oversampling : 2.0;
  c->seed = o.seed;
  if (o.stream) {
    c->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return LRP_EDEVICE;
    }
    c->own_stream = true;
  }
  const int rc = create_impl(c);
  if (rc != LRP_OK) {
    free_ctx(c);
    return rc;
  }
  *ctx = c;
  return LRP_OK;
}

int lrp_solve(lrp_ctx* c, int32_t r_F, const double* U_F, int64_t ldu, const double* sigma_F,
              const double* V_F, int64_t ldv, double* U_out, int64_t ldou, double* S_out,
              double* V_out, int64_t ldov, int32_t* r_out, lrp_info* info) {
  if (!c || !r_out || !sigma_F || c->matrix != LRP_MAT_POISSON) return LRP_EINVAL;
  const int rc = check_solve_args(c->n, c->r_max, r_F, U_F, ldu, sigma_F, V_F, ldv, U_out, ldou, S_out, V_out, ldov);
  if (rc != LRP_OK) return rc;
  c->solved = false;
  return solve_impl(c, r_F, U_F, ldu, sigma_F, V_F, ldv, U_out, ldou, S_out, V_out, ldov, r_out, info);
}

int lrp_cross_solve(lrp_ctx* c, int32_t r0, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0,
                    double* U_out, int64_t ldou, double* S_out, double* V_out, int64_t ldov, int32_t* r_out,
                    lrp_info* info) {
  if (!c || !r_out || c->matrix == LRP_MAT_POISSON) return LRP_EINVAL;
  // the guess takes the place of the right-hand side factors (no weights)
  const int rc = check_solve_args(c->n, c->r_max, r0, U0, ldu0, nullptr, V0, ldv0, U_out, ldou, S_out, V_out, ldov);
  if (rc != LRP_OK) return rc;
  c->solved = false;
  c->guess_r0 = 0;
  return solve_impl(c, r0, U0, ldu0, nullptr, V0, ldv0, U_out, ldou, S_out, V_out, ldov, r_out, info);
}

int64_t lrp_context_bytes(int64_t n, int32_t r_max, int32_t maxiter, int32_t precision) {
  if (n < 2 || n + 1 > (int64_t(1) << 23) || (!pow2(n + 1) && n + 1 > (int64_t(1) << 22))) return 0;
  if (r_max < 1 || r_max > kPMax || r_max > n) return 0;
  if (maxiter < 0 || (precision != LRP_FP64 && precision != LRP_MIXED)) return 0;
  return context_bytes(n, r_max, maxiter == 0 ? 20 : maxiter, precision == LRP_MIXED);
}

int lrp_get_profile(const lrp_ctx* c, int32_t* count, lrp_kernel_time* out) {
  static const char* const names[K_COUNT] = {
      "k_init_state", "k_scan", "k_dst_single", "k_dst_pass1", "k_dst_pass2", "k_fiber",
      "k_tsqr_factor", "k_tsqr_apply", "k_core_warm", "k_core", "k_prod", "k_pi", "k_gmax",
      "k_topk_block", "k_topk_merge", "k_select", "k_rho_a", "k_rho_b", "k_rho_reduce",
      "k_rho_final", "k_eta", "k_finalize", "copy", "empty kernel", "k_qdeim_step"};
  if (!c || !count || *count < 0 || (*count > 0 && !out)) return LRP_EINVAL;
  if (!c->profile || !c->solved) {
    *count = 0;
    return c->profile ? LRP_EINVAL : LRP_OK;
  }
  int m = 0;
  for (int q = 0; q < K_COUNT; ++q) {
    if (c->prof_n[q] == 0) continue;
    if (m < *count) {
      out[m].name = names[q];
      out[m].launches = c->prof_n[q];
      out[m].ms = c->prof_ms[q];
    }
    ++m;
  }
  *count = m;
  return LRP_OK;
}

int lrp_get_index_sets(const lrp_ctx* c, int64_t* I, int32_t* nI, int64_t* J, int32_t* nJ) {
  if (!c || !c->solved || !I || !nI || !J || !nJ) return LRP_EINVAL;
  const DevState& s = *c->st_host;
  const int b = s.ret;
  *nI = s.nIb[b];
  *nJ = s.nJb[b];
  for (int q = 0; q < s.nIb[b]; ++q) I[q] = s.Ib[b][q];
  for (int q = 0; q < s.nJb[b]; ++q) J[q] = s.Jb[b][q];
  return LRP_OK;
}

int lrp_get_trace(const lrp_ctx* c, int32_t* count, int32_t* Ipre, int32_t* nIpre, int32_t* Jpre,
                  int32_t* nJpre, int32_t* nI, int32_t* nJ, int32_t* rank, double* indicator,
                  double* rho, int32_t* branch, int32_t* route, int32_t* sweeps) {
  if (!c || !c->solved || !count || *count < 0) return LRP_EINVAL;
  const int avail = std::min(c->st_host->k, c->maxiter);
  const int m = std::min(*count, avail);
  *count = m;
  if (m == 0) return LRP_OK;
  const TraceBuf& t = c->trace;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return dst ? hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) : hipSuccess;
  };
  if (Ipre && c->r_max > 0) {
    for (int k = 0; k < m; ++k)
      if (hipMemcpy(Ipre + (size_t)k * c->r_max, t.Ipre + (size_t)k * kPMax, sizeof(int) * c->r_max,
                    hipMemcpyDeviceToHost) != hipSuccess)
        return LRP_EDEVICE;
  }
  if (Jpre && c->r_max > 0) {
    for (int k = 0; k < m; ++k)
      if (hipMemcpy(Jpre + (size_t)k * c->r_max, t.Jpre + (size_t)k * kPMax, sizeof(int) * c->r_max,
                    hipMemcpyDeviceToHost) != hipSuccess)
        return LRP_EDEVICE;
  }
  if (cp(nIpre, t.nIpre, sizeof(int) * m) != hipSuccess || cp(nJpre, t.nJpre, sizeof(int) * m) != hipSuccess ||
      cp(nI, t.nI, sizeof(int) * m) != hipSuccess || cp(nJ, t.nJ, sizeof(int) * m) != hipSuccess ||
      cp(rank, t.rank, sizeof(int) * m) != hipSuccess || cp(indicator, t.ind, sizeof(double) * m) != hipSuccess ||
      cp(rho, t.rho, sizeof(double) * m) != hipSuccess || cp(branch, t.branch, sizeof(int) * m) != hipSuccess ||
      cp(route, t.route, sizeof(int) * m) != hipSuccess || cp(sweeps, t.sweeps, sizeof(int) * m) != hipSuccess)
    return LRP_EDEVICE;
  return LRP_OK;
}

int lrp_set_guess(lrp_ctx* c, int32_t r0, const double* U0, int64_t ldu0, const double* S0, const double* V0,
                  int64_t ldv0) {
  if (!c || r0 < 0 || r0 > c->r_max) return LRP_EINVAL;
  if (r0 == 0) {
    c->guess_r0 = 0;
    return LRP_OK;
  }
  if (!U0 || !V0 || ldu0 < c->n || ldv0 < c->n) return LRP_EINVAL;
  c->guess_r0 = r0;
  c->guess_U = U0;
  c->guess_ldu = ldu0;
  c->guess_S = S0;
  c->guess_V = V0;
  c->guess_ldv = ldv0;
  return LRP_OK;
}

int lrp_set_index_sets(lrp_ctx* c, int32_t npasses, const int64_t* I, const int32_t* nI, const int64_t* J,
                       const int32_t* nJ) {
  if (!c || npasses < 0 || npasses > c->maxiter) return LRP_EINVAL;
  if (npasses == 0) {
    c->replay_n = 0;
    return LRP_OK;
  }
  if (!I || !nI || !J || !nJ) return LRP_EINVAL;
  const int rm = c->r_max;
  std::vector<int> hI((size_t)npasses * kPMax, -1), hJ((size_t)npasses * kPMax, -1);
  std::vector<int> hnI(npasses), hnJ(npasses);
  for (int k = 0; k < npasses; ++k) {
    for (int side = 0; side < 2; ++side) {
      const int cnt = side == 0 ? nI[k] : nJ[k];
      const int64_t* src = (side == 0 ? I : J) + (size_t)k * rm;
      int* dst = (side == 0 ? hI.data() : hJ.data()) + (size_t)k * kPMax;
      if (cnt < 1 || cnt > rm) return LRP_EINVAL;
      for (int q = 0; q < cnt; ++q) {
        if (src[q] < 0 || src[q] >= c->n) return LRP_EINVAL;
        for (int u = 0; u < q; ++u)
          if (src[u] == src[q]) return LRP_EINVAL;
        dst[q] = (int)src[q];
      }
      (side == 0 ? hnI : hnJ)[k] = cnt;
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LRP_EDEVICE;
  if (hipMemcpy(c->replay.I, hI.data(), sizeof(int) * hI.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->replay.J, hJ.data(), sizeof(int) * hJ.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->replay.nI, hnI.data(), sizeof(int) * npasses, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->replay.nJ, hnJ.data(), sizeof(int) * npasses, hipMemcpyHostToDevice) != hipSuccess)
    return LRP_EDEVICE;
  c->replay_n = npasses;
  return LRP_OK;
}

int lrp_destroy(lrp_ctx* c) {
  if (!c) return LRP_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  return LRP_OK;
}

int lrp_dst1(lrp_ctx* c, int32_t ncols, const double* X, int64_t ldx, double* Y, int64_t ldy,
             const double* scale, double mul, int32_t precision) {
  if (!c || !X || !Y || ncols < 1 || ncols > 2 * c->r_max) return LRP_EINVAL;
  if (ldx < c->n || ldy < c->n) return LRP_EINVAL;
  if (precision != LRP_FP64 && precision != LRP_MIXED) return LRP_EINVAL;
  if (overlap(span(X, c->n, ldx, ncols, 8), span(Y, c->n, ldy, ncols, 8))) return LRP_EINVAL;
  DstArgs a{};
  a.X = X;
  a.ldx = ldx;
  a.Y = Y;
  a.ldy = ldy;
  a.ncols = ncols;
  a.ncols_out = ncols;
  a.scale = scale;
  a.outscale = mul;
  return dst_launch(c->dst, a, precision == LRP_MIXED, c->stream);
}

int lrp_tsqr(lrp_ctx* c, int32_t ncols, const double* A, int64_t lda, double* Q, int64_t ldq,
             double* R, int64_t ldr) {
  if (!c || !A || !Q || !R || ncols < 1 || ncols > c->r_max) return LRP_EINVAL;
  if (lda < c->n || ldq < c->n || ldr < ncols) return LRP_EINVAL;
  if (overlap(span(A, c->n, lda, ncols, 8), span(Q, c->n, ldq, ncols, 8))) return LRP_EINVAL;
  TsqrIO io{};
  io.st = nullptr;
  io.ncols[0] = ncols;
  io.ncols[1] = 0;
  io.nsides = 1;
  io.X[0] = A;
  io.x_f32 = 0;
  io.ldx = lda;
  io.Q[0] = Q;
  io.ldq = ldq;
  TRY(tsqr_run(c->tsqr, io, c->stream));
  if (hipMemcpy2DAsync(R, sizeof(double) * ldr, tsqr_R(c->tsqr, 0), sizeof(double) * c->r_max,
                       sizeof(double) * ncols, ncols, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return LRP_EDEVICE;
  return hipStreamSynchronize(c->stream) == hipSuccess ? LRP_OK : LRP_EDEVICE;
}

}  // extern "C"
