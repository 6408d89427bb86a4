// The library context (one solve shape) and the stages of a solve, shared by the plain
// solve entry point and the serving scheduler.
#pragma once

#include <vector>

#include "lrp_kernels.h"

struct lrp_ctx {
  using DevState = lrp::DevState;
  using TraceBuf = lrp::TraceBuf;
  using DstPlan = lrp::DstPlan;
  using TsqrPlan = lrp::TsqrPlan;
  using SelectPlan = lrp::SelectPlan;
  using RhoPlan = lrp::RhoPlan;

  int64_t n = 0;
  int r_max = 0;
  double tol = 0.0;
  int maxiter = 20;
  int precision = LRP_FP64;
  double tau = 1e-12;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;

  DevState* st = nullptr;
  DevState* st_host = nullptr;  // pinned
  int* done_host = nullptr;     // pinned, 2 slots
  double* lam = nullptr;
  float* lam32 = nullptr;
  double *Uh = nullptr, *Vh = nullptr;
  float *Uh32 = nullptr, *Vh32 = nullptr;
  double *C = nullptr, *Rt = nullptr;
  float *C32 = nullptr, *Rt32 = nullptr;
  double* Q[2] = {nullptr, nullptr};
  double* Uit[2] = {nullptr, nullptr};
  double* Vit[2] = {nullptr, nullptr};
  double *Uhat = nullptr, *Vtil = nullptr;
  TraceBuf trace{};
  // replay (lrp_set_index_sets): sets of passes 0 .. replay_n-1, device copies
  lrp::ReplayBuf replay{};
  int replay_n = 0;
  // initial guess of the next solve (lrp_set_guess); r0 = 0: none
  int guess_r0 = 0;
  const double *guess_U = nullptr, *guess_S = nullptr, *guess_V = nullptr;
  int64_t guess_ldu = 0, guess_ldv = 0;
  DstPlan dst{};
  TsqrPlan tsqr{};
  SelectPlan sel{};
  lrp::QdeimPlan qd{};  // QDEIM selection only
  int selector = LRP_SEL_LEVERAGE;
  int matrix = LRP_MAT_POISSON;  // the matrix G of the cross approximation
  double ls_rho = 2.0;  // sampled leverage scores: p_i = min(1, ls_rho pi_i)
  uint64_t seed = 0;
  RhoPlan rho{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evfin = nullptr, evit[2] = {nullptr, nullptr};
  // captured passes, per fiber build (narrow: rank <= 32) and parity: index 2 narrow + parity
  hipGraphExec_t gexec[4] = {};      // the whole pass (serving loop)
  hipGraphExec_t gexec_upd[4] = {};  // the split pass (solve): update part
  hipGraphExec_t gexec_sel[2] = {};  // selection part, per parity
  bool fiber_narrow = false;         // the right-hand side of the current solve has rank <= 32
  bool use_graphs = true;
  bool solved = false;
  // optional per-kernel timing (LRP_FLAG_PROFILE): events recorded before every launch
  bool profile = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_id;
  hipEvent_t prof_open = nullptr;  // stop event of the copy being timed
  size_t prof_used = 0;
  double prof_ms[lrp::K_COUNT] = {};
  int prof_n[lrp::K_COUNT] = {};
};


namespace lrp {

int create_impl(lrp_ctx* c);
void free_ctx(lrp_ctx* c);
// argument checks shared by lrp_solve and the server (no device work)
int check_solve_args(int64_t n, int r_max, int32_t r_F, const double* U_F, int64_t ldu, const double* sigma_F,
                     const double* V_F, int64_t ldv, const double* U_out, int64_t ldou, const double* S_out,
                     const double* V_out, int64_t ldov);
// asynchronous stages on the context's stream
int enqueue_selection(lrp_ctx* c, const double* U[2]);
int enqueue_start(lrp_ctx* c, int rF, const double* U_F, int64_t ldu, const double* sigma_F,
                  const double* V_F, int64_t ldv);
int enqueue_pass(lrp_ctx* c, int k);
// The launches of pass k (they depend on its parity only) recorded, not made: for passes of
// several requests run as one launch per stage. LRP_EINVAL if a launch has no grouped form.
int record_pass(lrp_ctx* c, int k, PassRecord* out);
int enqueue_poll(lrp_ctx* c, int k);
int enqueue_finish(lrp_ctx* c, double* U_out, int64_t ldou, double* S_out, double* V_out, int64_t ldov);
int collect(lrp_ctx* c, int32_t* r_out, lrp_info* info);
// device bytes of a context of this shape
int64_t context_bytes(int64_t n, int r_max, int maxiter, bool mixed);

}  // namespace lrp
