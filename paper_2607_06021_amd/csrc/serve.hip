// Serving: a queue of Poisson solves with continuous admission (the lrp_server_* ABI).
//
// A scheduler thread owns a pool of contexts ("slots"), each with its own non-blocking HIP
// stream. Requests are admitted in arrival order as soon as a slot of their shape is idle,
// or a new one fits in the device-memory budget (idle slots of other shapes are freed, least
// recently used first, to make room). An admitted request runs the same stages as lrp_solve
// -- start, passes, finish -- but the scheduler advances all active requests together: it
// enqueues the next pass of a request while at most two of its passes are unchecked, reads
// each pass's stop flag through an event query (never blocking), and enqueues the finish
// stage once the flag is set or maxiter passes were made. A finished request frees its slot
// at once for the next one.
//
// Same-stage grouping: requests whose passes make the same launches (one shape) form a group
// with a stream of its own. Two or more of its requests that take their next pass together run
// it as one launch per stage: a captured graph per group size whose kernels take a table of the
// requests' argument areas and run request z's arguments in workgroup z (the grouped kernels of
// lrp_kernels.h). Once three or more of a group's requests run, the scheduler aligns them: a
// pass is launched when one of them has nothing in flight, and then for every one that may take
// a pass (a new request after its start stage), so requests that started apart end up in the
// same launches. With fewer running, each request takes its passes on its own stream, two
// passes deep, as without grouping. Start and finish stages stay on the slots' streams; work
// that follows work on another stream waits for it by an event.
// A request's kernels, arguments, grids and reductions are exactly those of a solo lrp_solve,
// so its result does not depend on what else is in flight or in its group.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "ctx.h"
#include "serve_policy.h"

using namespace lrp;

namespace {

using Clock = std::chrono::steady_clock;

struct Key {
  int64_t n;
  int r_max;
  double tol;
  int maxiter;
  int precision;
  bool operator==(const Key& o) const {
    return n == o.n && r_max == o.r_max && tol == o.tol && maxiter == o.maxiter && precision == o.precision;
  }
};

struct Job {
  int64_t ticket = 0;
  lrp_request req{};
  Key key{};
  int64_t bytes = 0;
  Clock::time_point t_submit, t_admit, t_done;
  bool admitted = false;
  bool done = false;
  int status = 0;
  int rank = 0;
  lrp_info info{};
};

struct Slot {
  lrp_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  Key key{};
  int64_t bytes = 0;
  Job* job = nullptr;  // null: idle
  int phase = 0;       // 0: start not enqueued, 1: passes, 2: finishing
  int k = 0;           // passes enqueued
  int checked = 0;     // passes whose stop flag has been read
  bool stop = false;
  uint64_t last_used = 0;
  // grouped passes
  int group = -1;            // index of the slot's group; -1: passes on the slot's stream
  char* area = nullptr;      // device: the pass's argument blocks, parity 0 then parity 1
  bool moved = false;        // the request's last pass ran on the group's stream
  uint64_t last_launch = 0;  // the group launch of that pass (0: its own stream)
  hipEvent_t ev_start = nullptr;  // end of the start stage (a first pass may run grouped)
};

// Largest group: the largest number of active requests.
constexpr int kMaxGroup = 64;

// Requests whose passes make the same launches (grids, kernels, argument offsets).
struct Group {
  std::vector<LaunchRec> recs;
  size_t area = 0;                    // bytes of one parity's argument blocks
  hipStream_t stream = nullptr;
  const char** table = nullptr;       // device: kTable entries (see GroupTable)
  hipGraphExec_t exec[kMaxGroup] = {};  // by group size - 1, captured on first use
  bool broken = false;                // a graph could not be built: passes run per slot
};

// The table of one grouped launch, per request z of the group: the base of its argument blocks
// (the GroupRef bases), its device stop flag and the pinned host slot the flag is copied to.
struct GroupTable {
  const char* base[kMaxGroup];
  const int* src[kMaxGroup];
  int* dst[kMaxGroup];
};
constexpr int kTable = 3 * kMaxGroup;

// The table of the group's next launch (written on the group's stream before its graph).
__global__ void k_group_table(const char** table, GroupTable g, int count) {
  const int t = threadIdx.x;
  if (t < count) {
    table[t] = g.base[t];
    table[kMaxGroup + t] = reinterpret_cast<const char*>(g.src[t]);
    table[2 * kMaxGroup + t] = reinterpret_cast<const char*>(g.dst[t]);
  }
}

// The last node of a grouped pass: each request's stop flag into its pinned host slot.
__global__ void k_group_poll(const char* const* table, int count) {
  const int t = threadIdx.x;
  if (t < count) {
    const int* src = reinterpret_cast<const int*>(table[kMaxGroup + t]);
    int* dst = reinterpret_cast<int*>(const_cast<char*>(table[2 * kMaxGroup + t]));
    *dst = *src;
  }
  __threadfence_system();
}

}  // namespace

struct lrp_server {
  int device = 0;
  int64_t budget = 0;
  int max_active = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::map<int64_t, Job*> jobs;
  std::vector<Slot> slots;  // touched only by the scheduler thread (sizes read under mu)
  std::vector<Group> groups;  // scheduler thread only
  std::vector<std::vector<Slot*>> members;  // per group, rebuilt each tick (scheduler thread)
  bool grouping = true;       // set under mu while nothing is queued or active
  bool grouping_tick = true;  // the scheduler's copy for the current tick
  int64_t passes = 0, pass_launches = 0;  // under mu
  uint64_t launch_seq = 0;                // group launches made (scheduler thread)
  int64_t bytes_in_use = 0;
  int64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, failed = 0, active = 0;
  bool stopping = false;
  uint64_t tick = 0;
  std::thread th;
};

namespace {

void finish_job(lrp_server* s, Job* j, int status, int rank, const lrp_info* info) {
  std::lock_guard<std::mutex> g(s->mu);
  j->status = status;
  j->rank = rank;
  if (info) j->info = *info;
  j->info.status = status;
  j->t_done = Clock::now();
  j->done = true;
  if (status < 0)
    ++s->failed;
  else
    ++s->completed;
  --s->active;
  s->cv_done.notify_all();
}

// Passes of this slot run grouped (on its group's stream).
bool grouped(const lrp_server* s, const Slot& sl) {
  return s->grouping_tick && sl.group >= 0 && !s->groups[sl.group].broken;
}

// A request that failed: its work on every stream it used has ended before its slot is reused.
void fail_slot(lrp_server* s, Slot& sl, int rc) {
  (void)hipStreamSynchronize(sl.stream);
  if (sl.group >= 0) (void)hipStreamSynchronize(s->groups[sl.group].stream);
  finish_job(s, sl.job, rc, 0, nullptr);
  sched::release(sl, ++s->tick);
}

// Records the slot's pass launches (both parities), uploads its argument blocks and joins the
// group of its launch sequence (created if new). On any failure the slot stays ungrouped.
void setup_group(lrp_server* s, Slot& sl) {
  PassRecord r0, r1;
  if (record_pass(sl.ctx, 0, &r0) != LRP_OK || record_pass(sl.ctx, 1, &r1) != LRP_OK) return;
  if (!(r0.recs == r1.recs) || r0.blob.size() != r1.blob.size()) return;
  const size_t half = (r0.blob.size() + 255) & ~(size_t)255;
  if (hipEventCreateWithFlags(&sl.ev_start, hipEventDisableTiming) != hipSuccess) {
    sl.ev_start = nullptr;
    (void)hipGetLastError();
    return;
  }
  bool ok = hipMalloc(&sl.area, 2 * half) == hipSuccess;
  if (ok) ok = hipMemcpyAsync(sl.area, r0.blob.data(), r0.blob.size(), hipMemcpyHostToDevice, sl.stream) == hipSuccess;
  if (ok)
    ok = hipMemcpyAsync(sl.area + half, r1.blob.data(), r1.blob.size(), hipMemcpyHostToDevice, sl.stream) ==
         hipSuccess;
  if (ok) ok = hipStreamSynchronize(sl.stream) == hipSuccess;
  int idx = -1;
  for (size_t g = 0; ok && idx < 0 && g < s->groups.size(); ++g)
    if (s->groups[g].area == half && s->groups[g].recs == r0.recs) idx = (int)g;
  if (ok && idx < 0) {
    Group G;
    G.recs = r0.recs;
    G.area = half;
    ok = hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) == hipSuccess;
    if (ok && hipMalloc((void**)&G.table, sizeof(char*) * kTable) != hipSuccess) {
      (void)hipStreamDestroy(G.stream);
      ok = false;
    }
    if (ok) {
      s->groups.push_back(G);
      idx = (int)s->groups.size() - 1;
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    if (sl.area) (void)hipFree(sl.area);
    (void)hipEventDestroy(sl.ev_start);
    sl.area = nullptr;
    sl.ev_start = nullptr;
    return;
  }
  sl.group = idx;
}

// The graph of one grouped pass of m requests: the recorded launches with grid z = m, each
// kernel reading its argument block through the group's table, then the stop-flag copies.
int build_group_graph(Group& G, int m, hipGraphExec_t* out) {
  hipGraph_t gr = nullptr;
  if (hipStreamBeginCapture(G.stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return LRP_EINVAL;
  }
  bool ok = true;
  for (const LaunchRec& r : G.recs) {
    GroupRef ref{G.table, r.off};
    void* args[] = {&ref};
    if (hipLaunchKernel(r.fn, dim3(r.gx, r.gy, (unsigned)m), dim3(r.bx), args, r.shm, G.stream) != hipSuccess) {
      ok = false;
      break;
    }
  }
  if (ok) {
    hipLaunchKernelGGL(k_group_poll, dim3(1), dim3(kMaxGroup), 0, G.stream, G.table, m);
    ok = hipGetLastError() == hipSuccess;
  }
  ok = (hipStreamEndCapture(G.stream, &gr) == hipSuccess) && ok;
  if (ok) ok = hipGraphInstantiate(out, gr, nullptr, nullptr, 0) == hipSuccess;
  if (gr) (void)hipGraphDestroy(gr);
  if (!ok) {
    *out = nullptr;
    (void)hipGetLastError();
    return LRP_EINVAL;
  }
  return LRP_OK;
}

// One grouped pass of the m slots in mem (each at its own pass index): the table, the graph
// (whose last node copies the stop flags to the host) and each slot's pass event. LRP_EINVAL: no graph (nothing
// enqueued); LRP_EDEVICE: a launch failed.
int launch_group(lrp_server* s, Group& G, Slot* const* mem, int m) {
  hipGraphExec_t& ex = G.exec[m - 1];
  if (!ex && build_group_graph(G, m, &ex) != LRP_OK) return LRP_EINVAL;
  for (int i = 0; i < m; ++i) {  // work enqueued on a slot's own stream comes first
    const Slot& sl = *mem[i];
    if (sl.moved) continue;
    const hipEvent_t e = sl.k > 0 ? sl.ctx->evit[(sl.k - 1) & 1] : sl.ev_start;
    if (hipStreamWaitEvent(G.stream, e, 0) != hipSuccess) return LRP_EDEVICE;
  }
  const uint64_t id = ++s->launch_seq;
  GroupTable gt{};
  for (int i = 0; i < m; ++i) {
    const Slot& sl = *mem[i];
    gt.base[i] = sl.area + (size_t)(sl.k & 1) * G.area;
    gt.src[i] = &sl.ctx->st->done;
    gt.dst[i] = &sl.ctx->done_host[sl.k & 1];
  }
  hipLaunchKernelGGL(k_group_table, dim3(1), dim3(kMaxGroup), 0, G.stream, G.table, gt, m);
  if (hipGetLastError() != hipSuccess) return LRP_EDEVICE;
  if (hipGraphLaunch(ex, G.stream) != hipSuccess) return LRP_EDEVICE;
  for (int i = 0; i < m; ++i) {
    Slot& sl = *mem[i];
    if (hipEventRecord(sl.ctx->evit[sl.k & 1], G.stream) != hipSuccess) return LRP_EDEVICE;
    ++sl.k;
    sl.moved = true;
    sl.last_launch = id;
  }
  std::lock_guard<std::mutex> g(s->mu);
  s->passes += m;
  ++s->pass_launches;
  return LRP_OK;
}

// The slot's next pass on its own stream (after its previous pass if that ran on the group's
// stream), with the stop-flag copy and its event.
int solo_pass(lrp_server* s, Slot& sl) {
  lrp_ctx* c = sl.ctx;
  if (sl.moved) {
    if (hipStreamWaitEvent(sl.stream, c->evit[(sl.k - 1) & 1], 0) != hipSuccess) return LRP_EDEVICE;
    sl.moved = false;
  }
  int rc = enqueue_pass(c, sl.k);
  if (rc == LRP_OK) rc = enqueue_poll(c, sl.k);
  if (rc != LRP_OK) return rc;
  ++sl.k;
  sl.last_launch = 0;
  std::lock_guard<std::mutex> g(s->mu);
  ++s->passes;
  ++s->pass_launches;
  return LRP_OK;
}

// Advance one active slot without blocking; true if anything was enqueued or completed.
bool advance(lrp_server* s, Slot& sl) {
  lrp_ctx* c = sl.ctx;
  Job* j = sl.job;
  const lrp_request& q = j->req;
  if (sl.phase == 0) {
    int rc = enqueue_start(c, q.r_F, q.U_F, q.ldu, q.sigma_F, q.V_F, q.ldv);
    if (rc == LRP_OK && sl.ev_start && hipEventRecord(sl.ev_start, sl.stream) != hipSuccess) rc = LRP_EDEVICE;
    if (rc != LRP_OK) {
      fail_slot(s, sl, rc);
      return true;
    }
    sl.phase = 1;
    return true;
  }
  if (sl.phase == 1) {
    bool progress = false;
    if (sl.checked < sl.k) {
      const hipError_t e = hipEventQuery(c->evit[sl.checked & 1]);
      if (e == hipSuccess) {
        if (c->done_host[sl.checked & 1]) sl.stop = true;
        ++sl.checked;
        progress = true;
      } else if (e != hipErrorNotReady) {
        fail_slot(s, sl, LRP_EDEVICE);
        return true;
      } else {
        (void)hipGetLastError();  // not ready is not an error; leave no error state behind
      }
    }
    if (!grouped(s, sl) && !sl.stop && sl.k < c->maxiter && sl.k - sl.checked < 2) {
      const int rc = solo_pass(s, sl);
      if (rc != LRP_OK) {
        fail_slot(s, sl, rc);
        return true;
      }
      progress = true;
    }
    if (sl.stop || (sl.k == c->maxiter && sl.checked == sl.k)) {
      int rc = LRP_OK;
      // the finish follows the last pass enqueued, wherever it ran
      if (sl.moved && hipStreamWaitEvent(sl.stream, c->evit[(sl.k - 1) & 1], 0) != hipSuccess) rc = LRP_EDEVICE;
      if (rc == LRP_OK) rc = enqueue_finish(c, q.U_out, q.ldou, q.S_out, q.V_out, q.ldov);
      if (rc != LRP_OK) {
        fail_slot(s, sl, rc);
        return true;
      }
      sl.phase = 2;
      progress = true;
    }
    return progress;
  }
  // phase 2: wait (without blocking) for the finish stage
  const hipError_t e = hipEventQuery(c->evfin);
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();  // not ready is not an error; leave no error state behind
    return false;
  }
  int32_t rank = 0;
  lrp_info info{};
  const int status = (e == hipSuccess) ? collect(c, &rank, &info) : LRP_EDEVICE;
  finish_job(s, j, status, rank, &info);
  sched::release(sl, ++s->tick);
  return true;
}

void destroy_slot(lrp_server* s, Slot& sl) {
  if (sl.ctx) {
    (void)hipStreamSynchronize(sl.stream);
    lrp_destroy(sl.ctx);
  }
  if (sl.area) (void)hipFree(sl.area);
  if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  s->bytes_in_use -= sl.bytes;
  sl = Slot{};
}

// The server side of admission (sched::admit): slots, budget and context creation. Used with
// mu held.
struct AdmitHost {
  lrp_server* s;
  std::deque<Job*>& queue() { return s->queue; }
  const std::vector<Slot>& slots() const { return s->slots; }
  const Key& key(const Job* j) const { return j->key; }
  int64_t bytes(const Job* j) const { return j->bytes; }
  int64_t in_use() const { return s->bytes_in_use; }
  int64_t budget() const { return s->budget; }
  int64_t active() const { return s->active; }
  int64_t max_active() const { return s->max_active; }
  void evict(int i) { destroy_slot(s, s->slots[i]); }

  // A context of j's shape on a new stream, in the first empty entry (or a new one).
  int create(Job* j) {
    Slot sl;
    sl.key = j->key;
    sl.bytes = j->bytes;
    int rc = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess ? LRP_OK : LRP_EDEVICE;
    if (rc == LRP_OK) {
      lrp_opts o{};
      o.maxiter = j->key.maxiter;
      o.precision = j->key.precision;
      o.stream = sl.stream;
      rc = lrp_create(&sl.ctx, j->key.n, j->key.r_max, j->key.tol, &o);
    }
    if (rc != LRP_OK) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      return rc;
    }
    s->bytes_in_use += sl.bytes;
    if (s->grouping) setup_group(s, sl);
    for (size_t i = 0; i < s->slots.size(); ++i)
      if (!s->slots[i].ctx) {
        s->slots[i] = sl;
        return (int)i;
      }
    s->slots.push_back(sl);
    return (int)s->slots.size() - 1;
  }

  void fail(Job* j, int rc) {
    j->status = rc;
    j->info.status = rc;
    j->t_done = Clock::now();
    j->done = true;
    ++s->failed;
    s->cv_done.notify_all();
  }

  void start(Job* j, int i) {
    Slot& sl = s->slots[i];
    j->t_admit = Clock::now();
    j->admitted = true;
    sl.job = j;
    sl.phase = 0;
    sl.k = sl.checked = 0;
    sl.stop = false;
    ++s->active;
  }
};

// Running requests of one group below which each takes its passes on its own stream, two deep,
// as without grouping: aligning them would hold a pass back for the others (up to one pass of
// latency) to save launches that a few concurrent streams overlap anyway.
constexpr int kAlignMin = 3;

// The passes of the grouped slots, per group as sched::plan_group decides: each on its own
// stream while fewer than kAlignMin of the group's requests run, else one launch for every
// request that may take a pass once one of them has nothing in flight (or all of them sit in
// flight in one launch), keeping them aligned two passes deep.
bool launch_groups(lrp_server* s) {
  bool progress = false;
  if (!s->grouping_tick) return false;
  // the running requests of each group, in slot order (one scan of the slots per tick)
  std::vector<std::vector<Slot*>>& by = s->members;
  by.resize(s->groups.size());
  for (std::vector<Slot*>& v : by) v.clear();
  for (Slot& sl : s->slots)
    if (sl.job && sl.group >= 0 && sl.phase == 1 && !sl.stop && sl.k < sl.ctx->maxiter)
      by[sl.group].push_back(&sl);
  for (size_t g = 0; g < s->groups.size(); ++g) {
    Group& G = s->groups[g];
    if (G.broken || by[g].empty()) continue;
    Slot* cand[kMaxGroup];
    int ncand = 0;
    const sched::Plan plan =
        sched::plan_group(by[g].data(), (int)by[g].size(), cand, kMaxGroup, kAlignMin, ncand);
    if (plan == sched::Plan::None) continue;
    progress = true;
    if (plan == sched::Plan::Solo) {
      for (int i = 0; i < ncand; ++i) {
        const int rc = solo_pass(s, *cand[i]);
        if (rc != LRP_OK) fail_slot(s, *cand[i], rc);
      }
      continue;
    }
    const int m = ncand;
    Slot* const* mem = cand;
    const int rc = launch_group(s, G, mem, m);
    if (rc == LRP_EINVAL) {  // no graph: the members go on with passes on their own streams
      G.broken = true;
    } else if (rc != LRP_OK) {
      (void)hipStreamSynchronize(G.stream);
      for (int i = 0; i < m; ++i) fail_slot(s, *mem[i], LRP_EDEVICE);
    }
  }
  return progress;
}

void scheduler(lrp_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool progress;
    {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->stopping) {
        // drop queued requests; running ones are finished below
        while (!s->queue.empty()) {
          Job* j = s->queue.front();
          s->queue.pop_front();
          j->status = LRP_EDEVICE;
          j->info.status = LRP_EDEVICE;
          j->t_done = Clock::now();
          j->done = true;
          ++s->failed;
        }
        s->cv_done.notify_all();
        if (s->active == 0) break;
      }
      AdmitHost h{s};
      progress = sched::admit(h);
      s->grouping_tick = s->grouping;
    }
    for (Slot& sl : s->slots)
      if (sl.job) progress |= advance(s, sl);
    progress |= launch_groups(s);
    if (!progress) {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->queue.empty() || s->active >= s->max_active)
        s->cv_work.wait_for(g, std::chrono::microseconds(20));
    }
  }
  for (Group& G : s->groups) (void)hipStreamSynchronize(G.stream);
  for (Slot& sl : s->slots) destroy_slot(s, sl);
  s->slots.clear();
  for (Group& G : s->groups) {
    for (hipGraphExec_t& e : G.exec)
      if (e) (void)hipGraphExecDestroy(e);
    if (G.table) (void)hipFree(G.table);
    if (G.stream) (void)hipStreamDestroy(G.stream);
  }
  s->groups.clear();
}

Job* find_job(lrp_server* s, int64_t ticket) {
  auto it = s->jobs.find(ticket);
  return it == s->jobs.end() ? nullptr : it->second;
}

void report(const Job* j, int32_t* status, int32_t* rank, lrp_info* info, double* latency_ms) {
  if (status) *status = j->status;
  if (rank) *rank = j->rank;
  if (info) *info = j->info;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count();
}

}  // namespace

extern "C" {

int lrp_server_create(lrp_server** out, int64_t budget_bytes, int32_t max_active) {
  if (!out || budget_bytes <= 0 || max_active < 1 || max_active > 64) return LRP_EINVAL;
  *out = nullptr;
  lrp_server* s = new (std::nothrow) lrp_server();
  if (!s) return LRP_ENOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return LRP_EDEVICE;
  }
  s->budget = budget_bytes;
  s->max_active = max_active;
  s->slots.reserve(64);
  s->th = std::thread(scheduler, s);
  *out = s;
  return LRP_OK;
}

int lrp_server_submit(lrp_server* s, const lrp_request* r, int64_t* ticket) {
  if (!s || !r || !ticket) return LRP_EINVAL;
  // stamped before anything else, so time spent waiting for the scheduler's lock counts
  const Clock::time_point t_call = Clock::now();
  const int64_t n = r->n;
  if (lrp_context_bytes(n, r->r_max, r->maxiter, r->precision) <= 0) return LRP_EINVAL;
  if (r->r_max < 1 || r->r_max > kPMax || r->r_max > n) return LRP_EINVAL;
  if (!(r->tol >= 0.0) || r->maxiter < 0 || r->maxiter > 1000) return LRP_EINVAL;
  if (r->precision != LRP_FP64 && r->precision != LRP_MIXED) return LRP_EINVAL;
  const int rc = check_solve_args(n, r->r_max, r->r_F, r->U_F, r->ldu, r->sigma_F, r->V_F, r->ldv, r->U_out,
                                  r->ldou, r->S_out, r->V_out, r->ldov);
  if (rc != LRP_OK) return rc;
  Job* j = new (std::nothrow) Job();
  if (!j) return LRP_ENOMEM;
  j->req = *r;
  j->key = Key{n, r->r_max, r->tol, r->maxiter == 0 ? 20 : r->maxiter, r->precision};
  j->bytes = context_bytes(n, r->r_max, j->key.maxiter, r->precision == LRP_MIXED);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (j->bytes > s->budget) {
      delete j;
      return LRP_ENOMEM;
    }
    if (s->stopping) {
      delete j;
      return LRP_EINVAL;
    }
    j->ticket = s->next_ticket++;
    j->t_submit = t_call;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    ++s->submitted;
    *ticket = j->ticket;
  }
  s->cv_work.notify_one();
  return LRP_OK;
}

int lrp_server_poll(lrp_server* s, int64_t ticket, int32_t* done, int32_t* status, int32_t* rank,
                    lrp_info* info, double* latency_ms) {
  if (!s || !done) return LRP_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return LRP_EINVAL;
  *done = j->done ? 1 : 0;
  if (j->done) report(j, status, rank, info, latency_ms);
  return LRP_OK;
}

int lrp_server_wait(lrp_server* s, int64_t ticket, int32_t* status, int32_t* rank, lrp_info* info,
                    double* latency_ms) {
  if (!s) return LRP_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  Job* j = find_job(s, ticket);
  if (!j) return LRP_EINVAL;
  s->cv_done.wait(g, [&] { return j->done; });
  report(j, status, rank, info, latency_ms);
  return LRP_OK;
}

int lrp_server_times(lrp_server* s, int64_t ticket, double* queue_ms, double* run_ms) {
  if (!s) return LRP_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  Job* j = find_job(s, ticket);
  if (!j || !j->done) return LRP_EINVAL;
  using ms = std::chrono::duration<double, std::milli>;
  const Clock::time_point a = j->admitted ? j->t_admit : j->t_done;
  if (queue_ms) *queue_ms = ms(a - j->t_submit).count();
  if (run_ms) *run_ms = ms(j->t_done - a).count();
  return LRP_OK;
}

int lrp_server_release(lrp_server* s, int64_t ticket) {
  if (!s) return LRP_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  Job* j = find_job(s, ticket);
  if (!j || !j->done) return LRP_EINVAL;
  s->jobs.erase(ticket);
  delete j;
  return LRP_OK;
}

int lrp_server_get_stats(lrp_server* s, lrp_server_stats* out) {
  if (!s || !out) return LRP_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (int64_t)s->queue.size();
  out->active = s->active;
  out->bytes_in_use = s->bytes_in_use;
  out->bytes_budget = s->budget;
  int nc = 0;
  for (const Slot& sl : s->slots) nc += sl.ctx ? 1 : 0;
  out->contexts = nc;
  out->grouping = s->grouping ? 1 : 0;
  out->passes = s->passes;
  out->pass_launches = s->pass_launches;
  return LRP_OK;
}

int lrp_server_set_grouping(lrp_server* s, int32_t enabled) {
  if (!s) return LRP_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->queue.empty() || s->active > 0) return LRP_EINVAL;
  s->grouping = enabled != 0;
  return LRP_OK;
}

int lrp_server_destroy(lrp_server* s) {
  if (!s) return LRP_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  for (auto& kv : s->jobs) delete kv.second;
  delete s;
  return LRP_OK;
}

}  // extern "C"
