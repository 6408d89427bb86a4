// CPU checks of the serving queue's scheduling policy (paper_2607_06021_amd/csrc/serve_policy.h):
// admission against a device-memory budget, slot reuse and least-recently-used eviction,
// arrival order, failure handling, and the alignment of a group's passes. Fake slots, a fake
// budget and a fake clock stand in for contexts, device memory and time; the policy code is the
// server's own. Built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sched.py. Prints one line per case and "ALL OK" at the end; exits non-zero on the
// first failed check.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <set>
#include <vector>

#include "serve_policy.h"

using namespace lrp::sched;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);            \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

namespace {

constexpr int kFail = -3;  // a failed context creation or run

struct Key {
  int shape = -1;
  bool operator==(const Key& o) const { return shape == o.shape; }
};

struct FakeCtx {
  int maxiter;
};

struct Job {
  int id = 0;
  Key key;
  int64_t bytes = 0;
  int64_t duration = 1;
  bool fail_create = false;
  bool fail_run = false;
  bool done = false;
  int status = 0;
};

struct Slot {
  FakeCtx* ctx = nullptr;
  Job* job = nullptr;
  Key key;
  int64_t bytes = 0;
  uint64_t last_used = 0;
  int phase = 0, k = 0, checked = 0;
  bool stop = false, moved = false;
  uint64_t last_launch = 0;
  int64_t finish = 0;  // fake clock: when the running request ends
};

// The host side of admission, as the server's, over fake contexts (heap objects, so the
// sanitizers see a leak or a use after free).
struct Host {
  std::deque<Job*> q;
  std::vector<Slot> sl;
  int64_t use = 0, bud = 0, act = 0, maxact = 1, now = 0;
  uint64_t tick = 0;
  int creates = 0, evicts = 0, create_failures = 0;
  std::vector<int> order;  // ids in admission order (failed creations included)

  std::deque<Job*>& queue() { return q; }
  const std::vector<Slot>& slots() const { return sl; }
  const Key& key(const Job* j) const { return j->key; }
  int64_t bytes(const Job* j) const { return j->bytes; }
  int64_t in_use() const { return use; }
  int64_t budget() const { return bud; }
  int64_t active() const { return act; }
  int64_t max_active() const { return maxact; }

  void evict(int i) {
    CHECK(i >= 0 && i < (int)sl.size());
    CHECK(sl[i].ctx && !sl[i].job);
    delete sl[i].ctx;
    use -= sl[i].bytes;
    sl[i] = Slot{};
    ++evicts;
  }
  int create(Job* j) {
    if (j->fail_create) return kFail;
    Slot s;
    s.ctx = new FakeCtx{20};
    s.key = j->key;
    s.bytes = j->bytes;
    use += s.bytes;
    ++creates;
    for (size_t i = 0; i < sl.size(); ++i)
      if (!sl[i].ctx) {
        sl[i] = s;
        return (int)i;
      }
    sl.push_back(s);
    return (int)sl.size() - 1;
  }
  void fail(Job* j, int rc) {
    CHECK(j->fail_create && rc == kFail);
    ++create_failures;
    j->done = true;
    j->status = rc;
    order.push_back(j->id);
  }
  void start(Job* j, int i) {
    CHECK(i >= 0 && i < (int)sl.size() && sl[i].ctx && !sl[i].job && sl[i].key == j->key);
    if (sl[i].bytes != j->bytes) CHECK(false);
    sl[i].job = j;
    sl[i].finish = now + j->duration;
    ++act;
    order.push_back(j->id);
  }

  // Requests whose time is up finish (or fail) and release their slots.
  void complete() {
    for (Slot& s : sl)
      if (s.job && s.finish <= now) {
        s.job->done = true;
        s.job->status = s.job->fail_run ? kFail : 0;
        release(s, ++tick);
        --act;
      }
  }

  void invariants() const {
    int64_t held = 0, running = 0;
    std::set<const Job*> seen;
    for (const Slot& s : sl) {
      if (!s.ctx) {
        CHECK(!s.job && s.bytes == 0);
        continue;
      }
      held += s.bytes;
      if (s.job) {
        ++running;
        CHECK(seen.insert(s.job).second);
        CHECK(s.job->key == s.key);
        CHECK(!s.job->done);
      }
    }
    CHECK(held == use);
    CHECK(use <= bud);
    CHECK(running == act);
    CHECK(act <= maxact);
  }

  void drop_all() {
    for (size_t i = 0; i < sl.size(); ++i)
      if (sl[i].ctx) evict((int)i);
    CHECK(use == 0);
  }
};

Job mk(int id, int shape, int64_t bytes, int64_t duration) {
  Job j;
  j.id = id;
  j.key.shape = shape;
  j.bytes = bytes;
  j.duration = duration;
  return j;
}

void run_until_idle(Host& h, int64_t limit) {
  for (; h.now < limit; ++h.now) {
    h.complete();
    admit(h);
    h.invariants();
    if (h.q.empty() && h.act == 0) return;
  }
  CHECK(false);  // did not drain in time
}

// A request that does not fit beside a running one queues; when the running one finishes its
// idle slot (another shape) is freed and the waiting one is admitted.
void case_budget_exhausted_queues() {
  Host h;
  h.bud = 100;
  h.maxact = 4;
  Job a = mk(0, 1, 60, 5), b = mk(1, 2, 60, 5);
  h.q = {&a, &b};
  CHECK(admit(h));
  h.invariants();
  CHECK(h.order == std::vector<int>({0}));
  CHECK(h.q.size() == 1 && h.act == 1);
  CHECK(!admit(h));  // nothing changes while a is running
  h.now = 5;
  h.complete();
  CHECK(h.act == 0 && a.done && a.status == 0);
  CHECK(admit(h));
  h.invariants();
  CHECK(h.evicts == 1 && h.creates == 2);
  CHECK(h.order == std::vector<int>({0, 1}));
  run_until_idle(h, 100);
  h.drop_all();
  std::printf("ok budget_exhausted_queues\n");
}

// An idle slot of the request's shape is reused without a new context.
void case_reuse_same_shape() {
  Host h;
  h.bud = 100;
  h.maxact = 2;
  Job a = mk(0, 7, 80, 3), b = mk(1, 7, 80, 3);
  h.q = {&a};
  admit(h);
  h.now = 3;
  h.complete();
  h.q.push_back(&b);
  admit(h);
  h.invariants();
  CHECK(h.creates == 1 && h.evicts == 0 && h.act == 1);
  run_until_idle(h, 100);
  CHECK(b.done && b.status == 0);
  h.drop_all();
  std::printf("ok reuse_same_shape\n");
}

// A large request at the head waits for memory; later small ones that would fit are not
// admitted before it.
void case_fifo_no_overtake() {
  Host h;
  h.bud = 100;
  h.maxact = 8;
  Job a = mk(0, 1, 50, 10), b = mk(1, 2, 60, 2), c = mk(2, 3, 10, 2), d = mk(3, 4, 10, 2);
  h.q = {&a, &b, &c, &d};
  admit(h);
  h.invariants();
  CHECK(h.order == std::vector<int>({0}));
  CHECK(h.q.size() == 3);
  for (h.now = 1; h.now < 10; ++h.now) {
    h.complete();
    admit(h);
    h.invariants();
    CHECK(h.order.size() == 1);  // b still waits for a, and c, d wait behind b
  }
  run_until_idle(h, 100);
  CHECK(h.order == std::vector<int>({0, 1, 2, 3}));
  h.drop_all();
  std::printf("ok fifo_no_overtake\n");
}

// No more than max_active requests run, whatever the budget.
void case_max_active() {
  Host h;
  h.bud = 1000;
  h.maxact = 2;
  std::vector<Job> jobs;
  for (int i = 0; i < 6; ++i) jobs.push_back(mk(i, i % 3, 10, 4));
  for (Job& j : jobs) h.q.push_back(&j);
  admit(h);
  CHECK(h.act == 2 && h.q.size() == 4);
  run_until_idle(h, 100);
  CHECK(h.order == std::vector<int>({0, 1, 2, 3, 4, 5}));
  h.drop_all();
  std::printf("ok max_active\n");
}

// A request whose context cannot be created fails, holds no slot and no memory, and the next
// request is admitted in the same step.
void case_create_failure() {
  Host h;
  h.bud = 100;
  h.maxact = 4;
  Job a = mk(0, 1, 40, 3), b = mk(1, 2, 40, 3);
  a.fail_create = true;
  h.q = {&a, &b};
  CHECK(admit(h));
  h.invariants();
  CHECK(a.done && a.status == kFail);
  CHECK(h.act == 1 && h.use == 40 && h.creates == 1);
  run_until_idle(h, 100);
  CHECK(b.done && b.status == 0);
  h.drop_all();
  std::printf("ok create_failure\n");
}

// A request that fails while running releases its slot; the slot serves the next request of
// its shape.
void case_failed_request_frees_slot() {
  Host h;
  h.bud = 100;
  h.maxact = 1;
  Job a = mk(0, 5, 90, 2), b = mk(1, 5, 90, 2);
  a.fail_run = true;
  h.q = {&a, &b};
  run_until_idle(h, 100);
  CHECK(a.done && a.status == kFail);
  CHECK(b.done && b.status == 0);
  CHECK(h.creates == 1 && h.evicts == 0);
  for (const Slot& s : h.sl) CHECK(!s.job && s.k == 0 && s.checked == 0 && !s.stop && s.last_launch == 0);
  h.drop_all();
  std::printf("ok failed_request_frees_slot\n");
}

// Idle slots are freed least recently used first, and only as many as needed.
void case_lru_eviction() {
  Host h;
  h.bud = 100;
  h.maxact = 1;
  // shapes 1, 2, 3 run one after another (30 bytes each) and stay idle; then 1 runs again
  Job a = mk(0, 1, 30, 1), b = mk(1, 2, 30, 1), c = mk(2, 3, 30, 1), a2 = mk(3, 1, 30, 1);
  h.q = {&a, &b, &c, &a2};
  run_until_idle(h, 100);
  CHECK(h.creates == 3 && h.evicts == 0);  // shape 1 reused
  // shape 2 is now the least recently used, then 3, then 1
  Job d = mk(4, 4, 40, 1);
  h.q = {&d};
  admit(h);
  h.invariants();
  CHECK(h.evicts == 1);
  for (const Slot& s : h.sl) CHECK(!(s.ctx && s.key.shape == 2));
  h.now += 1;
  h.complete();
  Job e = mk(5, 5, 60, 1);
  h.q = {&e};
  admit(h);
  h.invariants();
  // 30 (shape 1) + 30 (shape 3) + 40 (shape 4) in use: to fit 60, free shape 3, then shape 1
  CHECK(h.evicts == 3);
  for (const Slot& s : h.sl) CHECK(!(s.ctx && (s.key.shape == 1 || s.key.shape == 3)));
  run_until_idle(h, 100);
  h.drop_all();
  std::printf("ok lru_eviction\n");
}

// A random stream of requests on a fake clock: shapes, sizes, durations and failures drawn from
// a seeded generator. Checked at every step: the invariants; at the end: every request done,
// admitted in arrival order, memory all released.
void case_random_stream(unsigned seed) {
  std::mt19937_64 rng(seed);
  Host h;
  h.bud = 150;
  h.maxact = 1 + (int)(rng() % 8);
  const int njobs = 2000;
  std::vector<Job> jobs(njobs);
  std::vector<int64_t> arrival(njobs);
  int64_t t = 0;
  for (int i = 0; i < njobs; ++i) {
    const int shape = (int)(rng() % 6);
    jobs[i] = mk(i, shape, 5 + 25 * shape, 1 + (int64_t)(rng() % 20));
    jobs[i].fail_create = rng() % 100 == 0;
    jobs[i].fail_run = rng() % 100 == 0;
    t += (int64_t)(rng() % 4);
    arrival[i] = t;
  }
  int next = 0;
  for (h.now = 0; h.now < 1000000; ++h.now) {
    h.complete();
    while (next < njobs && arrival[next] <= h.now) h.q.push_back(&jobs[next++]);
    admit(h);
    h.invariants();
    if (next == njobs && h.q.empty() && h.act == 0) break;
  }
  CHECK(next == njobs && h.q.empty() && h.act == 0);
  CHECK((int)h.order.size() == njobs);
  for (int i = 0; i < njobs; ++i) CHECK(h.order[i] == i);
  for (const Job& j : jobs) {
    CHECK(j.done);
    // a request whose creation would fail may reuse an idle slot of its shape instead
    if (j.fail_run) CHECK(j.status == kFail);
    if (!j.fail_run && !j.fail_create) CHECK(j.status == 0);
  }
  int failed = 0;
  for (const Job& j : jobs) failed += j.status == kFail ? 1 : 0;
  CHECK(h.create_failures > 0 && failed > h.create_failures);
  h.drop_all();
  std::printf("ok random_stream seed=%u max_active=%lld creates=%d evicts=%d\n", seed, (long long)h.maxact,
              h.creates, h.evicts);
}

// ---- group passes ----

struct GroupSlot : Slot {
  bool member = true;
};

// The plan for the members among v (the server passes a group's running requests in slot order).
Plan plan(std::vector<GroupSlot>& v, std::vector<int>& cand_idx) {
  std::vector<GroupSlot*> mem;
  for (GroupSlot& s : v)
    if (s.member) mem.push_back(&s);
  GroupSlot* cand[64];
  int ncand = -1;
  const Plan p = plan_group(mem.data(), (int)mem.size(), cand, 64, 3, ncand);
  CHECK(ncand >= 0 && ncand <= (int)v.size());
  cand_idx.clear();
  for (int i = 0; i < ncand; ++i) cand_idx.push_back((int)(cand[i] - v.data()));
  return p;
}

GroupSlot gs(int k, int checked, uint64_t launch, bool member = true) {
  GroupSlot s;
  s.k = k;
  s.checked = checked;
  s.last_launch = launch;
  s.member = member;
  return s;
}

void case_plan_group() {
  std::vector<int> c;
  // nobody running, or nobody may take a pass
  std::vector<GroupSlot> v = {gs(0, 0, 0, false)};
  CHECK(plan(v, c) == Plan::None && c.empty());
  v = {gs(4, 2, 0), gs(6, 4, 0)};
  CHECK(plan(v, c) == Plan::None);
  // fewer than three running: each on its own stream
  v = {gs(0, 0, 0), gs(3, 2, 0)};
  CHECK(plan(v, c) == Plan::Solo && c == std::vector<int>({0, 1}));
  // three running, one with nothing in flight: all candidates in one launch
  v = {gs(2, 2, 0), gs(3, 2, 0), gs(5, 4, 9)};
  CHECK(plan(v, c) == Plan::Launch && c == std::vector<int>({0, 1, 2}));
  // three in flight in the same launch: their next pass together
  v = {gs(3, 2, 7), gs(5, 4, 7), gs(1, 0, 7)};
  CHECK(plan(v, c) == Plan::Launch && c.size() == 3);
  // in flight in different launches (or their own streams): wait to align
  v = {gs(3, 2, 7), gs(5, 4, 8), gs(1, 0, 7)};
  CHECK(plan(v, c) == Plan::None);
  v = {gs(3, 2, 7), gs(5, 4, 0), gs(1, 0, 7)};
  CHECK(plan(v, c) == Plan::None);
  // one aligned member two deep: the others wait for it
  v = {gs(4, 2, 7), gs(5, 4, 7), gs(1, 0, 7)};
  CHECK(plan(v, c) == Plan::None);
  // a single candidate with nothing in flight: a launch of its own
  v = {gs(4, 2, 7), gs(6, 4, 7), gs(1, 1, 0)};
  CHECK(plan(v, c) == Plan::Solo && c == std::vector<int>({2}));
  // non-members are ignored, also for the count
  v = {gs(2, 2, 0), gs(3, 2, 0, false), gs(5, 4, 0, false), gs(1, 0, 0)};
  CHECK(plan(v, c) == Plan::Solo && c == std::vector<int>({0, 3}));
  std::printf("ok plan_group\n");
}

// Requests of one group started at staggered times, on a fake clock: a pass takes `dur` ticks on
// the stream it runs on (a slot's own, or the group's, where launches queue one after another;
// a launch also waits for each member's previous pass). A pass's stop flag is read when it ends.
// Every request makes maxiter passes; passes never run more than two ahead of their flags; the
// members end up aligned, so launches are far fewer than passes; and lining up delays a request
// by no more than about one pass per request of the group.
void case_group_alignment(unsigned seed) {
  std::mt19937_64 rng(seed);
  const int nreq = 6, maxiter = 20;
  const int64_t dur = 10;
  std::vector<GroupSlot> v(nreq);
  std::vector<int64_t> start(nreq);
  std::vector<std::deque<int64_t>> inflight(nreq);  // end times of passes not yet checked
  std::vector<int64_t> stream_free(nreq, 0), finished(nreq, -1);
  int64_t group_free = 0;
  uint64_t seq = 0;
  int launches = 0, passes = 0, full = 0;
  for (int i = 0; i < nreq; ++i) {
    start[i] = (int64_t)(rng() % 40);
    v[i].member = false;
  }
  int64_t now = 0;
  for (; now < 100000; ++now) {
    for (int i = 0; i < nreq; ++i) {
      if (!v[i].member && v[i].k == 0 && now >= start[i]) v[i].member = true;
      while (!inflight[i].empty() && inflight[i].front() <= now) {
        inflight[i].pop_front();
        ++v[i].checked;
      }
      CHECK(v[i].k - v[i].checked == (int)inflight[i].size());
      if (v[i].checked == maxiter && finished[i] < 0) finished[i] = now;
      if (v[i].k == maxiter) v[i].member = false;
    }
    std::vector<int> c;
    const Plan p = plan(v, c);
    if (p == Plan::Solo) {
      for (int i : c) {
        const int64_t end = std::max(now, stream_free[i]) + dur;
        stream_free[i] = end;
        inflight[i].push_back(end);
        ++v[i].k;
        v[i].last_launch = 0;
        ++launches;
        ++passes;
      }
    } else if (p == Plan::Launch) {
      int64_t begin = std::max(now, group_free);
      for (int i : c) begin = std::max(begin, inflight[i].empty() ? now : inflight[i].back());
      const int64_t end = begin + dur;
      group_free = end;
      ++seq;
      for (int i : c) {
        inflight[i].push_back(end);
        stream_free[i] = end;
        ++v[i].k;
        v[i].last_launch = seq;
        ++passes;
      }
      ++launches;
      int running = 0;
      for (const GroupSlot& s : v) running += s.member ? 1 : 0;
      if ((int)c.size() == running && running == nreq) ++full;
    }
    for (int i = 0; i < nreq; ++i) CHECK(v[i].k - v[i].checked <= 2);
    bool all = true;
    for (int i = 0; i < nreq; ++i) all = all && v[i].checked == maxiter;
    if (all) break;
  }
  CHECK(now < 100000);
  CHECK(passes == nreq * maxiter);
  CHECK(launches * 2 < passes);  // aligned: most launches carry several requests
  CHECK(full > 0);               // and some carry all of them
  // alone a request takes maxiter passes back to back; lining up with each request that joins
  // later holds it back by at most about one pass
  for (int i = 0; i < nreq; ++i) CHECK(finished[i] - start[i] <= (maxiter + nreq) * dur);
  std::printf("ok group_alignment seed=%u launches=%d passes=%d full=%d ticks=%lld\n", seed, launches, passes,
              full, (long long)now);
}

}  // namespace

int main() {
  case_budget_exhausted_queues();
  case_reuse_same_shape();
  case_fifo_no_overtake();
  case_max_active();
  case_create_failure();
  case_failed_request_frees_slot();
  case_lru_eviction();
  for (unsigned seed = 0; seed < 4; ++seed) case_random_stream(seed);
  case_plan_group();
  for (unsigned seed = 0; seed < 16; ++seed) case_group_alignment(seed);
  std::printf("ALL OK\n");
  return 0;
}
