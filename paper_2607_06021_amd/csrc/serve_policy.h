// Scheduling policy of the serving queue, host code only (no device calls, no HIP headers):
// admission of queued requests against a device-memory budget, and when the running requests
// of one group take their next pass together. The server instantiates these templates with its
// slots and a host adapter; CPU tests instantiate them with fake slots, a fake budget and a
// fake clock.
//
// A slot type provides: ctx (non-null while the slot holds a context), job (non-null while a
// request runs in it), key (the request shape, comparable with ==), last_used (tick of the last
// release), and for passes k (passes enqueued), checked (passes whose stop flag was read),
// last_launch (the group launch of the last pass, 0 for a launch of its own), plus the fields
// that release() resets.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace lrp {
namespace sched {

enum class Step { Reuse, Create, Evict, Wait };

struct Choice {
  Step step;
  int slot;  // the slot to reuse or free; -1 otherwise
};

// The next step for the request at the head of the queue (shape key, context bytes). An idle
// slot of its shape is reused; otherwise a new context is created if its bytes fit beside those
// in use; otherwise the least recently used idle slot is freed (it holds another shape, since
// none of the request's own is idle) and the choice is made again; with no idle slot left the
// request waits for a running one to finish.
template <class SlotT, class KeyT>
Choice admit_choice(const std::vector<SlotT>& slots, const KeyT& key, int64_t bytes, int64_t in_use,
                    int64_t budget) {
  for (size_t i = 0; i < slots.size(); ++i)
    if (slots[i].ctx && !slots[i].job && slots[i].key == key) return {Step::Reuse, (int)i};
  if (in_use + bytes <= budget) return {Step::Create, -1};
  int victim = -1;
  for (size_t i = 0; i < slots.size(); ++i)
    if (slots[i].ctx && !slots[i].job && (victim < 0 || slots[i].last_used < slots[victim].last_used))
      victim = (int)i;
  if (victim < 0) return {Step::Wait, -1};
  return {Step::Evict, victim};
}

// Admission. Requests leave the queue strictly in arrival order -- only the head is considered,
// so a large request waiting for memory is never overtaken by later small ones -- while fewer
// than max_active run. A request whose context cannot be created fails and leaves the queue
// without holding a slot. The host H supplies:
//   queue()            the queue (front(), pop_front(), empty()) of request handles
//   slots()            the slot vector
//   key(j), bytes(j)   a request's shape and context bytes
//   in_use(), budget() context bytes held by slots, and their limit
//   active(), max_active()
//   evict(i)           free idle slot i (its bytes leave in_use())
//   create(j)          a new slot for j: its index, or a negative status
//   fail(j, status)    finish j with that status
//   start(j, i)        run j in slot i (active() grows by one)
// Returns whether any request left the queue or any slot was freed.
template <class H>
bool admit(H& h) {
  bool progress = false;
  while (!h.queue().empty() && h.active() < h.max_active()) {
    auto j = h.queue().front();
    const Choice c = admit_choice(h.slots(), h.key(j), h.bytes(j), h.in_use(), h.budget());
    if (c.step == Step::Wait) break;
    progress = true;
    if (c.step == Step::Evict) {
      h.evict(c.slot);
      continue;
    }
    h.queue().pop_front();
    int i = c.slot;
    if (c.step == Step::Create) {
      i = h.create(j);
      if (i < 0) {
        h.fail(j, i);
        continue;
      }
    }
    h.start(j, i);
  }
  return progress;
}

// A slot whose request finished or failed becomes idle: it keeps its context for the next
// request of its shape and records the tick for least-recently-used eviction.
template <class SlotT>
void release(SlotT& sl, uint64_t tick) {
  sl.job = nullptr;
  sl.phase = 0;
  sl.k = sl.checked = 0;
  sl.stop = false;
  sl.moved = false;
  sl.last_launch = 0;
  sl.last_used = tick;
}

enum class Plan { None, Solo, Launch };

// The next passes of one group, given its running requests (members, in slot order); a
// candidate is a member that may take a pass now (fewer than two passes unchecked). With
// fewer than align_min members, each candidate takes its pass on its own stream (Solo). With
// more, passes start when some candidate has nothing in flight -- then every candidate joins
// one launch -- or when all members sit in flight in the same launch (the next pass of all of
// them, two deep); otherwise the group waits (None) so that the members line up. A launch of a
// single candidate is Solo as well. The candidates are written to cand[0 .. ncand).
template <class SlotT>
Plan plan_group(SlotT* const* members, int nmem, SlotT** cand, int max_cand, int align_min, int& ncand) {
  ncand = 0;
  bool idle = false, aligned = true;
  uint64_t lid = 0;
  for (int i = 0; i < nmem; ++i) {
    SlotT& sl = *members[i];
    if (sl.k - sl.checked >= 2 || ncand == max_cand) {
      aligned = false;
      continue;
    }
    cand[ncand++] = &sl;
    if (sl.k == sl.checked) idle = true;
    if (sl.last_launch == 0 || (lid && sl.last_launch != lid)) aligned = false;
    lid = sl.last_launch;
  }
  if (ncand == 0) return Plan::None;
  if (nmem >= align_min && !idle && !(aligned && ncand == nmem)) return Plan::None;
  return nmem < align_min || ncand == 1 ? Plan::Solo : Plan::Launch;
}

}  // namespace sched
}  // namespace lrp
