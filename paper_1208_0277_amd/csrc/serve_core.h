// Host core of the serving loop: FIFO ring arenas for the resident job data,
// admission by footprint, and the grouping of admitted jobs into bounded
// launches.  Pure C++ (no HIP): the device side is an executor object, so the
// same scheduling logic runs against a fake executor in host-only tests.
//
// Jobs are admitted, launched and retired in submission order, so each arena
// is a ring whose allocations are released oldest first: an allocation is one
// contiguous range; one that does not fit before the end of the ring starts
// again at 0 and holds the skipped tail until it is released.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

namespace sccg {
namespace serve {

class Ring {
 public:
  explicit Ring(int64_t cap = 0) : cap_(cap) {}

  int64_t capacity() const { return cap_; }
  int64_t used() const { return used_; }
  size_t live() const { return live_.size(); }

  // Reserve n >= 1 contiguous elements; returns the offset or -1 if the
  // free space cannot hold them now.
  int64_t alloc(int64_t n) {
    if (n < 1 || n > cap_) return -1;
    if (live_.empty()) head_ = tail_ = 0;
    Entry e{};
    e.prev_head = head_;
    if (live_.empty() || head_ > tail_) {
      // free space: [head, cap) and [0, tail)
      if (cap_ - head_ >= n) {
        e.start = e.off = head_;
      } else if (tail_ >= n) {
        e.start = head_;  // the skipped tail [head, cap) belongs to this entry
        e.off = 0;
      } else {
        return -1;
      }
    } else {
      // free space: [head, tail)
      if (tail_ - head_ < n) return -1;
      e.start = e.off = head_;
    }
    e.len = n;
    e.held = (e.off == e.start) ? n : (cap_ - e.start) + n;
    head_ = e.off + n;
    used_ += e.held;
    live_.push_back(e);
    return e.off;
  }

  // Undo the most recent alloc (admission of a job that needs several arenas).
  void undo_last() {
    const Entry e = live_.back();
    live_.pop_back();
    used_ -= e.held;
    head_ = e.prev_head;
    if (live_.empty()) head_ = tail_ = 0;
  }

  // Release the oldest allocation.
  void release_oldest() {
    const Entry e = live_.front();
    live_.pop_front();
    used_ -= e.held;
    if (live_.empty()) {
      head_ = tail_ = 0;
    } else {
      tail_ = live_.front().start;
    }
  }

  // Offset of the i-th oldest live allocation (tests).
  int64_t offset_of(size_t i) const { return live_[i].off; }

 private:
  struct Entry {
    int64_t start;      // first element held (the skipped tail for a wrapped entry)
    int64_t off;        // first element handed out
    int64_t len;        // elements handed out
    int64_t held;       // elements held, including a skipped tail
    int64_t prev_head;  // head before this entry (undo)
  };
  int64_t cap_ = 0;
  int64_t head_ = 0;  // next free element
  int64_t tail_ = 0;  // first element held by the oldest entry
  int64_t used_ = 0;
  std::deque<Entry> live_;
};

// What a job needs from the three arenas.
struct Footprint {
  int64_t vertices;  // ring vertices of both sets
  int64_t slots;     // offset slots: (n_a + 1) + (n_b + 1)
  int64_t pairs;
};

// Places of an admitted job in the arenas.
struct Placement {
  int64_t vert_off;
  int64_t slot_off;
  int64_t pair_off;
};

class Arenas {
 public:
  Arenas(int64_t vertex_cap, int64_t slot_cap, int64_t pair_cap)
      : verts_(vertex_cap), slots_(slot_cap), pairs_(pair_cap) {}

  // A job that could never fit, even into empty arenas.
  bool too_big(const Footprint& f) const {
    return std::max<int64_t>(f.vertices, 1) > verts_.capacity() || f.slots > slots_.capacity() ||
           std::max<int64_t>(f.pairs, 1) > pairs_.capacity();
  }

  // All three reservations or none.
  bool admit(const Footprint& f, Placement* p) {
    const int64_t v = verts_.alloc(std::max<int64_t>(f.vertices, 1));
    if (v < 0) return false;
    const int64_t s = slots_.alloc(f.slots);
    if (s < 0) {
      verts_.undo_last();
      return false;
    }
    const int64_t q = pairs_.alloc(std::max<int64_t>(f.pairs, 1));
    if (q < 0) {
      slots_.undo_last();
      verts_.undo_last();
      return false;
    }
    *p = Placement{v, s, q};
    return true;
  }

  void retire_oldest() {
    pairs_.release_oldest();
    slots_.release_oldest();
    verts_.release_oldest();
  }

  const Ring& vertices() const { return verts_; }
  const Ring& slots() const { return slots_; }
  const Ring& pairs() const { return pairs_; }

 private:
  Ring verts_, slots_, pairs_;
};

// One launch (sequence number `seq`): `count` jobs whose pairs are the
// contiguous arena range [pair_off, pair_off + n_pairs).
struct Step {
  uint64_t seq;
  int count;
  int64_t pair_off;
  int64_t n_pairs;
};

// Group the oldest not-yet-launched admitted jobs into one launch: as many
// as fit under max_pairs (at least one) and max_jobs, stopping where the pair
// range would not be contiguous (a job that wrapped to the start of the ring
// begins a new launch).  `pair_off[i]`, `n_pairs[i]` describe the admitted
// jobs in order, starting with the first one not launched yet.
inline Step plan_step(uint64_t seq, const std::vector<int64_t>& pair_off, const std::vector<int64_t>& n_pairs,
                      int64_t max_pairs, int max_jobs) {
  Step s{seq, 0, 0, 0};
  if (pair_off.empty()) return s;
  s.pair_off = pair_off[0];
  int64_t end = pair_off[0];
  for (size_t i = 0; i < pair_off.size() && s.count < max_jobs; ++i) {
    if (pair_off[i] != end) break;  // wrapped: not contiguous with the previous job
    const int64_t np = std::max<int64_t>(n_pairs[i], 1);
    if (s.count > 0 && s.n_pairs + np > max_pairs) break;
    s.n_pairs += np;
    end += np;
    s.count += 1;
  }
  return s;
}

// The scheduling state of a server: jobs waiting for admission, admitted
// jobs (the oldest ones in launches on the device), and the launches in
// flight.  `Job` needs the fields `Footprint f`, `Placement pl`,
// `int64_t n_pairs` (>= 1) and `bool counted_wait`.
//
// pump() makes one pass with an executor `ex` providing
//   int  poll(int slot)               1 = that launch finished, 0 = not yet, < 0 = failure
//   bool upload(Job*)                 queue the copy of an admitted job into its placement
//   bool launch(const Step&, Job* const* jobs, int slot)
//   void finish(const Step&, Job* const* jobs, int slot)   results of a finished launch
//   void admission_wait(Job*)         the oldest waiting job did not fit (once per job)
// and returns the number of things that moved (0 = nothing), or < 0 after a
// failure of the executor.  Launch slots are used round robin over
// max_inflight: a slot is reused only after its previous launch finished.
template <class Job>
class Pipeline {
 public:
  Pipeline(int64_t vertex_cap, int64_t slot_cap, int64_t pair_cap, int64_t max_step_pairs, int max_inflight,
           int max_jobs)
      : caps_{vertex_cap, slot_cap, pair_cap},
        arenas_(vertex_cap, slot_cap, pair_cap),
        max_step_pairs_(max_step_pairs),
        max_inflight_(max_inflight),
        max_jobs_(max_jobs) {}

  bool too_big(const Footprint& f) const { return arenas_.too_big(f); }
  void push(Job* j) { pending_.push_back(j); }
  bool empty() const { return pending_.empty() && admitted_.empty(); }
  bool in_flight() const { return !inflight_.empty(); }
  size_t waiting() const { return pending_.size(); }
  const Arenas& arenas() const { return arenas_; }

  // Remove and return the waiting (not yet admitted) job with the fewest
  // pairs among those with at most max_pairs, the earliest on a tie; nullptr
  // if there is none.  The host-migration of Section 4.2 takes the smallest
  // tasks out of a congested device's input buffer.
  Job* take_smallest(int64_t max_pairs) {
    auto best = pending_.end();
    for (auto it = pending_.begin(); it != pending_.end(); ++it)
      if ((*it)->n_pairs <= max_pairs && (best == pending_.end() || (*it)->n_pairs < (*best)->n_pairs)) best = it;
    if (best == pending_.end()) return nullptr;
    Job* j = *best;
    pending_.erase(best);
    return j;
  }

  template <class Exec>
  int pump(Exec& ex) {
    int moved = 0;
    // deliver finished launches; they finish in launch order
    while (!inflight_.empty()) {
      const Launch L = inflight_.front();
      const int q = ex.poll(L.slot);
      if (q < 0) return q;
      if (q == 0) break;
      jobs_.assign(admitted_.begin(), admitted_.begin() + L.step.count);
      ex.finish(L.step, jobs_.data(), L.slot);
      for (int c = 0; c < L.step.count; ++c) {
        admitted_.pop_front();
        arenas_.retire_oldest();
      }
      launched_ -= (size_t)L.step.count;
      inflight_.pop_front();
      ++moved;
    }
    // admit in submission order while the oldest waiting job fits
    while (!pending_.empty()) {
      Job* j = pending_.front();
      Placement pl;
      if (!arenas_.admit(j->f, &pl)) {
        if (!j->counted_wait) {
          j->counted_wait = true;
          ex.admission_wait(j);
        }
        break;
      }
      j->pl = pl;
      pending_.pop_front();
      admitted_.push_back(j);
      if (!ex.upload(j)) return -1;
      ++moved;
    }
    // launch while fewer than max_inflight launches are queued
    while (launched_ < admitted_.size() && (int)inflight_.size() < max_inflight_) {
      po_.clear();
      np_.clear();
      const size_t end = std::min(admitted_.size(), launched_ + (size_t)max_jobs_);
      for (size_t i = launched_; i < end; ++i) {
        po_.push_back(admitted_[i]->pl.pair_off);
        np_.push_back(admitted_[i]->n_pairs);
      }
      const Step st = plan_step(n_launches_, po_, np_, max_step_pairs_, max_jobs_);
      const int slot = (int)(n_launches_ % (uint64_t)max_inflight_);
      jobs_.assign(admitted_.begin() + launched_, admitted_.begin() + launched_ + st.count);
      if (!ex.launch(st, jobs_.data(), slot)) return -1;
      launched_ += (size_t)st.count;
      inflight_.push_back(Launch{st, slot});
      ++n_launches_;
      ++moved;
    }
    return moved;
  }

  // After a failure: hand every held job to `drop` (admitted ones first, in
  // order) and start over with empty arenas.
  template <class F>
  void drain(F drop) {
    for (Job* j : admitted_) drop(j);
    for (Job* j : pending_) drop(j);
    admitted_.clear();
    pending_.clear();
    inflight_.clear();
    launched_ = 0;
    arenas_ = Arenas(caps_[0], caps_[1], caps_[2]);
  }

 private:
  struct Launch {
    Step step;
    int slot;
  };
  int64_t caps_[3];
  Arenas arenas_;
  int64_t max_step_pairs_;
  int max_inflight_;
  int max_jobs_;
  std::deque<Job*> pending_;
  std::deque<Job*> admitted_;
  size_t launched_ = 0;  // the first `launched_` admitted jobs are in launches
  std::deque<Launch> inflight_;
  uint64_t n_launches_ = 0;
  std::vector<Job*> jobs_;
  std::vector<int64_t> po_, np_;
};

}  // namespace serve
}  // namespace sccg
