// Host-only checks of the serving core (ring arenas, launch planning and the
// scheduling pipeline) against a fake executor that models the device: it
// keeps an owner map of every arena element, finishes launches after a random
// number of polls, and can be told to fail.  Built and run by
// tests/test_serve_core.py; prints "ALL OK" and exits 0 on success.
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>

#include <random>
#include <string>
#include <vector>

#include "serve_core.h"

using namespace sccg::serve;

static int g_fail = 0;
#define CHECK(cond, ...)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);                        \
      fprintf(stderr, "\n");                               \
      g_fail = 1;                                          \
      return false;                                        \
    }                                                      \
  } while (0)

// ------------------------------------------------------------------ Ring
struct Range {
  int64_t off, len;
};

static bool ring_random(uint64_t seed) {
  std::mt19937_64 rng(seed);
  const int64_t cap = 1 + (int64_t)(rng() % 300);
  Ring r(cap);
  std::deque<Range> live;
  std::vector<int> owner(cap, 0);
  for (int step = 0; step < 4000; ++step) {
    const int op = (int)(rng() % 10);
    if (op < 5) {
      const int64_t n = 1 + (int64_t)(rng() % (uint64_t)(op == 0 ? cap : std::max<int64_t>(cap / 4, 1)));
      const int64_t off = r.alloc(n);
      if (live.empty()) CHECK(off == 0, "empty ring of %lld refused %lld elements", (long long)cap, (long long)n);
      if (off >= 0) {
        CHECK(off + n <= cap, "range [%lld,%lld) outside capacity %lld", (long long)off, (long long)(off + n),
              (long long)cap);
        for (int64_t k = off; k < off + n; ++k) CHECK(owner[k] == 0, "element %lld handed out twice", (long long)k);
        for (int64_t k = off; k < off + n; ++k) owner[k] = 1;
        live.push_back({off, n});
        if (op == 1) {  // admission rolled back
          r.undo_last();
          for (int64_t k = off; k < off + n; ++k) owner[k] = 0;
          live.pop_back();
        }
      }
    } else if (!live.empty()) {
      const Range x = live.front();
      live.pop_front();
      r.release_oldest();
      for (int64_t k = x.off; k < x.off + x.len; ++k) owner[k] = 0;
    }
    int64_t handed = 0;
    for (const Range& x : live) handed += x.len;
    CHECK(r.live() == live.size(), "live count %zu != %zu", r.live(), live.size());
    CHECK(r.used() >= handed && r.used() <= cap, "used %lld outside [%lld, %lld]", (long long)r.used(),
          (long long)handed, (long long)cap);
    if (live.empty()) CHECK(r.used() == 0, "empty ring still holds %lld", (long long)r.used());
    for (size_t i = 0; i < live.size(); ++i) CHECK(r.offset_of(i) == live[i].off, "offset_of(%zu) mismatch", i);
  }
  while (!live.empty()) {
    live.pop_front();
    r.release_oldest();
  }
  CHECK(r.used() == 0 && r.alloc(cap) == 0, "ring of %lld not whole after releasing everything", (long long)cap);
  return true;
}

static bool ring_wrap_case() {
  Ring r(10);
  CHECK(r.alloc(4) == 0 && r.alloc(4) == 4, "sequential");
  r.release_oldest();                  // live: [4,8)
  CHECK(r.alloc(3) == 0, "wraps to 0");  // [8,10) skipped, held by this entry
  CHECK(r.used() == 4 + 2 + 3, "wrapped entry holds the skipped tail: used %lld", (long long)r.used());
  CHECK(r.alloc(2) == -1, "only [3,4) is free");
  CHECK(r.alloc(1) == 3, "fills [3,4)");
  r.release_oldest();  // live: wrapped [0,3)+tail, [3,4)
  CHECK(r.used() == 2 + 3 + 1, "after release: used %lld", (long long)r.used());
  CHECK(r.alloc(4) == 4, "[4,8) free again");
  return true;
}

// ------------------------------------------------------------ plan_step
static bool plan_cases() {
  Step s = plan_step(0, {0, 10, 30, 0}, {10, 20, 5, 7}, 100, 64);
  CHECK(s.count == 3 && s.pair_off == 0 && s.n_pairs == 35, "stops at the wrapped job");
  s = plan_step(0, {0, 10, 30}, {10, 20, 5}, 25, 64);
  CHECK(s.count == 1 && s.n_pairs == 10, "bounded by max_pairs");
  s = plan_step(0, {5}, {500}, 25, 64);
  CHECK(s.count == 1 && s.n_pairs == 500, "a large job runs alone");
  s = plan_step(0, {0, 1, 2, 3}, {1, 1, 1, 1}, 100, 2);
  CHECK(s.count == 2 && s.n_pairs == 2, "bounded by max_jobs");
  s = plan_step(0, {}, {}, 100, 2);
  CHECK(s.count == 0, "nothing to launch");
  return true;
}

// --------------------------------------------------------- the pipeline
struct FJob {
  int id = 0;
  Footprint f{};
  Placement pl{};
  int64_t n_pairs = 0;
  bool counted_wait = false;
  int waits = 0;
  bool uploaded = false, migrated = false;
};

struct FakeExec {
  std::mt19937_64 rng;
  int64_t caps[3];
  int64_t max_step_pairs;
  int max_inflight, max_jobs;
  std::vector<int> own[3];  // owner job id of each arena element, 0 = free
  std::deque<std::pair<int, int>> launches;  // (slot, polls left)
  std::vector<bool> slot_busy;
  int last_upload_id = 0;  // admissions and launches follow submission order
  int last_launch_id = 0;
  std::deque<int> launched_ids;  // jobs finish in launch order
  int admitted = 0, finished = 0, launched_n = 0, waits = 0;
  int fail_at = -1, calls = 0;  // fail the fail_at-th executor call
  bool ok = true;

  bool failing() { return ++calls == fail_at; }

  bool mark(FJob* j, bool set) {
    const int64_t off[3] = {j->pl.vert_off, j->pl.slot_off, j->pl.pair_off};
    const int64_t len[3] = {std::max<int64_t>(j->f.vertices, 1), j->f.slots, std::max<int64_t>(j->f.pairs, 1)};
    for (int a = 0; a < 3; ++a) {
      CHECK(off[a] >= 0 && off[a] + len[a] <= caps[a], "job %d outside arena %d", j->id, a);
      for (int64_t k = off[a]; k < off[a] + len[a]; ++k) {
        if (set) {
          CHECK(own[a][k] == 0, "job %d overlaps job %d in arena %d", j->id, own[a][k], a);
          own[a][k] = j->id;
        } else {
          CHECK(own[a][k] == j->id, "job %d lost its range in arena %d", j->id, a);
          own[a][k] = 0;
        }
      }
    }
    return true;
  }

  int poll(int slot) {
    if (failing()) return -1;
    if (launches.empty() || launches.front().first != slot) {
      ok = false;
      fprintf(stderr, "FAIL: polled slot %d, not the oldest launch\n", slot);
      return -1;
    }
    if (launches.front().second > 0) {
      launches.front().second -= 1;
      return 0;
    }
    return 1;
  }
  void admission_wait(FJob* j) {
    j->waits += 1;
    waits += 1;
  }
  bool upload(FJob* j) {
    if (failing()) return false;
    if (j->id <= last_upload_id || j->migrated) {
      fprintf(stderr, "FAIL: job %d admitted out of order or after migrating\n", j->id);
      ok = false;
    }
    last_upload_id = j->id;
    j->uploaded = true;
    if (!mark(j, true)) ok = false;
    admitted += 1;
    return ok;
  }
  bool launch(const Step& st, FJob* const* jobs, int slot) {
    if (failing()) return false;
    bool good = true;
    auto fail = [&](const char* what) {
      fprintf(stderr, "FAIL launch: %s\n", what);
      good = false;
    };
    if (st.count < 1 || st.count > max_jobs) fail("job count outside [1, max_jobs]");
    if ((int)launches.size() >= max_inflight) fail("more launches than max_inflight");
    if (slot_busy[slot]) fail("slot reused while its launch is in flight");
    int64_t pos = st.pair_off, total = 0;
    for (int c = 0; c < st.count; ++c) {
      if (jobs[c]->id <= last_launch_id) fail("jobs not launched in submission order");
      last_launch_id = jobs[c]->id;
      launched_ids.push_back(jobs[c]->id);
      if (jobs[c]->pl.pair_off != pos) fail("pair range not contiguous");
      pos += jobs[c]->n_pairs;
      total += jobs[c]->n_pairs;
    }
    if (total != st.n_pairs) fail("n_pairs is not the jobs' sum");
    if (st.count > 1 && st.n_pairs > max_step_pairs) fail("launch above max_step_pairs");
    launches.push_back({slot, (int)(rng() % 4)});
    slot_busy[slot] = true;
    launched_n += 1;
    if (!good) ok = false;
    return good;
  }
  void finish(const Step& st, FJob* const* jobs, int slot) {
    for (int c = 0; c < st.count; ++c) {
      if (launched_ids.empty() || jobs[c]->id != launched_ids.front()) {
        fprintf(stderr, "FAIL: job %d finished out of launch order\n", jobs[c]->id);
        ok = false;
      }
      if (!launched_ids.empty()) launched_ids.pop_front();
      if (!mark(jobs[c], false)) ok = false;
      finished += 1;
    }
    launches.pop_front();
    slot_busy[slot] = false;
  }
};

// With `migrate`, some pumps are followed by take_smallest (the host
// migration): the job it returns must be the waiting one with the fewest
// pairs under the bound (the earliest on a tie), and it never runs on the
// device.
static bool pipeline_random(uint64_t seed, int fail_at, bool migrate = false) {
  std::mt19937_64 rng(seed);
  const int64_t vcap = 50 + (int64_t)(rng() % 400), scap = 20 + (int64_t)(rng() % 100),
                pcap = 10 + (int64_t)(rng() % 200);
  const int64_t max_step = 1 + (int64_t)(rng() % 60);
  const int max_inflight = 1 + (int)(rng() % 4), max_jobs = 1 + (int)(rng() % 8);
  Pipeline<FJob> pipe(vcap, scap, pcap, max_step, max_inflight, max_jobs);
  FakeExec ex;
  ex.rng.seed(seed * 7 + 1);
  ex.caps[0] = vcap;
  ex.caps[1] = scap;
  ex.caps[2] = pcap;
  for (int a = 0; a < 3; ++a) ex.own[a].assign(ex.caps[a], 0);
  ex.max_step_pairs = max_step;
  ex.max_inflight = max_inflight;
  ex.max_jobs = max_jobs;
  ex.slot_busy.assign(max_inflight, false);
  ex.fail_at = fail_at;
  std::vector<FJob*> all;
  const int n_jobs = 300;
  int submitted = 0, rejected = 0, dropped = 0, migrated = 0;
  bool failed = false;
  for (int round = 0; round < 100000 && !failed; ++round) {
    if (submitted < n_jobs && rng() % 3 == 0) {
      FJob* j = new FJob();
      const int64_t na = (int64_t)(rng() % 12), nb = (int64_t)(rng() % 12);
      j->f = Footprint{(int64_t)(rng() % (uint64_t)(vcap / 2 + 1)), na + nb + 2,
                       1 + (int64_t)(rng() % (uint64_t)(pcap / 2))};
      if (rng() % 25 == 0) j->f.vertices = vcap + 1;  // never fits
      j->n_pairs = j->f.pairs;
      if (pipe.too_big(j->f)) {
        rejected += 1;
        delete j;
      } else {
        j->id = ++submitted;
        all.push_back(j);
        pipe.push(j);
      }
    }
    const int moved = pipe.pump(ex);
    if (!ex.ok) return false;
    if (migrate && moved >= 0 && rng() % 4 == 0) {
      const int64_t bound = rng() % 2 ? INT64_MAX : 1 + (int64_t)(rng() % (uint64_t)(pcap / 2));
      const FJob* want = nullptr;
      size_t n_waiting = 0;
      for (const FJob* w : all) {
        if (w->uploaded || w->migrated) continue;
        n_waiting += 1;
        if (w->n_pairs <= bound && (!want || w->n_pairs < want->n_pairs)) want = w;
      }
      CHECK(n_waiting == pipe.waiting(), "waiting() %zu, expected %zu", pipe.waiting(), n_waiting);
      FJob* got = pipe.take_smallest(bound);
      CHECK(got == want, "take_smallest returned job %d, expected job %d", got ? got->id : 0, want ? want->id : 0);
      if (got) {
        got->migrated = true;
        migrated += 1;
        CHECK(pipe.waiting() == n_waiting - 1, "the migrated job is still waiting");
      }
    }
    if (moved < 0) {
      CHECK(fail_at > 0, "pump failed without an injected failure");
      pipe.drain([&](FJob* j) {
        dropped += 1;
        (void)j;
      });
      failed = true;
    }
    if (submitted >= n_jobs && pipe.empty()) break;
  }
  const int accepted = submitted;
  if (migrate && fail_at < 0) CHECK(migrated > 0, "seed %llu: nothing migrated", (unsigned long long)seed);
  if (!failed) {
    CHECK(pipe.empty(), "pipeline did not drain (%d of %d finished)", ex.finished, accepted);
    CHECK(ex.finished + migrated == accepted, "%d finished + %d migrated of %d jobs", ex.finished, migrated,
          accepted);
    CHECK(pipe.arenas().vertices().used() == 0 && pipe.arenas().slots().used() == 0 &&
              pipe.arenas().pairs().used() == 0,
          "arenas not empty at the end");
  } else {
    // every accepted job is either finished or handed back by drain, once
    CHECK(ex.finished + dropped + migrated == accepted, "%d finished + %d dropped + %d migrated != %d accepted",
          ex.finished, dropped, migrated, accepted);
    CHECK(pipe.empty() && !pipe.in_flight(), "drain left state behind");
  }
  for (FJob* j : all) {
    CHECK(j->waits <= 1, "admission wait counted %d times for job %d", j->waits, j->id);
    delete j;
  }
  return true;
}

int main() {
  int n = 0;
  for (uint64_t seed = 1; seed <= 300; ++seed) n += ring_random(seed);
  n += ring_wrap_case();
  n += plan_cases();
  for (uint64_t seed = 1; seed <= 200; ++seed) n += pipeline_random(seed, -1);
  for (uint64_t seed = 1; seed <= 50; ++seed) n += pipeline_random(1000 + seed, 5 + (int)(seed * 13 % 200));
  for (uint64_t seed = 1; seed <= 100; ++seed) n += pipeline_random(2000 + seed, -1, true);
  for (uint64_t seed = 1; seed <= 30; ++seed) n += pipeline_random(3000 + seed, 5 + (int)(seed * 17 % 200), true);
  if (g_fail) {
    fprintf(stderr, "%d checks passed before the failure\n", n);
    return 1;
  }
  printf("ALL OK (%d scenarios)\n", n);
  return 0;
}
