// CPU test of the request server's memory policy (paper_2206_05269_amd/csrc/wc_admission.h)
// with a fake executor and a fake clock: workers, requests, counts and client releases are
// discrete events; no GPU, no threads. Prints one line per scenario; exit status 0 when every
// check holds.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <string>
#include <vector>

#include "wc_admission.h"

using wc::Admission;
using wc::Admit;

static int failures = 0;
#define CHECK(c)                                                           \
  do {                                                                     \
    if (!(c)) {                                                            \
      printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);                  \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

constexpr uint64_t MiB = 1ull << 20;

// The sequence that failed a request under a single first-fit pool: two workers count side by
// side, each keeps its resident table while still holding count memory, both finish, then a
// large request arrives. With resident tables placed first-fit they land between the freed
// count regions and the large request finds no contiguous block although the total would do.
static void scenario_fragmentation() {
  Admission a;
  a.init(64 * MiB);
  uint64_t ca, cb, ra, rb, big;
  CHECK(a.try_count(20 * MiB, &ca) == Admit::kGranted);
  CHECK(a.try_count(20 * MiB, &cb) == Admit::kGranted);
  CHECK(a.try_resident(1 * MiB, &ra) == Admit::kGranted);
  CHECK(ra + 1 * MiB == 64 * MiB);  // the top of the pool
  a.free_count(ca);
  CHECK(a.try_resident(1 * MiB, &rb) == Admit::kGranted);
  a.free_count(cb);
  CHECK(a.holders == 0);
  CHECK(a.pool.largest_free() == 62 * MiB);
  CHECK(a.try_count(60 * MiB, &big) == Admit::kGranted);
  a.free_count(big);
  // the same sequence with resident tables taken first-fit (the old policy) splits the pool
  wc::TwoEndedPool p;
  p.init(64 * MiB);
  uint64_t x, y, r1, r2;
  p.alloc_low(20 * MiB, &x);
  p.alloc_low(20 * MiB, &y);
  p.alloc_low(1 * MiB, &r1);
  p.release(x);
  p.alloc_low(1 * MiB, &r2);  // lands in the freed region of the first count
  p.release(y);
  CHECK(p.free_bytes() == 62 * MiB && p.largest_free() < 60 * MiB);
  printf("ok fragmentation: largest free block %llu MiB (first fit: %llu MiB)\n",
         (unsigned long long)(a.pool.largest_free() / MiB),
         (unsigned long long)(p.largest_free() / MiB));
}

// Resident tables fill the pool and nothing runs: a count fails at once (only the client can
// free memory); while something runs, the same request waits.
static void scenario_resident_full() {
  Admission a;
  a.init(16 * MiB);
  uint64_t c, r[15], q;
  CHECK(a.try_count(1 * MiB, &c) == Admit::kGranted);
  for (int i = 0; i < 15; ++i) CHECK(a.try_resident(1 * MiB, &r[i]) == Admit::kGranted);
  CHECK(a.try_count(2 * MiB, &q) == Admit::kWait);  // the running count will return 1 MiB
  a.free_count(c);
  CHECK(a.try_count(2 * MiB, &q) == Admit::kFail);  // nothing runs, resident tables hold 15
  CHECK(a.try_count(1 * MiB, &q) == Admit::kGranted);
  a.free_count(q);
  a.free_resident(r[3]);
  a.free_resident(r[4]);
  CHECK(a.try_count(2 * MiB, &q) == Admit::kGranted);  // the released tables left 2 MiB
  a.free_count(q);
  // a request larger than the budget fails on an empty pool
  Admission e;
  e.init(4 * MiB);
  CHECK(e.try_count(5 * MiB, &q) == Admit::kFail);
  printf("ok resident_full\n");
}

// Two holders need resident memory and none is free: the first waits (the other still
// holds count memory it will return), the second fails, returns its count memory, and the
// first then gets its block.
static void scenario_resident_waiters() {
  Admission a;
  a.init(8 * MiB);
  uint64_t c1, c2, r1, r2;
  CHECK(a.try_count(4 * MiB, &c1) == Admit::kGranted);
  CHECK(a.try_count(4 * MiB, &c2) == Admit::kGranted);
  CHECK(a.try_resident(1 * MiB, &r1) == Admit::kWait);
  ++a.resident_waiters;  // worker 1 waits
  CHECK(a.try_resident(1 * MiB, &r2) == Admit::kFail);  // worker 2 would wait on worker 1
  a.free_count(c2);                                      // worker 2 gives up its request
  --a.resident_waiters;                                  // worker 1 is woken
  CHECK(a.try_resident(1 * MiB, &r1) == Admit::kGranted);
  a.free_count(c1);
  a.free_resident(r1);
  CHECK(a.pool.free_bytes() == 8 * MiB && a.pool.n_used() == 0 && a.holders == 0);
  printf("ok resident_waiters\n");
}

// A merge pins its inputs at submission; a release before the merge has run defers the free.
static void scenario_merge_pins() {
  Admission a;
  a.init(8 * MiB);
  uint64_t r;
  CHECK(a.try_resident(1 * MiB, &r) == Admit::kGranted);
  wc::ResidentLife life;
  life.pin();                // merge submitted
  CHECK(!life.release());    // the client releases the input: not freed yet
  CHECK(a.pool.free_bytes() == 7 * MiB);
  if (life.unpin()) a.free_resident(r);  // the merge is done
  CHECK(a.pool.free_bytes() == 8 * MiB);
  wc::ResidentLife two;
  two.pin();
  two.pin();
  CHECK(!two.unpin());
  CHECK(!two.unpin());  // not released: stays
  CHECK(two.release());  // released with no reader: freed at once
  printf("ok merge_pins\n");
}

// ---- fake executor: workers take requests in arrival order; times are fake seconds ------
static uint64_t TwoEndedRound(uint64_t b) { return wc::TwoEndedPool::round(b); }

struct Req {
  int id;
  double arrive;
  uint64_t count_bytes, resident_bytes;
  double duration;      // device time of the count
  double release_after; // the client releases the table this long after completion (<0: never)
  // outcome
  int status = 0;  // 0 pending, 1 done, -2 failed (ENOMEM)
  double done = 0;
  uint64_t res_off = 0;
};

struct Worker {
  int state = 0;  // 0 idle, 1 waiting count, 2 counting, 3 waiting resident
  Req* r = nullptr;
  uint64_t count_off = 0;
  double until = 0;
};

struct Trace {
  std::vector<std::string> lines;
  void add(double t, const char* what, int id) {
    char b[96];
    snprintf(b, sizeof b, "%.6f %s %d", t, what, id);
    lines.push_back(b);
  }
};

static Trace simulate(std::vector<Req>& reqs, uint64_t budget, int n_workers, int* fails,
                      bool check_rules) {
  Admission a;
  a.init(budget);
  std::vector<Worker> W(n_workers);
  std::deque<Req*> queue;
  struct Rel {
    double t;
    Req* r;
  };
  std::vector<Rel> releases;
  Trace tr;
  size_t next = 0;
  double now = 0;
  *fails = 0;
  for (int guard = 0; guard < 1000000; ++guard) {
    // progress at the current time until nothing changes
    bool changed = true;
    while (changed) {
      changed = false;
      while (next < reqs.size() && reqs[next].arrive <= now) {
        queue.push_back(&reqs[next++]);
        changed = true;
      }
      for (size_t i = 0; i < releases.size();) {
        if (releases[i].t <= now) {
          a.free_resident(releases[i].r->res_off);
          tr.add(now, "release", releases[i].r->id);
          releases.erase(releases.begin() + i);
          changed = true;
        } else {
          ++i;
        }
      }
      for (auto& w : W) {
        if (w.state == 0 && !queue.empty()) {
          w.r = queue.front();
          queue.pop_front();
          w.state = 1;
          changed = true;
        }
        if (w.state == 1) {
          const uint64_t largest = a.pool.largest_free();
          const uint32_t holders = a.holders;
          Admit d = a.try_count(w.r->count_bytes, &w.count_off);
          if (d == Admit::kGranted) {
            w.state = 2;
            w.until = now + w.r->duration;
            tr.add(now, "start", w.r->id);
            changed = true;
          } else if (d == Admit::kFail) {
            // the rule: fail only when nothing holds count memory and no block fits
            if (check_rules) CHECK(holders == 0 && largest < TwoEndedRound(w.r->count_bytes));
            w.r->status = -2;
            ++*fails;
            tr.add(now, "enomem", w.r->id);
            w.state = 0;
            changed = true;
          }
        }
        if (w.state == 2 && w.until <= now) {
          w.state = 3;
          changed = true;
        }
        if (w.state == 3) {
          const bool was_waiting = w.until < 0;
          if (was_waiting) --a.resident_waiters;
          Admit d = a.try_resident(w.r->resident_bytes, &w.r->res_off);
          if (d == Admit::kGranted) {
            a.free_count(w.count_off);
            w.r->status = 1;
            w.r->done = now;
            tr.add(now, "done", w.r->id);
            if (w.r->release_after >= 0) releases.push_back({now + w.r->release_after, w.r});
            w.state = 0;
            changed = true;
          } else if (d == Admit::kFail) {
            if (check_rules) CHECK(a.holders <= a.resident_waiters + 1);
            a.free_count(w.count_off);
            w.r->status = -2;
            ++*fails;
            tr.add(now, "enomem-resident", w.r->id);
            w.state = 0;
            changed = true;
          } else {
            ++a.resident_waiters;
            w.until = -1;  // marks "waiting" for the next try
          }
        }
      }
    }
    // next event time
    double t = 1e300;
    if (next < reqs.size()) t = std::min(t, reqs[next].arrive);
    for (auto& r : releases) t = std::min(t, r.t);
    for (auto& w : W)
      if (w.state == 2) t = std::min(t, w.until);
    if (t == 1e300) break;
    now = t;
  }
  for (auto& w : W)
    if (w.state == 3) --a.resident_waiters;
  // every request ended; all memory that is not resident came back
  uint64_t resident = 0;
  for (auto& r : reqs) {
    CHECK(r.status != 0);
    if (r.status == 1 && r.release_after < 0) resident += TwoEndedRound(r.resident_bytes);
  }
  CHECK(a.holders == 0 && a.resident_waiters == 0);
  CHECK(a.pool.free_bytes() + resident == budget);
  return tr;
}

static std::vector<Req> workload(uint64_t seed, int n, uint64_t budget) {
  // lognormal-ish sizes from a fixed linear congruential sequence (deterministic)
  std::vector<Req> v;
  uint64_t x = seed * 6364136223846793005ull + 1442695040888963407ull;
  auto u = [&] {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(x >> 11) / 9007199254740992.0;
  };
  double t = 0;
  for (int i = 0; i < n; ++i) {
    t += -0.001 * __builtin_log(1.0 - u());
    const double z = u() + u() + u() - 1.5;  // roughly normal
    uint64_t len = (uint64_t)(256.0 * 1024 * __builtin_exp(2.0 * z));
    len = std::max<uint64_t>(1024, std::min<uint64_t>(len, budget / 6));
    Req r;
    r.id = i;
    r.arrive = t;
    r.count_bytes = 4 * len;
    r.release_after = (i % 3 == 0) ? -1.0 : 0.002 + 0.001 * (i % 7);
    // tables that are never released are large, so that they fill the pool during the run
    r.resident_bytes = r.release_after < 0 ? len : len / 8 + 4096;
    r.duration = 1e-6 * (double)len / 1000.0 + 1e-5;
    v.push_back(r);
  }
  return v;
}

// Poisson arrivals, lognormal sizes up to a sixth of the budget, tables released after a
// while (a third never): every failure obeys the rules, memory balances, and the run is
// deterministic.
static void scenario_executor() {
  const uint64_t budget = 64 * MiB;
  int total_fails = 0;
  for (uint64_t seed = 1; seed <= 6; ++seed) {
    for (int workers : {1, 4, 8}) {
      auto r1 = workload(seed, 400, budget);
      auto r2 = workload(seed, 400, budget);
      int f1, f2;
      Trace t1 = simulate(r1, budget, workers, &f1, true);
      Trace t2 = simulate(r2, budget, workers, &f2, true);
      CHECK(t1.lines == t2.lines);
      total_fails += f1;
    }
  }
  CHECK(total_fails > 0);  // the rules were exercised
  // with every table released, nothing fails
  for (uint64_t seed = 1; seed <= 6; ++seed) {
    auto r = workload(seed, 400, budget);
    for (auto& q : r) q.release_after = 0.0005;
    int f;
    simulate(r, budget, 4, &f, true);
    CHECK(f == 0);
  }
  printf("ok executor: %d requests failed across runs where unreleased tables fill the pool\n",
         total_fails);
}

int main() {
  scenario_fragmentation();
  scenario_resident_full();
  scenario_resident_waiters();
  scenario_merge_pins();
  scenario_executor();
  if (failures) {
    printf("%d checks failed\n", failures);
    return 1;
  }
  printf("all ok\n");
  return 0;
}
