// Host-only checks of the serving loop's bookkeeping (no GPU): the arena
// allocator (kde_arena.h) and the admission rule (kde_admit.h), driven by a
// seeded random workload.  Prints "OK" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "kde_admit.h"
#include "kde_arena.h"

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

static void arena_random(uint64_t seed) {
  std::mt19937_64 rng(seed);
  const uint64_t size = 1 << 24;
  kde::Arena a(size);
  std::map<int64_t, uint64_t> live;  // offset -> rounded length
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const uint64_t want = 1 + rng() % (1 << 18);
      const int64_t off = a.alloc(want);
      if (off < 0) {
        CHECK(a.largest_free() < kde::Arena::round(want));
        continue;
      }
      const uint64_t len = kde::Arena::round(want);
      CHECK(off % kde::Arena::kAlign == 0 && (uint64_t)off + len <= a.size());
      auto nx = live.lower_bound(off);  // no overlap with live ranges
      if (nx != live.end()) CHECK((uint64_t)off + len <= (uint64_t)nx->first);
      if (nx != live.begin()) {
        auto pv = std::prev(nx);
        CHECK((uint64_t)pv->first + pv->second <= (uint64_t)off);
      }
      live[off] = len;
    } else {
      auto it = live.begin();
      std::advance(it, rng() % live.size());
      CHECK(a.release(it->first));
      live.erase(it);
    }
    uint64_t sum = 0;
    for (auto& kv : live) sum += kv.second;
    CHECK(sum == a.in_use() && a.used_ranges() == live.size());
  }
  CHECK(!a.release(12345));  // not an allocated offset
  for (auto& kv : live) CHECK(a.release(kv.first));
  CHECK(a.in_use() == 0 && a.free_ranges() == 1 && a.largest_free() == a.size());
  CHECK(a.alloc(a.size()) == 0);
}

// A queue of requests with footprints and work; each admitted request stays
// resident for as many iterations as its work.  Checks: the budget is never
// exceeded, every request is admitted, and waits stay bounded (no request is
// starved by later, smaller ones).
static void admission_random(uint64_t seed) {
  std::mt19937_64 rng(seed);
  const uint64_t budget = 1 << 22;
  kde::Arena arena(budget);
  struct Req {
    int id;
    uint64_t fp;
    int work;
  };
  std::deque<Req> queue;
  struct Res {
    int id;
    int64_t off;
    uint64_t fp;
    int left;
  };
  std::vector<Res> resident;
  uint64_t used = 0;
  int next_id = 0, admitted_total = 0;
  const int total = 3000, slots = 16;
  std::vector<int> admitted_at(total, -1), arrived_at(total, -1);
  int iter = 0;
  for (; iter < 200000 && admitted_total < total; ++iter) {
    // arrivals: mostly small, sometimes close to the whole budget
    for (int a = rng() % 3; a > 0 && next_id < total; --a) {
      const bool big = rng() % 10 == 0;
      const uint64_t fp = big ? budget / 2 + rng() % (budget / 2) : 256 + rng() % (budget / 16);
      arrived_at[next_id] = iter;
      queue.push_back(Req{next_id++, kde::Arena::round(fp), big ? 4 + (int)(rng() % 8) : 1 + (int)(rng() % 4)});
    }
    std::vector<uint64_t> fps;
    std::vector<double> work;
    for (auto& q : queue) {
      fps.push_back(q.fp);
      work.push_back(q.work);
    }
    std::vector<kde::Resident> res;
    for (auto& r : resident) res.push_back(kde::Resident{r.fp, (double)r.left});
    std::vector<int64_t> offs(queue.size(), -1);
    const int free_slots = slots - (int)resident.size();
    const uint64_t before = used;
    std::vector<size_t> take = kde::admit(fps, work, res, budget, used, free_slots, [&](size_t k) {
      offs[k] = arena.alloc(fps[k]);
      return offs[k] >= 0;
    });
    CHECK(used <= budget && (int)take.size() <= free_slots);
    uint64_t added = 0;
    for (size_t k : take) added += fps[k];
    CHECK(used == before + added);
    for (size_t k = 0; k < offs.size(); ++k) {  // only admitted requests hold a range
      bool in = false;
      for (size_t t : take) in |= (t == k);
      if (!in) CHECK(offs[k] < 0);
    }
    for (size_t t = take.size(); t-- > 0;) {
      const size_t k = take[t];
      resident.push_back(Res{queue[k].id, offs[k], queue[k].fp, queue[k].work});
      admitted_at[queue[k].id] = iter;
      ++admitted_total;
      queue.erase(queue.begin() + (long)k);
    }
    // one iteration of work; finished requests leave
    std::vector<Res> keep;
    for (auto& r : resident) {
      if (--r.left > 0) {
        keep.push_back(r);
      } else {
        CHECK(arena.release(r.off));
        used -= r.fp;
      }
    }
    resident.swap(keep);
    CHECK(arena.in_use() == used);
  }
  CHECK(admitted_total == total);
  int worst = 0;
  for (int id = 0; id < total; ++id) worst = std::max(worst, admitted_at[id] - arrived_at[id]);
  CHECK(worst < 400);
}

static void admission_cases() {
  const uint64_t U = 256;
  auto run = [](std::vector<uint64_t> fp, std::vector<kde::Resident> res, uint64_t budget, uint64_t used,
                int slots) {
    kde::Arena arena(budget);
    if (used) CHECK(arena.alloc(used) == 0);
    std::vector<double> work(fp.size(), 1.0);
    return kde::admit(fp, work, res, budget, used, slots, [&](size_t k) { return arena.alloc(fp[k]) >= 0; });
  };
  // budget 100 units with a resident of 60: the 50-unit head waits; a 30-unit
  // request passes (30 + 50 fit once the resident is done), a 15-unit one then
  // exceeds the budget now, a 10-unit one passes
  std::vector<size_t> t = run({50 * U, 30 * U, 15 * U, 10 * U}, {{60 * U, 5.0}}, 100 * U, 60 * U, 8);
  CHECK(t.size() == 2 && t[0] == 1 && t[1] == 3);
  // two residents; the head needs the one with least work to finish: a later
  // request passes only within what is left next to the head at that point
  // (the 30-unit resident, least work, must finish: then 40 + 50 leave room 10)
  t = run({50 * U, 30 * U, 20 * U}, {{40 * U, 9.0}, {30 * U, 1.0}}, 100 * U, 70 * U, 8);
  CHECK(t.empty());
  t = run({45 * U, 30 * U, 10 * U}, {{40 * U, 9.0}, {30 * U, 1.0}}, 100 * U, 70 * U, 8);
  CHECK(t.size() == 1 && t[0] == 2);  // room 15 at the shadow
  // a head that fits is simply admitted, in order; slots bound the count
  t = run({10 * U, 10 * U, 10 * U, 10 * U}, {}, 100 * U, 0, 3);
  CHECK(t.size() == 3 && t[0] == 0 && t[2] == 2);
}

int main() {
  for (uint64_t s = 1; s <= 4; ++s) arena_random(1998000 + s);
  admission_cases();
  for (uint64_t s = 1; s <= 3; ++s) admission_random(1998100 + s);
  std::printf("OK\n");
  return 0;
}
