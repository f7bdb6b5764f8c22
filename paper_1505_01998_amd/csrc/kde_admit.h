// kde_admit.h -- admission rule of the serving loop: which queued requests
// join the device now.  Host-only and independent of HIP, so the rule is
// exercised on the CPU by itself.
//
// Requests are considered in arrival order.  A request is admitted when a
// slot is free, its footprint fits the HBM budget next to what is resident,
// and the arena places its block.  The first request that does not fit (the
// head) is not passed in a way that would delay it: its "shadow" is the
// point at which enough resident requests have finished for it to fit,
// taking residents in order of least remaining work (the order the
// scheduler favours, so the order they are expected to finish in).  A later
// request may be admitted before the head only if it also fits at that
// point next to the head, counting it as still resident then.  So small
// requests do not wait behind a large one, and the large one is admitted as
// soon as the residents ahead of it finish.  If the head fits the budget but
// the arena cannot place it (its free space is split), nothing more is
// admitted until it is placed, so the arena drains towards one free range.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace kde {

struct Resident {
  uint64_t fp;       // footprint
  double remaining;  // pair-term evaluations left
};

// fp[k], work[k]: footprint and pair-term evaluations of the k-th queued
// request (arrival order), each footprint at most `budget`; residents: the
// requests on the device.  place(k) tries to reserve the k-th request's block
// and returns whether it succeeded.  Returns the admitted positions in order;
// `used` is updated.
template <typename Place>
std::vector<size_t> admit(const std::vector<uint64_t>& fp, const std::vector<double>& work,
                          std::vector<Resident> residents, uint64_t budget, uint64_t& used, int free_slots,
                          Place&& place) {
  std::vector<size_t> out;
  bool blocked = false;
  uint64_t room = 0;  // budget left at the head's shadow point, next to the head
  for (size_t k = 0; k < fp.size() && (int)out.size() < free_slots; ++k) {
    const bool fits = used + fp[k] <= budget;
    if (!blocked) {
      if (fits && place(k)) {
        used += fp[k];
        out.push_back(k);
        residents.push_back(Resident{fp[k], work[k]});
        continue;
      }
      if (fits) break;  // budget room but no contiguous range: let the arena drain
      blocked = true;
      std::stable_sort(residents.begin(), residents.end(),
                       [](const Resident& a, const Resident& b) { return a.remaining < b.remaining; });
      uint64_t freed = 0;
      for (const Resident& r : residents) {
        if (used - freed + fp[k] <= budget) break;
        freed += r.fp;
      }
      const uint64_t at_shadow = used - freed + fp[k];
      room = at_shadow <= budget ? budget - at_shadow : 0;
      continue;
    }
    if (fits && fp[k] <= room && place(k)) {
      used += fp[k];
      room -= fp[k];
      out.push_back(k);
    }
  }
  return out;
}

}  // namespace kde
