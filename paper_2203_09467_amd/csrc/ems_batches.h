// ems_batches.h -- events waiting for admission, kept per submitted batch (plain
// C++, no HIP: also built on its own for the sanitizer tests).  The host holds no
// record per event: a batch keeps the primary offsets it was submitted with and,
// when admission is limited by energy, the running sum of its events' energies, and
// admission cuts it with two binary searches.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

namespace ems {

struct PendingBatch {
  // primaries of event e: off()[e] .. off()[e+1]-1, off()[0] = 0: the caller's array
  // while it is lent (for the duration of the call that submitted it), else a copy
  const int64_t* lent = nullptr;
  std::vector<int64_t> own;
  uint32_t ne = 0;
  std::vector<double> ecum;  // energy of events [0, e); empty when not tracked
  uint32_t next = 0;         // first event not yet admitted
  uint32_t n_events() const { return ne; }
  const int64_t* off() const { return lent ? lent : own.data(); }
};

struct Admitted {
  uint64_t prims = 0;
  uint64_t events = 0;
  double energy = 0.0;
};

class PendingEvents {
 public:
  // Queue a batch of ne events (off has ne + 1 entries, off[0] = 0); e, if not
  // null, holds the kinetic energy of each event.  With lend, off is used in place
  // until keep() is called, which must happen before the caller's array goes away.
  void push(const int64_t* off, uint32_t ne, const double* e, bool lend = false) {
    if (ne == 0) return;
    PendingBatch b;
    b.ne = ne;
    if (lend) b.lent = off;
    else b.own.assign(off, off + ne + 1);
    if (e) {
      b.ecum.resize(ne + 1);
      b.ecum[0] = 0.0;
      for (uint32_t j = 0; j < ne; ++j) b.ecum[j + 1] = b.ecum[j] + e[j];
    }
    events_ += ne;
    prims_ += (uint64_t)(off[ne] - off[0]);
    q_.push_back(std::move(b));
  }

  // Admit whole events in submission order while the pool (n_active tracks) plus
  // the primaries admitted stay within room and, with budget > 0, the energy e_now
  // plus that of the events admitted stays within budget (no energy limit while
  // that energy is zero); a pool with no track and nothing admitted yet always
  // takes the next event, so admission cannot stall.
  Admitted admit(uint64_t n_active, uint64_t room, double e_now, double budget) {
    Admitted r;
    while (!q_.empty()) {
      PendingBatch& b = q_.front();
      const uint32_t a = b.next, n = b.n_events();
      const int64_t* off = b.off();
      const bool energy = budget > 0.0 && !b.ecum.empty();
      const uint64_t used = n_active + r.prims;
      const double e0 = e_now + r.energy;
      // event a alone
      const int64_t pa = off[a + 1] - off[a];
      const double ea = energy ? b.ecum[a + 1] - b.ecum[a] : 0.0;
      const bool first = used == 0;
      const bool fits_a = used + (uint64_t)pa <= room && !(energy && e0 > 0.0 && e0 + ea > budget);
      if (!first && !fits_a) break;
      // events a .. c - 1 with c the end of the longest prefix within both limits
      uint32_t c = a + 1;
      if (used + (uint64_t)pa <= room) {
        const int64_t lim = off[a] + (int64_t)(room - used);
        c = (uint32_t)(std::upper_bound(off + a + 1, off + n + 1, lim) - off) - 1;
        c = std::max(c, a + 1);
      }
      if (energy && c > a + 1) {
        const double elim = budget - e0 + b.ecum[a];
        const uint32_t ce =
            (uint32_t)(std::upper_bound(b.ecum.begin() + a + 1, b.ecum.end(), elim) - b.ecum.begin()) - 1;
        c = std::min(c, std::max(ce, a + 1));
      }
      r.prims += (uint64_t)(off[c] - off[a]);
      r.events += c - a;
      if (!b.ecum.empty()) r.energy += b.ecum[c] - b.ecum[a];
      events_ -= c - a;
      prims_ -= (uint64_t)(off[c] - off[a]);
      b.next = c;
      if (c < n) break;  // the next event does not fit
      q_.pop_front();
    }
    return r;
  }

  // Copy every lent offsets array that is still needed.
  void keep() {
    for (PendingBatch& b : q_)
      if (b.lent) {
        b.own.assign(b.lent, b.lent + b.ne + 1);
        b.lent = nullptr;
      }
  }

  uint64_t events() const { return events_; }
  uint64_t prims() const { return prims_; }
  bool empty() const { return q_.empty(); }
  void clear() {
    q_.clear();
    events_ = prims_ = 0;
  }

 private:
  std::deque<PendingBatch> q_;
  uint64_t events_ = 0, prims_ = 0;
};

}  // namespace ems
