// Randomised checks of the library's event bookkeeping, built on the CPU with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize.py:
//  * the id -> slot table (the probing the kernels run, here with a plain
//    compare-and-swap) against std::unordered_map, with erased entries left as
//    tombstones and the table rebuilt as the library does past a quarter of them;
//  * the free-slot bitmap (a batch takes the lowest free slots in order) against a
//    std::set;
//  * admission of queued batches (two binary searches per batch) against the same
//    rule applied event by event.  Energies are integers, so every sum is exact and
//    both sides must take identical decisions.
#include <cstdio>
#include <deque>
#include <random>
#include <set>
#include <unordered_map>
#include <vector>

#define EMS_HD
#include "ems_batches.h"
#include "ems_slotmap.h"

struct HostCas {
  static unsigned long long cas(unsigned long long* p, unsigned long long cmp, unsigned long long val) {
    const unsigned long long old = *p;
    if (old == cmp) *p = val;
    return old;
  }
};

static int fuzz_map() {
  for (uint32_t E : {1u, 7u, 64u, 1000u}) {
    uint32_t cap = 16;
    while (cap < 2 * E) cap <<= 1;
    const uint32_t mask = cap - 1;
    std::vector<unsigned long long> map(cap, 0ull);
    std::vector<uint32_t> free_slots, slot_id(E, 0);
    std::vector<int> used(E, 0);
    for (uint32_t i = 0; i < E; ++i) free_slots.push_back(E - 1 - i);
    std::unordered_map<uint32_t, uint32_t> ref;
    uint64_t tombs = 0;
    std::mt19937_64 rng(777 + E);
    const uint32_t id_range = 3 * E + 5;
    for (int op = 0; op < 200000; ++op) {
      const uint32_t id = (uint32_t)(rng() % id_range) * 2654435761u;  // colliding homes
      const int kind = (int)(rng() % 3);
      if (kind == 0 && !free_slots.empty()) {
        const uint32_t slot = free_slots.back();
        const int r = ems::map_insert<HostCas>(map.data(), mask, id, slot);
        if (r < 0) {
          std::printf("table full at E=%u\n", E);
          return 1;
        }
        if ((r == 1) != (ref.count(id) == 0)) {
          std::printf("insert mismatch E=%u op=%d\n", E, op);
          return 1;
        }
        if (r == 1) {
          ref[id] = slot;
          slot_id[slot] = id;
          used[slot] = 1;
          free_slots.pop_back();
        }
      } else if (kind == 1) {
        const uint32_t h = ems::map_find(map.data(), mask, id);
        const auto it = ref.find(id);
        if ((h == ems::kNoSlot) != (it == ref.end()) ||
            (h != ems::kNoSlot && ems::map_slot(map.data(), h) != it->second)) {
          std::printf("find mismatch E=%u op=%d\n", E, op);
          return 1;
        }
      } else {
        const auto it = ref.find(id);
        if (it == ref.end()) continue;
        ems::map_erase(map.data(), mask, id, it->second);
        used[it->second] = 0;
        free_slots.push_back(it->second);
        ref.erase(it);
        if (++tombs * 4 > cap) {  // rebuild: clear, re-enter every slot in use
          for (auto& v : map) v = 0ull;
          for (uint32_t s = 0; s < E; ++s)
            if (used[s] && ems::map_insert<HostCas>(map.data(), mask, slot_id[s], s) != 1) {
              std::printf("rebuild failed E=%u\n", E);
              return 1;
            }
          tombs = 0;
        }
      }
    }
  }
  return 0;
}

// The free-slot bitmap: a batch takes the slots of free ranks 0 .. ne-1, i.e. the
// ne lowest free slots in increasing order (the reference is a std::set).
static int fuzz_bitmap() {
  std::mt19937_64 rng(99);
  for (uint32_t n : {1u, 31u, 32u, 33u, 100u, 1000u}) {
    const uint32_t words = (n + 31) / 32;
    std::vector<uint32_t> bits(words, 0u), pre(words + 1, 0u);
    std::set<uint32_t> ref;
    for (uint32_t j = 0; j < n; ++j) {
      bits[j / 32] |= 1u << (j % 32);
      ref.insert(j);
    }
    std::vector<uint32_t> taken;
    for (int op = 0; op < 20000; ++op) {
      if (rng() % 2 == 0) {
        const uint32_t ne = ref.empty() ? 0 : 1 + (uint32_t)(rng() % ref.size());
        uint32_t run = 0;
        for (uint32_t w = 0; w < words; ++w) {
          pre[w] = run;
          run += (uint32_t)__builtin_popcount(bits[w]);
        }
        pre[words] = run;
        if (run != ref.size()) {
          std::printf("bitmap count mismatch n=%u\n", n);
          return 1;
        }
        std::vector<uint32_t> got;
        for (uint32_t e = 0; e < ne; ++e) got.push_back(ems::free_slot_of_rank(bits.data(), pre.data(), words, e));
        auto it = ref.begin();
        for (uint32_t e = 0; e < ne; ++e, ++it)
          if (got[e] != *it) {
            std::printf("bitmap take mismatch n=%u op=%d e=%u: %u vs %u\n", n, op, e, got[e], *it);
            return 1;
          }
        for (uint32_t g : got) {
          bits[g / 32] &= ~(1u << (g % 32));
          ref.erase(g);
          taken.push_back(g);
        }
      } else if (!taken.empty()) {
        const size_t k = 1 + rng() % taken.size();
        for (size_t j = 0; j < k; ++j) {
          const size_t i = rng() % taken.size();
          const uint32_t g = taken[i];
          taken[i] = taken.back();
          taken.pop_back();
          bits[g / 32] |= 1u << (g % 32);
          ref.insert(g);
        }
      }
    }
  }
  for (uint32_t x = 1; x != 0; x = x * 2654435761u + 12345u) {  // bit_select on assorted words
    if (x > 0xFFFF0000u) break;
    uint32_t r = 0;
    for (uint32_t b = 0; b < 32; ++b)
      if (x >> b & 1u) {
        if (ems::bit_select(x, r) != b) {
          std::printf("bit_select(%08x, %u) != %u\n", x, r, b);
          return 1;
        }
        ++r;
      }
  }
  return 0;
}

struct Ev {
  int64_t prims;
  double e;
};

static int fuzz_batches() {
  std::mt19937_64 rng(4242);
  for (int round = 0; round < 300; ++round) {
    ems::PendingEvents pe;
    std::deque<Ev> ref;
    uint64_t n_active = rng() % 50;
    for (int op = 0; op < 200; ++op) {
      if (rng() % 3 == 0) {
        const uint32_t ne = 1 + (uint32_t)(rng() % 40);
        const bool energy = rng() % 2;
        std::vector<int64_t> off(ne + 1, 0);
        std::vector<double> e(ne);
        for (uint32_t j = 0; j < ne; ++j) {
          off[j + 1] = off[j] + 1 + (int64_t)(rng() % 6);
          e[j] = (double)(1 + rng() % 100);
          ref.push_back({off[j + 1] - off[j], energy ? e[j] : 0.0});
        }
        // a batch without energies is admitted by room alone: the reference then
        // sees zero energies, which never exceed a budget
        // half of the batches are lent and kept (copied) before their array goes away
        const bool lend = rng() % 2;
        pe.push(off.data(), ne, energy ? e.data() : nullptr, lend);
        if (lend && rng() % 4 == 0) {  // some admission while lent
          const ems::Admitted got = pe.admit(n_active, 0, 0.0, 0.0);
          uint64_t m = 0, ev = 0;
          double ea = 0.0;
          while (!ref.empty() && n_active + m == 0) {  // room 0: only a first event goes
            m += (uint64_t)ref.front().prims;
            ea += ref.front().e;
            ev += 1;
            ref.pop_front();
          }
          if (got.prims != m || got.events != ev || got.energy != ea) {
            std::printf("lent admit mismatch round %d op %d\n", round, op);
            return 1;
          }
          n_active += m;
        }
        pe.keep();
      } else {
        const uint64_t room = rng() % 120;
        const double e_now = (double)(rng() % 3 == 0 ? 0 : rng() % 200);
        const double budget = (double)(rng() % 2 == 0 ? 0 : rng() % 400);
        const ems::Admitted got = pe.admit(n_active, room, e_now, budget);
        uint64_t m = 0, ev = 0;
        double ea = 0.0;
        while (!ref.empty()) {
          const Ev& x = ref.front();
          const bool first = n_active + m == 0;
          if (!first && n_active + m + (uint64_t)x.prims > room) break;
          const double en = e_now + ea;
          if (!first && budget > 0.0 && en > 0.0 && x.e > 0.0 && en + x.e > budget) break;
          m += (uint64_t)x.prims;
          ea += x.e;
          ev += 1;
          ref.pop_front();
        }
        if (got.prims != m || got.events != ev || got.energy != ea) {
          std::printf("admit mismatch round %d op %d: %llu/%llu events, %llu/%llu prims\n", round, op,
                      (unsigned long long)got.events, (unsigned long long)ev,
                      (unsigned long long)got.prims, (unsigned long long)m);
          return 1;
        }
        n_active = rng() % 2 ? 0 : n_active + m;
      }
      uint64_t rp = 0;
      for (const Ev& x : ref) rp += (uint64_t)x.prims;
      if (pe.events() != ref.size() || pe.prims() != rp) {
        std::printf("queue size mismatch round %d\n", round);
        return 1;
      }
    }
  }
  return 0;
}

int main() {
  if (fuzz_map() != 0) return 1;
  if (fuzz_batches() != 0) return 1;
  if (fuzz_bitmap() != 0) return 1;
  std::printf("slots ok\n");
  return 0;
}
