// ems_slotmap.h -- the event id -> slot table that the library keeps in device
// memory: open addressing with linear probing over a power-of-two array of 64-bit
// entries (slot + 1) << 32 | id, 0 = empty, kMapTomb = erased.  Erased entries stay
// as tombstones (probe runs are not shifted while other lanes probe them) until the
// table is rebuilt.  The probing is written once, for the kernels and for a plain
// CPU build under the sanitizers; Cas supplies the compare-and-swap (a device
// atomic in the kernels, a plain one on the CPU) and EMS_HD the function's targets.
#pragma once

#include <stdint.h>

#ifndef EMS_HD
#define EMS_HD __host__ __device__
#endif

namespace ems {

constexpr unsigned long long kMapTomb = 0xFFFFFFFFull << 32;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

EMS_HD inline uint32_t map_home(uint32_t id, uint32_t mask) {
  return (uint32_t)(((unsigned long long)id * 0x9E3779B97F4A7C15ull) >> 32) & mask;
}

EMS_HD inline unsigned long long map_entry(uint32_t id, uint32_t slot) {
  return ((unsigned long long)(slot + 1u) << 32) | id;
}

// Insert id -> slot: 1 if inserted, 0 if id is present already, -1 if no empty entry
// is left on the probe path.  Entries only go from empty to taken while inserts run,
// so a stale read of an empty entry is corrected by the compare-and-swap's answer.
template <class Cas>
EMS_HD int map_insert(unsigned long long* map, uint32_t mask, uint32_t id, uint32_t slot) {
  const unsigned long long entry = map_entry(id, slot);
  uint32_t h = map_home(id, mask);
  for (uint32_t p = 0; p <= mask; ++p, h = (h + 1u) & mask) {
    unsigned long long v = map[h];
    if (v == 0ull) {
      const unsigned long long old = Cas::cas(&map[h], 0ull, entry);
      if (old == 0ull) return 1;
      v = old;
    }
    if (v != kMapTomb && (uint32_t)v == id) return 0;
  }
  return -1;
}

// Index of the entry of id, or kNoSlot.
EMS_HD inline uint32_t map_find(const unsigned long long* map, uint32_t mask, uint32_t id) {
  uint32_t h = map_home(id, mask);
  for (uint32_t p = 0; p <= mask; ++p, h = (h + 1u) & mask) {
    const unsigned long long v = map[h];
    if (v == 0ull) return kNoSlot;
    if (v != kMapTomb && (uint32_t)v == id) return h;
  }
  return kNoSlot;
}

// Slot held by entry h (h from map_find).
EMS_HD inline uint32_t map_slot(const unsigned long long* map, uint32_t h) {
  return (uint32_t)(map[h] >> 32) - 1u;
}

// Erase the entry id -> slot if present (the entry itself, not just the id: a batch
// that is taken back erases only what it entered).
EMS_HD inline void map_erase(unsigned long long* map, uint32_t mask, uint32_t id, uint32_t slot) {
  const unsigned long long entry = map_entry(id, slot);
  uint32_t h = map_home(id, mask);
  for (uint32_t p = 0; p <= mask; ++p, h = (h + 1u) & mask) {
    const unsigned long long v = map[h];
    if (v == 0ull) return;
    if (v == entry) {
      map[h] = kMapTomb;
      return;
    }
  }
}

// Free slots are the set bits of a bitmap; pre[w] counts the set bits of words
// [0, w).  The free slot of rank r (0-based, in increasing slot order) is in the
// word w with pre[w] <= r < pre[w + 1], at the bit of rank r - pre[w] within it.
// The device computes pre per tile of kFreeTile words, then adds the tiles'
// offsets.
constexpr uint32_t kFreeTile = 4096;

// Index (0..31) of the set bit of rank r in x (r < popcount(x)): binary descent on
// the popcounts of the low halves.
EMS_HD inline uint32_t bit_select(uint32_t x, uint32_t r) {
  uint32_t pos = 0;
  for (uint32_t half = 16; half > 0; half >>= 1) {
    const uint32_t low = x & ((1u << half) - 1u);
    const uint32_t c = (uint32_t)__builtin_popcount(low);
    if (r >= c) {
      r -= c;
      x >>= half;
      pos += half;
    } else {
      x = low;
    }
  }
  return pos;
}

// Slot of free rank r given the bitmap and its word prefix counts (words + 1
// entries); r must be below pre[words].
EMS_HD inline uint32_t free_slot_of_rank(const uint32_t* bits, const uint32_t* pre, uint32_t words,
                                         uint32_t r) {
  uint32_t lo = 0, hi = words;  // pre[lo] <= r < pre[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= r) lo = mid;
    else hi = mid;
  }
  return lo * 32u + bit_select(bits[lo], r - pre[lo]);
}

}  // namespace ems
