/*
 * philox.c -- counter-based random numbers for the oracle (test infrastructure).
 *
 * Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a
 * 2x32-bit key; each round multiplies counter words 0 and 2 by two fixed
 * odd constants, mixes high/low halves with the other words and the key,
 * and the key is advanced by two Weyl increments between rounds.
 * Pinned by the published known-answer vectors (tests/golden/philox_kat.txt).
 *
 * Stream layout (a reading: the paper uses XORWOW with thread-dependent
 * streams, paper Sec. 3.2; here streams are keyed by track lineage so that
 * results do not depend on scheduling):
 *   draw d of step s of a track with key (k0,k1,k2), run seed S:
 *     counter = (k0, k1, s, d >> 1), key = (S, k2);
 *     words (2j, 2j+1) with j = d & 1 form a 64-bit integer w = hi:lo;
 *     u = (floor(w / 2^12) + 1/2) * 2^-52, so 0 < u < 1 exactly.
 *   primary key   = first three words of Philox(ctr = (event, index, 0, 0), key = (S, 0x243F6A88))
 *   child key     = first three words of Philox(ctr = (k0, k1, k2, step), key = (S, 0xB7E15162 ^ ordinal))
 */
#include "oracle.h"

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  out[0] = c[0];
  out[1] = c[1];
  out[2] = c[2];
  out[3] = c[3];
}

double or_uniform(uint32_t seed, const uint32_t key[3], uint32_t step, uint32_t draw) {
  const uint32_t ctr[4] = {key[0], key[1], step, draw >> 1};
  const uint32_t k[2] = {seed, key[2]};
  uint32_t o[4];
  or_philox4x32_10(ctr, k, o);
  const int j = (int)(draw & 1u);
  const uint64_t w = ((uint64_t)o[2 * j] << 32) | (uint64_t)o[2 * j + 1];
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

void or_primary_key(uint32_t seed, uint32_t event_id, uint32_t index, uint32_t out[3]) {
  const uint32_t ctr[4] = {event_id, index, 0u, 0u};
  const uint32_t k[2] = {seed, 0x243F6A88u};
  uint32_t o[4];
  or_philox4x32_10(ctr, k, o);
  out[0] = o[0];
  out[1] = o[1];
  out[2] = o[2];
}

void or_child_key(uint32_t seed, const uint32_t parent[3], uint32_t step, uint32_t ordinal,
                  uint32_t out[3]) {
  const uint32_t ctr[4] = {parent[0], parent[1], parent[2], step};
  const uint32_t k[2] = {seed, 0xB7E15162u ^ ordinal};
  uint32_t o[4];
  or_philox4x32_10(ctr, k, o);
  out[0] = o[0];
  out[1] = o[1];
  out[2] = o[2];
}
