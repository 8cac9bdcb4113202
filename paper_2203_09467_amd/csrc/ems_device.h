// ems_device.h -- data layout shared by the host side of the library and its HIP kernels.
//
// Track state lives in HBM as structure-of-arrays, one slot per track, so that
// consecutive lanes of a wavefront read and write consecutive addresses (paper
// Sec. 2.1: parameter data separate from per-track state; one track per thread).
// The pool is double-buffered: a step iteration reads tracks [0, n) of one
// buffer and writes survivors and secondaries, compacted, into the other.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ems {

constexpr int kGrid = 200;            // nodes of the log energy grid, 1 keV .. 100 GeV
constexpr int kQ = 4;                 // quantities per (material, species, node)
constexpr int kMaxMat = 8;
// per-event ledger words: escaped (fixed point), killed (fixed point), pair conversions,
// annihilations, track-steps of photons, electrons, positrons, one spare word
constexpr int kLedger = 8;
constexpr int kLedgerSteps = 4;       // first of the three track-step words
// doubles per event row gathered for tally_read after the deposits: E_in, escaped,
// killed, pairs, annihilations, track-steps of photons, electrons, positrons
constexpr uint32_t kRowLedger = 8;
constexpr uint32_t kVolOut = 0x3FFFFFFu;  // meta volume of a primary that starts outside
constexpr uint32_t kRestStep = 0xFFFFFFFFu;
constexpr int kMaxTrial = 1000;
constexpr int kBlock = 256;
constexpr uint32_t kStageMaxBytes = 64u * 1024u;  // per-block LDS budget of the staged run data

// Tracks in flight, SoA.  meta = species (bits 0-1) | pending (bit 2) | queue of
// the pending interaction (bits 3-5) | volume << 6; a pending track ended its last
// step in an interaction that was put off for lack of output room.  Photons and
// charged tracks live in separate pools so that a wavefront steps one species
// class, each double-buffered.  A Pool passed to the step kernels is the set of
// all four buffers: for every field, buffer (class c, parity b) occupies elements
// [(2c + b) N, (2c + b + 1) N), so a lane picks its destination buffer with one
// integer offset.  src (diagnostics only) is the input index of a single-step call.
struct Pool {
  double *x, *y, *z, *u, *v, *w, *T, *nlam;
  uint32_t *k0, *k1, *k2, *evt, *nstep, *meta, *src;
};

// Tracks that ended their step in a discrete interaction (or a positron that
// stopped), one queue per process so that the interaction kernel runs each
// process in wavefronts of its own.  Post-step state with the step count not yet
// incremented (it keys the interaction's random numbers and children).
enum QueueId {
  kQCompton = 0, kQPhoto = 1, kQPair = 2, kQMoller = 3, kQBhabha = 4, kQBrems = 5,
  kQAnnihilation = 6, kQRest = 7, kNumQueues = 8
};

struct IQueue {
  double *x, *y, *z, *u, *v, *w, *T;
  uint32_t *k0, *k1, *k2, *evt, *nstep, *meta, *src;
  uint32_t capacity;  // per queue; queue q occupies [q * capacity, (q + 1) * capacity)
};

// Device counters of one iteration.  Each counter line is 256 bytes apart so that
// concurrent atomics on different counters meet different cache lines and memory
// channels; two 32-bit counters share one 64-bit word (low, high) and are
// advanced together by one 64-bit atomic.  Statistics are spread over kStatCopies
// lines (a block adds to copy blockIdx % kStatCopies) so that no single address
// takes one atomic per block.
enum CounterLine {
  kLOut = 0,      // output pools, survivors of the transport kernel: photons (low), charged (high)
  kLQueue = 1,    // lines 1..4: queue sizes (2i low, 2i+1 high)
  kLDone = 5,     // finished-event list length (low)
  kLAdmit = 6,    // admission cursors = pool sizes: photons (low), charged (high)
  kLOutI = 7,     // output pools, tracks written by the interaction kernel (low, high)
  kLStats = 8,    // lines 8 .. 8 + kStatCopies - 1: interval statistics, words kS*
};
constexpr int kStatCopies = 16;
constexpr int kNumLines = kLStats + kStatCopies;
// words of a statistics line (sums over the iterations of a sync interval)
enum StatWord {
  kSIn = 0,        // tracks in the pool at the start of an iteration
  kSStepG = 1,     // photon track-steps
  kSStepC = 2,     // charged track-steps
  kSStepPos = 3,   // positron track-steps
  kSPending = 4,   // pending tracks sent back to their interaction queue
  kSDeferred = 5,  // interactions put off (written back as pending tracks)
  kSOut = 6,       // tracks in the output pools
  kSQueued = 7,    // tracks queued for an interaction
  kSStall = 8,     // iterations in which no interaction could be done for lack of room
  kSBusy = 9,      // iterations with a non-empty pool
  kSPeak = 10      // largest pool
};
constexpr int kLineWords = 32;  // 64-bit words per line

struct MatParams {
  double Tc, kc;      // production thresholds (delta rays, brems photons)
  double Rtrk[3];     // range table at the tracking cut, per species
  float Rtrk_f[3];
  float Tc_f, kc_f;
  int vacuum;
};

// Immutable parameters of a run, passed by value to every step launch.
struct Params {
  const double* tab_d;  // [mat][species][node][kQ]
  const float* tab_f;
  double lnE0, inv_dlnE, dlnE;
  float lnE0_f, inv_dlnE_f, dlnE_f;
  MatParams mat[kMaxMat];
  int n_mats;
  double tcut, alpha, rfinal;
  float tcut_f, alpha_f, rfinal_f;
  uint32_t max_steps;
  int charged_local, cont_loss;
  int gkind, nvol, nbins;
  uint32_t max_events;
  const double* bounds;
  const int* vmat;
  const int* vbin;
  double hx, hy, hz, bz, ftol;
  // quadric-surface cells (gkind == EMS_GEOM_CSG): surface coefficients (10 each),
  // the faces of each cell (surface * 2 + side), and per face code the cells that
  // have it, in increasing order (the candidates entered through that face)
  int n_surf;
  const double* surf;
  const int* face_off;
  const int* faces;
  const int* cand_off;
  const int* cand;
  uint32_t seed;
  // tallies (per event slot) and run counters
  unsigned long long* tally;     // [slot][nbins], fixed point
  unsigned long long* ledger;    // [slot][kLedger]
  int* alive;                    // [slot] tracks alive or queued
  const double* scale;           // [slot] fixed-point scale 2^s
  uint32_t* done;                // [slot] list of finished slots (append)
  unsigned long long* ctr;       // kNumLines x kLineWords iteration counters
  unsigned long long* esc_hist;  // [3][kGrid] escaping tracks of the run
  unsigned long long* ev_esc;    // [slot][3][kGrid] escaping tracks per event, or null
};

// Pending primaries (ring of queue_capacity entries).
struct Queue {
  int32_t* species;
  double *T, *x, *y, *z, *u, *v, *w;
  uint32_t *slot, *index, *event_id;
  uint32_t capacity;
};

}  // namespace ems
