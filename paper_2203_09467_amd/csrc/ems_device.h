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

#include "ems_slotmap.h"

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
constexpr int kLifeBins = 17;  // steps per track: 0, 1, 2-3, 4-7, ..., >= 32768
constexpr uint32_t kVolOut = 0xFFFFFu;  // meta volume of a primary that starts outside
constexpr uint32_t kVolMask = 0xFFFFFu;  // meta bits 6-25: volume
constexpr int kVcapShift = 26;           // meta bits 26-31: capped vacuum field steps in a row
// meta bit 3 with bit 2 (put-off interaction) clear: a curved move suspended
// between launches (with bit 2 set, bits 3-5 name the interaction's queue)
constexpr uint32_t kMidMove = 8u;
constexpr uint32_t kRestStep = 0xFFFFFFFFu;
constexpr int kMaxTrial = 1000;
constexpr int kBlock = 256;
constexpr uint32_t kStageMaxBytes = 64u * 1024u;  // per-block LDS budget of the staged run data

// Tracks in flight, SoA.  meta = species (bits 0-1) | pending (bit 2) | queue of
// the pending interaction (bits 3-5) | volume (bits 6-25) | field steps in vacuum
// that ended on their substep cap, in a row (bits 26-31); a pending track ended its
// last step in an interaction that was put off for lack of output room.  Photons and
// charged tracks live in separate pools so that a wavefront steps one species
// class, each double-buffered.  A Pool passed to the step kernels is the set of
// all four buffers: for every field, buffer (class c, parity b) occupies elements
// [(2c + b) N, (2c + b + 1) N), so a lane picks its destination buffer with one
// integer offset.  src (diagnostics only) is the input index of a single-step call.
struct Pool {
  double *x, *y, *z, *u, *v, *w, *T, *nlam;
  uint32_t *k0, *k1, *k2, *evt, *nstep, *meta, *src;
  // state of a curved move suspended between launches (read and written only for
  // tracks whose meta word carries kMidMove): substeps done, next trial length,
  // path travelled
  uint32_t* fsub;
  double *fh, *ftrav;
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
  uint4* rec;  // 5 x 16 B per entry: (x, y) (z, u) (v, w) (T, k0 k1) (k2 evt nstep meta)
  uint32_t* src;
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
  kLDone = 5,     // events finished in the interval (low); word 1: check bits of a submitted batch
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
  kSPeak = 10,     // largest pool
  kSEnergy = 11    // kinetic energy (keV) of the tracks written to the output pools this
                   // iteration: cleared at every iteration, so after the interval it is
                   // the pool's (summed over the copies)
};
constexpr int kLineWords = 32;  // 64-bit words per line
// the steps-per-track histogram is kept in kStatCopies copies kLifeStride words apart
// (a block adds to copy blockIdx % kStatCopies): its few bins take an update from
// nearly every block
constexpr int kLifeStride = 64;
// Per-event scores (tally bins, ledger words, alive count) are kept in kEvCopies
// copies; a block adds to copy blockIdx % kEvCopies.  An event's tracks can fill
// most blocks of an iteration (serving: hundreds of primaries per event), and one
// copy per event took every block's atomic on the same few addresses.  Reads sum
// the copies; an event is finished when its copies' alive counts sum to zero,
// checked once per host synchronisation (the host reads completions only then).
constexpr int kEvCopies = 8;

struct MatParams {
  double Tc, kc;      // production thresholds (delta rays, brems photons)
  double Rtrk[3];     // range table at the tracking cut, per species
  double X0;          // radiation length, cm
  float Rtrk_f[3];
  float Tc_f, kc_f, X0_f;
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
  uint32_t sub_per_step;  // curved-move substeps per track-step of a launch before suspension
  int charged_local, cont_loss, msc;
  int gkind, nvol, nbins;
  uint32_t max_events;
  const double* bounds;
  const int* vmat;
  const int* vbin;
  double hx, hy, hz, bz, ftol;
  // quadric-surface cells (gkind == EMS_GEOM_CSG): surface coefficients (10 each),
  // the faces of each cell (surface * 2 + side), and per face code the cells that
  // have it, in increasing order (the candidates entered through that face)
  int n_surf, n_faces;
  const double* surf;
  const unsigned char* plane;  // 1 if surface s has no quadratic term
  const int* face_off;
  const int* faces;
  const int* cand_off;
  const int* cand;
  uint32_t seed;
  // tallies (per event slot) and run counters
  unsigned long long* tally;     // [slot][kEvCopies][nbins], fixed point
  unsigned long long* ledger;    // [slot][kEvCopies][kLedger]
  int* alive;                    // [slot] tracks alive or queued
  const double* scale;           // [slot] fixed-point scale 2^s
  uint32_t* slot_state;          // [slot] 0 free, 1 in flight, 2 finished, 3 being read
  unsigned long long* ctr;       // kNumLines x kLineWords iteration counters
  unsigned long long* esc_hist;  // [3][kGrid] escaping tracks of the run
  unsigned long long* ev_esc;    // [slot][3][kGrid] escaping tracks per event, or null
  unsigned long long* life_hist; // [kStatCopies][kLifeStride]: [3][kLifeBins] tracks ended,
                                 // by species and steps taken
};

// Event slots and ids, kept on the device so that submitting and reading a batch
// costs the host nothing per event.  bits: one bit per slot, set while the slot is
// free (the host mirrors their count); before a batch takes slots, pre[w] = free
// slots in words [0, w) and the batch takes the lowest free slots in order, so that
// events submitted together get neighbouring slots in submission order; map:
// open-addressing id -> slot table (power-of-two size, linear probing) of entries
// (slot + 1) << 32 | id, 0 = empty, kMapTomb = erased; id: the id of each slot;
// claim: during a read, the first position in the call naming the slot.
struct EvSlots {
  uint32_t* bits;
  uint32_t* pre;      // words + 1 entries
  uint32_t* tile;     // per tile of kFreeTile words: its free count, then its offset
  uint32_t words;     // ceil(n / 32)
  unsigned long long* map;
  uint32_t mask;
  uint32_t* state;
  uint32_t* id;
  uint32_t* claim;
  uint32_t n;         // slots
};
// bits of the batch check word set by the submission kernels
enum BatchFlag : unsigned long long {
  kBadSpecies = 1, kBadEnergy = 2, kBadPos = 4, kBadDir = 8,
  kBadEmpty = 16,     // an event without primaries
  kBadLarge = 32,     // an event with more primaries than a quarter of the pool
  kBadDup = 64,       // an id already unread, or twice in the batch
  kBadMap = 128       // the id table is full (cannot happen while it is rebuilt in time)
};

// Pending primaries (ring of queue_capacity entries).
struct Queue {
  int32_t* species;
  double *T, *x, *y, *z, *u, *v, *w;
  uint32_t *slot, *index, *event_id;
  uint32_t capacity;
};

}  // namespace ems
