// ems_host.h -- internal declarations shared by the host-side sources of the library.
#pragma once

#include <string>
#include <vector>

#include "emshower.h"
#include "ems_device.h"

namespace ems {

// Record `msg` as the thread's last error and return s.
ems_status fail_status(ems_status s, const std::string& msg);

ems_status create_context(const ems_config* cfg, void* d_workspace, size_t bytes, bool pinned,
                          const char* who, ems_ctx** out);

int build_physics_tables(const ems_material* mats, int n_mats, const ems_physics_options& o,
                         std::vector<double>& tab, MatParams* mp);

hipError_t launch_iteration(const Params& P, const Pool& S, uint32_t N, int cur, const IQueue& Q,
                            uint32_t bound, uint32_t msteps, bool mixed, ems_step_record* rec,
                            hipStream_t s);
hipError_t launch_iter_begin(unsigned long long* ctr, bool explicit_counts, uint32_t nG,
                             uint32_t nC, uint32_t j_iter, uint32_t* log, hipStream_t s);
hipError_t launch_admit(const Params& P, const Queue& q, const Pool& S, uint32_t N, int cur,
                        uint32_t head, uint32_t m, hipStream_t s);
hipError_t launch_enqueue(const Queue& q, uint32_t tail, const int64_t* off, const uint32_t* slots,
                          const uint32_t* ids, uint32_t n_events, const int32_t* sp,
                          const double* T, const double* pos, const double* dir, uint32_t n,
                          unsigned long long* bad, hipStream_t s);
hipError_t launch_event_init(const Params& P, const int64_t* off, const uint32_t* slots,
                             const double* T, const int32_t* sp, uint32_t n_events, int64_t n,
                             double* e_in, double* scale, double* e_row, int64_t quarter,
                             unsigned long long* bad, hipStream_t s);
hipError_t launch_slots_take(const EvSlots& M, const uint32_t* ids, uint32_t n, uint32_t* slots,
                             uint32_t* flag, unsigned long long* bad, hipStream_t s);
hipError_t launch_slots_undo(const EvSlots& M, const uint32_t* ids, const uint32_t* slots,
                             const uint32_t* flag, uint32_t n, hipStream_t s);
hipError_t launch_events_reset(const EvSlots& M, hipStream_t s);
hipError_t launch_map_rebuild(const EvSlots& M, hipStream_t s);
hipError_t launch_read_find(const EvSlots& M, const uint32_t* ids, uint32_t n, uint32_t* slots,
                            int32_t* status, hipStream_t s);
hipError_t launch_read_unclaim(const EvSlots& M, const uint32_t* slots, uint32_t n, hipStream_t s);
hipError_t launch_read_release(const EvSlots& M, const uint32_t* ids, const uint32_t* slots,
                               uint32_t n, hipStream_t s);
hipError_t launch_slots_reset(const Params& P, hipStream_t s);
hipError_t launch_done_scan(const Params& P, hipStream_t s);
hipError_t launch_spill_hist(const Params& P, const Pool& S, uint32_t N, int cur, uint32_t nG,
                             uint32_t nC, unsigned long long* hist, hipStream_t s);
hipError_t launch_spill_split(const Params& P, const Pool& S, uint32_t N, int cur, uint32_t nG,
                              uint32_t nC, int bmin, uint32_t* cnt, hipStream_t s);
hipError_t launch_unspill(const Params& P, const Pool& S, uint32_t N, int cur, uint32_t m,
                          hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, uint32_t n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t s);
hipError_t launch_pool_load(const Params& P, const Pool& S, uint32_t N, const ems_track_soa& src,
                            uint32_t n, hipStream_t s);
hipError_t launch_pool_dump(const Pool& p, const ems_track_soa& dst, uint32_t n, uint32_t off,
                            hipStream_t s);
hipError_t launch_gather_tallies(const Params& P, const uint32_t* slots, uint32_t n,
                                 const double* e_in, double* dep, double* ledger,
                                 unsigned long long* steps, unsigned long long* esc, hipStream_t s);

}  // namespace ems
