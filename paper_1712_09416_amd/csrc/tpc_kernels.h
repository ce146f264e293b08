// Kernels of the tracker, launched by the C ABI (api.hip).
#pragma once

#include "tpc_device.h"
#include "tpc_merge.h"

namespace tpc {

// launchers of the kernels instantiated for tuning knobs (results never
// depend on the knobs): wb = window hits read per round trip (2, 4, 8),
// rb = hit-list rows read per round trip (4, 8, 16)
void launch_neighbours(int wb, int blocks, hipStream_t st, const Slot& S, const DevConst& K, int g0,
                       int ns);
void launch_tracklets(int wb, int blocks, int threads, hipStream_t st, const Slot& S,
                      const DevConst& K, int g0);
void launch_select(int rb, int blocks, hipStream_t st, const Slot& S, const DevConst& K, int g0);
void launch_track_write(int rb, int blocks, hipStream_t st, const Slot& S, int g0, int ns);
// stage + grid
__global__ void k_count(Slot S);
__global__ void k_row_layout(Slot S, DevConst K);
__global__ void k_row_finish(Slot S, int n_min_chain, int n_min_track);
__global__ void k_scatter(Slot S);
__global__ void k_row_sort_tiny(Slot S);
__global__ void k_row_sort_small(Slot S);
__global__ void k_row_sort_large(Slot S);
// cellular automaton
__global__ void k_clean_rows(Slot S, int g0, int ns, int n_min_chain);
__global__ void k_start_write(Slot S, int g0, int ns, int n_min_chain);
// Kalman filter
__global__ void k_refit(Slot S, DevConst K, int g0, int ns);
// output
__global__ void k_scan_tiles(const uint32_t* in, const uint32_t* n_dev, int64_t n_host,
                             uint32_t* partial);
__global__ void k_scan_partials(uint32_t* partial, int nb, uint32_t* out, const uint32_t* n_dev,
                                int64_t n_host, uint32_t* total_out, int write_end);
__global__ void k_scan_apply(const uint32_t* in, const uint32_t* n_dev, int64_t n_host,
                             const uint32_t* partial, uint32_t* out);
constexpr int kSmallPerThread = 16;
constexpr int64_t kSmallScanMax = 1024 * kSmallPerThread;
__global__ void k_scan_small(uint32_t* data, const uint32_t* n_dev, int64_t n_host,
                             uint32_t* total_out, int write_end);
__global__ void k_flags(Slot S);
__global__ void k_order(Slot S);
__global__ void k_event_hits(Slot S);
__global__ void k_write_out(Slot S, DevConst K);
// cross-sector merger
__global__ void k_mg_count(Slot S, MergeSlot M);
__global__ void k_mg_scatter(Slot S, MergeSlot M);
__global__ void k_mg_outer(Slot S, DevConst K, MergeSlot M, MergeConst C);
template <bool kFinal>
__global__ void k_mg_pairs(Slot S, DevConst K, MergeSlot M, MergeConst C);
__global__ void k_mg_final(Slot S, MergeSlot M);
__global__ void k_mg_pair_best(MergeSlot M);
__global__ void k_mg_link(Slot S, MergeSlot M);
__global__ void k_mg_chain(Slot S, DevConst K, MergeSlot M, MergeConst C);
__global__ void k_mg_emit(Slot S, MergeSlot M);
__global__ void k_mg_event_off(Slot S, MergeSlot M);
__global__ void k_mg_write(Slot S, DevConst K, MergeSlot M);
// drift-velocity calibration
__global__ void k_cal_accumulate(Slot S, DevConst K, uint32_t* hist, int n_bins, double z_lo,
                                 double w);
__global__ void k_cal_fit(const uint32_t* hist, int n_bins, double z_lo, double w, double z_max,
                          double eps_t, double* out);
__global__ void k_cal_correct(const uint8_t* sector, float* z, int64_t n, double eps, double z_max);

}  // namespace tpc
