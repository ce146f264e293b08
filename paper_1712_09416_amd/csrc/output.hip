// Output: tracks in canonical order (event, cluster ID of the innermost hit)
// with their hit lists (cluster IDs of the event, ascending pad row).
// The order is obtained without a sort: the refit marks each track's
// innermost cluster; an exclusive scan over the clusters of the slot gives
// every track its position.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

constexpr int kScanPerThread = 4;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanBlock * kScanPerThread;

__device__ __forceinline__ uint32_t scan_n(const uint32_t* n_dev, int64_t n_host) {
  return n_dev ? *n_dev : (uint32_t)n_host;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(x, d, 64);
    if (lane >= d) x += t;
  }
  return x;
}

// exclusive scan of one 256-thread block's values; returns the block total
__device__ __forceinline__ uint32_t block_scan256(uint32_t v, uint32_t* excl) {
  __shared__ uint32_t ws[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < w) before += ws[i];
    tot += ws[i];
  }
  __syncthreads();
  *excl = before + inc - v;
  return tot;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(const uint32_t* in, const uint32_t* n_dev,
                                                           int64_t n_host, uint32_t* partial) {
  const uint32_t n = scan_n(n_dev, n_host);
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPerThread;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPerThread; ++j)
    if (base + j < n) s += in[base + j];
  uint32_t ex;
  const uint32_t tot = block_scan256(s, &ex);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_partials(uint32_t* partial, int nb, uint32_t* out,
                                                        const uint32_t* n_dev, int64_t n_host,
                                                        uint32_t* total_out, int write_end) {
  __shared__ uint32_t w[32];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? partial[i] : 0u;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) w[wv] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int j = 0; j < (int)(blockDim.x >> 6); ++j) {
      if (j < wv) before += w[j];
      tot += w[j];
    }
    if (i < nb) partial[i] = carry + before + inc - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t n = scan_n(n_dev, n_host);
    if (write_end) out[n] = carry;
    if (total_out) *total_out = carry;
  }
}

// Whole scan in one 1024-thread block for n <= kSmallScanMax (the per-row
// and per-sector tables): each thread scans a contiguous run of
// kSmallPerThread values in registers.  In place; writes the total to
// data[n] (write_end) and *total_out (if given).
__global__ void __launch_bounds__(1024) k_scan_small(uint32_t* data, const uint32_t* n_dev,
                                                     int64_t n_host, uint32_t* total_out,
                                                     int write_end) {
  __shared__ uint32_t ws[16];
  const uint32_t n = scan_n(n_dev, n_host);
  const uint32_t base = threadIdx.x * kSmallPerThread;
  uint32_t v[kSmallPerThread];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kSmallPerThread; ++j) {
    v[j] = base + j < n ? data[base + j] : 0u;
    s += v[j];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(s);
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i < w) before += ws[i];
    tot += ws[i];
  }
  uint32_t run = before + inc - s;
#pragma unroll
  for (int j = 0; j < kSmallPerThread; ++j) {
    if (base + j < n) data[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) {
    if (write_end) data[n] = tot;
    if (total_out) *total_out = tot;
  }
}

// in-place capable: each thread reads its values before writing them
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const uint32_t* in, const uint32_t* n_dev,
                                                           int64_t n_host, const uint32_t* partial,
                                                           uint32_t* out) {
  const uint32_t n = scan_n(n_dev, n_host);
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPerThread;
  uint32_t v[kScanPerThread];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPerThread; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0u;
    s += v[j];
  }
  uint32_t ex;
  block_scan256(s, &ex);
  uint32_t run = partial[blockIdx.x] + ex;
#pragma unroll
  for (int j = 0; j < kScanPerThread; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
}

__global__ void k_flags(Slot S) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += stride)
    S.scan_a[i] = S.tmap[i] >= 0 ? 1u : 0u;
}

// Canonical position of every track, its hit count, per-event track ranges.
__global__ void k_order(Slot S) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < S.n; i += stride) {
    const int32_t k = S.tmap[i];
    if (k < 0) continue;
    const uint32_t pos = S.scan_a[i];
    S.out_order[pos] = k;
    S.out_ntk[pos] = (uint32_t)S.tk_info[(size_t)k * 4 + 1];
  }
  if (t0 <= S.n_events) S.ev_track_off[t0] = S.scan_a[S.ev_off[t0]];
  if (t0 == 0) S.out_count[0] = S.scan_a[S.n];
}

// Per-event hit ranges (after the scan of the hit counts).
__global__ void k_event_hits(Slot S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e <= S.n_events) S.ev_hit_off[e] = S.out_ntk[S.ev_track_off[e]];
}

// Track records and hit lists (hit offsets relative to the event).  A group
// of kOutLanes lanes per track: its first lane writes the record, the group
// copies the hit IDs (lane u of the group takes every kOutLanes-th hit, up
// to kOutBatch of them per memory round trip).
constexpr int kOutLanes = 8;
constexpr int kOutBatch = 8;

__global__ void k_write_out(Slot S, DevConst K) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t ngroups = gridDim.x * blockDim.x / kOutLanes;
  const uint32_t gid = (blockIdx.x * blockDim.x + threadIdx.x) / kOutLanes;
  const int sub = (int)(threadIdx.x % kOutLanes);
  for (uint32_t pos = gid; pos < ntk; pos += ngroups) {
    const int32_t k = S.out_order[pos];
    const int32_t* ti = S.tk_info + (size_t)k * 4;
    const int nown = S.tk_nown[k];
    const int32_t* own = S.tk_own + (size_t)k * kRows;
    const int nh = ti[1];
    const int j0 = nown - nh;             // the fitted hits are the last n_hits owned ones
    const uint32_t gidx = S.hit[own[j0]].id;
    int e = 0;
    {
      int lo = 0, hi = S.n_events - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.ev_off[mid] <= (int64_t)gidx) lo = mid; else hi = mid - 1;
      }
      e = lo;
    }
    const int64_t ev0 = S.ev_off[e];
    const uint32_t hoff = S.out_ntk[pos];
    if (sub == 0) {
      const int32_t T = S.tk_tracklet[k];
      const uint32_t ehoff = S.ev_hit_off[e];
      tpc_track o;
      o.sector = (int32_t)S.sector[gidx];
      o.n_hits = nh;
      o.row_in = ti[2];
      o.row_out = ti[3];
      o.hit_off = (int64_t)(hoff - ehoff);
      o.inner_id = (int32_t)((int64_t)gidx - ev0);
      o.start_id = (int32_t)((int64_t)S.hit[S.start_hit[T]].id - ev0);
      o.x_ref = (double)K.row_x[ti[2]];
      o.ndf = 2 * nh - 5;
      o.event = e;
      const double* par = S.tk_par + (size_t)k * 5;
      const double* cov = S.tk_cov + (size_t)k * 15;
      for (int i = 0; i < 5; ++i) o.par[i] = par[i];
      for (int i = 0; i < 15; ++i) o.cov[i] = cov[i];
      o.chi2 = S.tk_chi2[k];
      S.out_tracks[pos] = o;
    }
    int32_t* dst = S.out_hits + hoff;
    for (int ib = sub; ib < nh; ib += kOutLanes * kOutBatch) {
      int32_t pv[kOutBatch];
#pragma unroll
      for (int u = 0; u < kOutBatch; ++u) {
        const int i = ib + u * kOutLanes;
        pv[u] = i < nh ? own[j0 + i] : -1;
      }
      uint32_t iv[kOutBatch];
#pragma unroll
      for (int u = 0; u < kOutBatch; ++u) iv[u] = pv[u] >= 0 ? S.hit[pv[u]].id : 0u;
#pragma unroll
      for (int u = 0; u < kOutBatch; ++u) {
        const int i = ib + u * kOutLanes;
        if (i < nh) dst[i] = (int32_t)((int64_t)iv[u] - ev0);
      }
    }
  }
}

}  // namespace tpc
