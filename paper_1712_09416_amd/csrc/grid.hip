// Stage and grid: clusters -> per (sector, pad row) hit lists ordered by
// (bin, cluster ID), with a 2-D y x z bin index per row.
//
// This is the input step of the CA tracker: the neighbours finder and the
// Kalman search query "all hits of row r inside a window", and the bins make
// those queries touch a handful of hits.  Results never depend on the bin
// layout: queries scan every bin that can hold a hit of the window and then
// apply the exact window test on each hit.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

// Event of cluster i (binary search over the slot's event offsets).
__device__ __forceinline__ int event_of(const int64_t* ev_off, int n_events, int64_t i) {
  int lo = 0, hi = n_events - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ev_off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// a1: validate, count clusters per (sector, row) and give each its rank
// inside the row (arrival order; the row sort below makes it canonical).
// One block per chunk of kCountChunk clusters of one event (blockIdx.y):
// ranks are taken in an LDS histogram of the event's rows, then one global
// atomic per row and block reserves the block's range.
constexpr int kCountChunk = 4096;
constexpr int kEventRows = kSectorsPerEvent * kRows;
constexpr int kCountThreads = 256;
constexpr int kRowsPerThread = (kEventRows + kCountThreads - 1) / kCountThreads;
constexpr int kCountBatch = 4;

__global__ void __launch_bounds__(kCountThreads) k_count(Slot S) {
  __shared__ uint32_t hist[kEventRows];
  const int e = blockIdx.y;
  const int64_t e0 = S.ev_off[e], e1 = S.ev_off[e + 1];
  const int64_t i0 = e0 + (int64_t)blockIdx.x * kCountChunk;
  if (i0 >= e1) return;
  const int64_t i1 = min(e1, i0 + (int64_t)kCountChunk);
  for (int r = threadIdx.x; r < kEventRows; r += blockDim.x) hist[r] = 0u;
  __syncthreads();
  // clusters kCountBatch per thread at a time: loads first, then the LDS
  // ranks
  for (int64_t ib = i0 + threadIdx.x; ib < i1; ib += kCountBatch * kCountThreads) {
    int sec[kCountBatch], row[kCountBatch];
    float y[kCountBatch], z[kCountBatch];
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      const int64_t i = ib + u * kCountThreads;
      sec[u] = 0;
      row[u] = 0;
      y[u] = 0.0f;
      z[u] = 0.0f;
      if (i < i1) {
        sec[u] = S.sector[i];
        row[u] = S.row[i];
        y[u] = S.y[i];
        z[u] = S.z[i];
      }
    }
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      const int64_t i = ib + u * kCountThreads;
      if (i >= i1) continue;
      S.tmap[i] = -1;
      if (sec[u] >= kSectorsPerEvent || row[u] >= kRows || !isfinite(y[u]) || !isfinite(z[u])) {
        atomicAdd(&S.err[0], 1u);
        S.rank[i] = kNoHit;
        continue;
      }
      S.rank[i] = atomicAdd(&hist[sec[u] * kRows + row[u]], 1u);
    }
  }
  __syncthreads();
  // every atomic of the thread is issued before the first result is used
  uint32_t* cnt = S.row_cnt + (size_t)e * kEventRows;
  uint32_t res[kRowsPerThread];
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const int r = threadIdx.x + k * kCountThreads;
    const uint32_t c = r < kEventRows ? hist[r] : 0u;
    res[k] = c ? atomicAdd(&cnt[r], c) : 0u;
  }
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const int r = threadIdx.x + k * kCountThreads;
    if (r < kEventRows) hist[r] = res[k];
  }
  __syncthreads();
  for (int64_t ib = i0 + threadIdx.x; ib < i1; ib += kCountBatch * kCountThreads) {
    uint32_t rk[kCountBatch];
    int sr[kCountBatch];
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      const int64_t i = ib + u * kCountThreads;
      rk[u] = kNoHit;
      sr[u] = 0;
      if (i < i1) {
        rk[u] = S.rank[i];
        sr[u] = S.sector[i] * kRows + S.row[i];
      }
    }
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      const int64_t i = ib + u * kCountThreads;
      if (i < i1 && rk[u] != kNoHit) S.rank[i] = rk[u] + hist[sr[u]];
    }
  }
}

// Bin layout of one row with n hits: ~bin_target hits per bin, edges at
// least bin_min_edge, at most kBinsPerHit * max(n, 1) bins.
__device__ RowBins make_bins(const DevConst& K, int row, bool side_c, uint32_t n) {
  RowBins b;
  const float ymax = K.row_x[row] * K.tanh_half + K.medge;
  const float wy = 2.0f * ymax;
  const float wz = K.z_max + 2.0f * K.mz;
  b.y0 = -ymax;
  b.z0 = side_c ? -(K.z_max + K.mz) : -K.mz;
  const float nn = n > 0 ? (float)n : 1.0f;
  float edge = sqrtf(wy * wz * K.bin_target / nn);
  if (edge < K.bin_min_edge) edge = K.bin_min_edge;
  int ny = 1, nz = 1;
  const uint32_t nmax = (uint32_t)kBinsPerHit * (n > 0 ? n : 1u);
  for (int it = 0; it < 32; ++it) {
    ny = (int)ceilf(wy / edge);
    nz = (int)ceilf(wz / edge);
    ny = ny < 1 ? 1 : (ny > 128 ? 128 : ny);
    nz = nz < 1 ? 1 : (nz > 128 ? 128 : nz);
    if ((uint32_t)(ny * nz) <= nmax) break;
    edge *= 1.25f;
  }
  if ((uint32_t)(ny * nz) > nmax) { ny = 1; nz = 1; }
  b.ny = ny;
  b.nz = nz;
  b.iby = (float)ny / wy;
  b.ibz = (float)nz / wz;
  b.base = 0;
  b.first = 0;
  return b;
}

// a2: per row, the bin layout (from the row's count) and the two counts
// the scans turn into offsets: clusters -> row_off, bins -> row_bin.
__global__ void k_row_layout(Slot S, DevConst K) {
  const int SR = S.n_sectors * kRows;
  const int stride = gridDim.x * blockDim.x;
  for (int sr = blockIdx.x * blockDim.x + threadIdx.x; sr < SR; sr += stride) {
    const uint32_t cnt = S.row_cnt[sr];
    const int g = sr / kRows, row = sr - (sr / kRows) * kRows;
    const RowBins b = make_bins(K, row, (g % kSectorsPerEvent) >= kSectorsPerEvent / 2, cnt);
    if (cnt > (uint32_t)kMaxRowHits) atomicAdd(&S.err[1], 1u);
    S.bins[sr] = b;
    S.row_off[sr] = cnt;
    S.row_bin[sr] = (uint32_t)(b.ny * b.nz);
  }
}

// a2 (after the scans): bin bases of the rows, and the per-sector regions
// for start hits / tracklets (<= n_g/n_min_chain + 1: each heads its own
// cleaned chain of >= n_min_chain hits, and the chains are disjoint) and tracks (<= n_g/n_min_track + 1: each track owns at least
// n_min_track hits no other track owns), as counts for the next scans.
__global__ void k_row_finish(Slot S, int n_min_chain, int n_min_track) {
  const int SR = S.n_sectors * kRows;
  const int stride = gridDim.x * blockDim.x;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) S.range_cnt[2] = 0;   // rows over 1024 hits, listed by the row sort
  for (int sr = t0; sr < SR; sr += stride) {
    S.bins[sr].base = (int32_t)S.row_bin[sr];
    S.bins[sr].first = (int32_t)S.row_off[sr];
  }
  for (int g = t0; g < S.n_sectors; g += stride) {
    const uint32_t ng = S.row_off[(g + 1) * kRows] - S.row_off[g * kRows];
    S.tl_base[g] = ng / (uint32_t)n_min_chain + 1;
    S.tk_base[g] = ng / (uint32_t)n_min_track + 1;
  }
}

// a2: clusters to their row (arrival order within the row), as hit
// records; the row sort then orders each row in place
// Clusters kCountBatch per thread at a time (strided by the grid, so each
// load stays coalesced): the batch's fields, then its row offsets, are
// loaded together.
__global__ void k_scatter(Slot S) {
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t ib = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ib < S.n;
       ib += kCountBatch * nthreads) {
    uint32_t rk[kCountBatch];
    int sr[kCountBatch];
    float y[kCountBatch], z[kCountBatch];
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      const int64_t i = ib + u * nthreads;
      rk[u] = kNoHit;
      sr[u] = 0;
      y[u] = 0.0f;
      z[u] = 0.0f;
      if (i < S.n) {
        rk[u] = S.rank[i];
        sr[u] = S.sector[i] * kRows + S.row[i];
        y[u] = S.y[i];
        z[u] = S.z[i];
      }
    }
    uint32_t base[kCountBatch];
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      base[u] = 0u;
      if (rk[u] != kNoHit) {
        const int e = event_of(S.ev_off, S.n_events, ib + u * nthreads);
        base[u] = S.row_off[e * kEventRows + sr[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
      if (rk[u] == kNoHit) continue;
      Hit h;                               // one 16-byte store per cluster
      h.y = y[u];
      h.z = z[u];
      h.id = (uint32_t)(ib + u * nthreads);
      h.upc = -1;
      S.hit[base[u] + rk[u]] = h;
    }
  }
}

// a2: one block per (sector, row): order the row's hits by (bin, cluster
// index) — counting sort by bin in LDS, then an insertion sort by index
// inside each bin (bins hold a hit or two) — write them as Hit records with
// their (sector, row) beside them, and fill the row's bin offsets.  CAP is the largest row the instance handles; the
// instance for rows up to kMaxRowHits also handles the over-full rows.
template <int CAP>
__device__ __forceinline__ void row_sort(Slot& S, int sr, uint32_t skip_upto, bool small) {
  __shared__ float ly[CAP];
  __shared__ float lz[CAP];
  __shared__ uint32_t lid[CAP];
  __shared__ uint16_t lbin[CAP];
  __shared__ uint16_t lrank[CAP];
  __shared__ uint16_t perm[CAP];
  __shared__ uint32_t hist[kBinsPerHit * CAP + 1];
  __shared__ uint32_t wsum[4];
  const uint32_t off = S.row_off[sr];
  const uint32_t n = S.row_off[sr + 1] - off;
  if (n <= skip_upto && skip_upto > 0) return;   // a smaller instance's row
  if (small && n > (uint32_t)CAP) {          // left to the large instance
    if (threadIdx.x == 0) S.big_rows[atomicAdd(&S.range_cnt[2], 1u)] = sr;
    return;
  }
  const RowBins b = S.bins[sr];
  const int nb = b.ny * b.nz;
  if (n > (uint32_t)kMaxRowHits) {
    // flagged in k_row_layout (the slot's result is refused); keep the row
    // harmless for the kernels that still run: no coordinates, empty bins
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
      Hit h;
      h.y = __builtin_nanf("");
      h.z = __builtin_nanf("");
      h.id = S.hit[off + j].id;
      h.upc = -1;
      S.hit[off + j] = h;
      S.hit_sr[off + j] = (uint32_t)sr;
    }
    for (int bb = threadIdx.x; bb <= nb; bb += blockDim.x) S.bin_off[b.base + bb] = off;
    return;
  }
  for (int bb = threadIdx.x; bb <= nb; bb += blockDim.x) hist[bb] = 0u;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const Hit hr = S.hit[off + j];
    const float y = hr.y, z = hr.z;
    ly[j] = y;
    lz[j] = z;
    lid[j] = hr.id;
    const uint32_t bin = (uint32_t)(bin_z(b, z) * b.ny + bin_y(b, y));
    lbin[j] = (uint16_t)bin;
    lrank[j] = (uint16_t)atomicAdd(&hist[bin], 1u);
  }
  __syncthreads();
  // exclusive scan of hist[0, nb) (each thread a contiguous stretch)
  {
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    const int a = threadIdx.x * per, z = min(nb, a + per);
    uint32_t sum = 0;
    for (int k = a; k < z; ++k) sum += hist[k];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = sum;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t t = __shfl_up(inc, d, 64);
      if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int i = 0; i < w; ++i) run += wsum[i];
    for (int k = a; k < z; ++k) {
      const uint32_t c = hist[k];
      hist[k] = run;
      run += c;
    }
    if (threadIdx.x == 0) hist[nb] = n;
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) perm[hist[lbin[j]] + lrank[j]] = (uint16_t)j;
  __syncthreads();
  for (int bb = threadIdx.x; bb < nb; bb += blockDim.x) {
    const uint32_t p0 = hist[bb], p1 = hist[bb + 1];
    for (uint32_t i = p0 + 1; i < p1; ++i) {
      const uint16_t v = perm[i];
      const uint32_t key = lid[v];
      uint32_t k = i;
      while (k > p0 && lid[perm[k - 1]] > key) {
        perm[k] = perm[k - 1];
        --k;
      }
      perm[k] = v;
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint16_t src = perm[j];
    Hit h;
    h.y = ly[src];
    h.z = lz[src];
    h.id = lid[src];
    h.upc = -1;
    S.hit[off + j] = h;
    S.hit_sr[off + j] = (uint32_t)sr;
  }
  for (int bb = threadIdx.x; bb <= nb; bb += blockDim.x) S.bin_off[b.base + bb] = off + hist[bb];
}

// rows of at most kTinyRow hits (most rows of a batch of small events):
// one wave per row, so many rows share a CU
constexpr int kTinyRow = 256;
__global__ void __launch_bounds__(64) k_row_sort_tiny(Slot S) {
  const int sr = blockIdx.x;
  if (S.row_off[sr + 1] - S.row_off[sr] > (uint32_t)kTinyRow) return;
  row_sort<kTinyRow>(S, sr, 0, false);
}
// rows of kTinyRow+1 .. 1024 hits; larger ones are listed for the large instance
__global__ void __launch_bounds__(256) k_row_sort_small(Slot S) {
  row_sort<1024>(S, blockIdx.x, kTinyRow, true);
}
// the listed rows (1025..4096 hits, and the over-full ones)
__global__ void __launch_bounds__(256) k_row_sort_large(Slot S) {
  const uint32_t nbig = S.range_cnt[2];
  for (uint32_t i = blockIdx.x; i < nbig; i += gridDim.x) {
    row_sort<kMaxRowHits>(S, (int)S.big_rows[i], 0, false);
    __syncthreads();
  }
}

}  // namespace tpc
