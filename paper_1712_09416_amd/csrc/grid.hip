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
// inside the row (order of arrival; the sort below makes it canonical).
__global__ void k_count(Slot S) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += stride) {
    S.tmap[i] = -1;
    const int sec = S.sector[i];
    const int row = S.row[i];
    const float y = S.y[i], z = S.z[i];
    if (sec >= kSectorsPerEvent || row >= kRows || !isfinite(y) || !isfinite(z)) {
      atomicAdd(&S.err[0], 1u);
      S.rank[i] = kNoHit;
      continue;
    }
    const int e = event_of(S.ev_off, S.n_events, i);
    const int sr = (e * kSectorsPerEvent + sec) * kRows + row;
    S.rank[i] = atomicAdd(&S.row_cnt[sr], 1u);
  }
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_w, uint32_t* total) {
  // 1024 threads, wave64: scan in waves, then over the 16 wave sums
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(x, d, 64);
    if (lane >= d) x += t;
  }
  if (lane == 63) lds_w[w] = x;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int nw = blockDim.x >> 6;
    uint32_t s = threadIdx.x < nw ? lds_w[threadIdx.x] : 0u;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t t = __shfl_up(s, d, 64);
      if ((int)threadIdx.x >= d) s += t;
    }
    if (threadIdx.x < nw) lds_w[32 + threadIdx.x] = s;
  }
  __syncthreads();
  const uint32_t before = w ? lds_w[32 + w - 1] : 0u;
  *total = lds_w[32 + (blockDim.x >> 6) - 1];
  __syncthreads();
  return before + x - v;
}

// Bin layout of one row with n hits: ~bin_target hits per bin, edges at
// least bin_min_edge, at most max(n, 1) bins.
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
  for (int it = 0; it < 32; ++it) {
    ny = (int)ceilf(wy / edge);
    nz = (int)ceilf(wz / edge);
    ny = ny < 1 ? 1 : (ny > 128 ? 128 : ny);
    nz = nz < 1 ? 1 : (nz > 128 ? 128 : nz);
    if ((uint32_t)(ny * nz) <= (n > 0 ? n : 1u)) break;
    edge *= 1.25f;
  }
  if ((uint32_t)(ny * nz) > (n > 0 ? n : 1u)) { ny = 1; nz = 1; }
  b.ny = ny;
  b.nz = nz;
  b.iby = (float)ny / wy;
  b.ibz = (float)nz / wz;
  b.base = 0;
  b.pad = 0;
  return b;
}

// a2 (one block): row offsets, bin layout and bin bases of every row, and the
// per-sector regions for start hits / tracklets (<= n_g/3 + 1: chains of >= 3
// hits are disjoint) and tracks (<= n_g/10 + 1: tracks own >= 10 hits).
__global__ void __launch_bounds__(1024) k_scan_rows(Slot S, DevConst K) {
  __shared__ uint32_t wsum[64];
  __shared__ uint32_t carry_rows, carry_bins;
  const int SR = S.n_sectors * kRows;
  if (threadIdx.x == 0) { carry_rows = 0; carry_bins = 0; }
  __syncthreads();
  for (int base = 0; base < SR; base += blockDim.x) {
    const int sr = base + threadIdx.x;
    const uint32_t cnt = sr < SR ? S.row_cnt[sr] : 0u;
    RowBins b;
    uint32_t nb = 0;
    if (sr < SR) {
      const int g = sr / kRows, row = sr % kRows;
      b = make_bins(K, row, (g % kSectorsPerEvent) >= kSectorsPerEvent / 2, cnt);
      nb = (uint32_t)(b.ny * b.nz);
      if (cnt > (uint32_t)kMaxRowHits) atomicAdd(&S.err[1], 1u);
    }
    uint32_t tot_r, tot_b;
    const uint32_t off_r = block_exclusive_scan(cnt, wsum, &tot_r);
    const uint32_t off_b = block_exclusive_scan(nb, wsum, &tot_b);
    if (sr < SR) {
      S.row_off[sr] = carry_rows + off_r;
      b.base = (int32_t)(carry_bins + off_b);
      S.bins[sr] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry_rows += tot_r;
      carry_bins += tot_b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S.row_off[SR] = carry_rows;
    S.bin_off[carry_bins] = carry_rows;
  }
  __syncthreads();
  // per-sector regions
  __shared__ uint32_t carry_tl, carry_tk;
  if (threadIdx.x == 0) { carry_tl = 0; carry_tk = 0; }
  __syncthreads();
  for (int base = 0; base < S.n_sectors; base += blockDim.x) {
    const int g = base + threadIdx.x;
    uint32_t a = 0, c = 0;
    if (g < S.n_sectors) {
      const uint32_t ng = S.row_off[(g + 1) * kRows] - S.row_off[g * kRows];
      a = ng / 3 + 1;
      c = ng / 10 + 1;
    }
    uint32_t ta, tc;
    const uint32_t oa = block_exclusive_scan(a, wsum, &ta);
    const uint32_t oc = block_exclusive_scan(c, wsum, &tc);
    if (g < S.n_sectors) {
      S.tl_base[g] = carry_tl + oa;
      S.tk_base[g] = carry_tk + oc;
    }
    __syncthreads();
    if (threadIdx.x == 0) { carry_tl += ta; carry_tk += tc; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S.tl_base[S.n_sectors] = carry_tl;
    S.tk_base[S.n_sectors] = carry_tk;
    if ((int64_t)carry_tl > S.cap_tl || (int64_t)carry_tk > S.cap_tk) atomicAdd(&S.err[2], 1u);
  }
}

// a2: clusters to their row (arrival order within the row)
__global__ void k_scatter(Slot S) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += stride) {
    const uint32_t rk = S.rank[i];
    if (rk == kNoHit) continue;
    const int e = event_of(S.ev_off, S.n_events, i);
    const int sr = (e * kSectorsPerEvent + S.sector[i]) * kRows + S.row[i];
    const uint32_t pos = S.row_off[sr] + rk;
    S.ty[pos] = S.y[i];
    S.tz[pos] = S.z[i];
    S.tid[pos] = (uint32_t)i;
  }
}

// a2: one block per (sector, row): sort the row's hits by (bin, cluster
// index) with a bitonic sort of 64-bit keys in LDS, write them in that order
// and fill the row's bin offsets.
// key = bin << 44 | cluster index << 12 | position in the row
__global__ void __launch_bounds__(256) k_row_sort(Slot S) {
  __shared__ unsigned long long key[kMaxRowHits];
  __shared__ float ly[kMaxRowHits];
  __shared__ float lz[kMaxRowHits];
  const int sr = blockIdx.x;
  const uint32_t off = S.row_off[sr];
  const uint32_t n = S.row_off[sr + 1] - off;
  const RowBins b = S.bins[sr];
  const int nb = b.ny * b.nz;
  if (n > (uint32_t)kMaxRowHits) {
    // flagged in k_scan_rows (the slot's result is refused); keep the row
    // harmless for the kernels that still run: no coordinates, empty bins
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
      Hit h;
      h.y = __builtin_nanf("");
      h.z = __builtin_nanf("");
      h.id = S.tid[off + j];
      h.upc = -1;
      S.hit[off + j] = h;
    }
    for (int bb = threadIdx.x; bb <= nb; bb += blockDim.x) S.bin_off[b.base + bb] = off;
    return;
  }
  uint32_t P = 1;
  while (P < n) P <<= 1;
  for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) {
    if (j < n) {
      const float y = S.ty[off + j], z = S.tz[off + j];
      ly[j] = y;
      lz[j] = z;
      const uint32_t bin = (uint32_t)(bin_z(b, z) * b.ny + bin_y(b, y));
      key[j] = ((unsigned long long)bin << 44) | ((unsigned long long)S.tid[off + j] << 12) | j;
    } else {
      key[j] = ~0ull;
    }
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
      for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        const uint32_t l = i ^ jj;
        if (l > i) {
          const unsigned long long a = key[i], c = key[l];
          const bool up = (i & k) == 0;
          if ((a > c) == up) {
            key[i] = c;
            key[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const unsigned long long kk = key[j];
    const uint32_t src = (uint32_t)(kk & 0xFFFull);
    Hit h;
    h.y = ly[src];
    h.z = lz[src];
    h.id = (uint32_t)((kk >> 12) & 0xFFFFFFFFull);
    h.upc = -1;
    S.hit[off + j] = h;
  }
  // bin offsets: first sorted position whose bin is >= each bin
  for (int bb = threadIdx.x; bb <= nb; bb += blockDim.x) {
    uint32_t lo = 0, hi = n;
    const unsigned long long t = (unsigned long long)bb << 44;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (key[mid] < t) lo = mid + 1; else hi = mid;
    }
    S.bin_off[b.base + bb] = off + lo;
  }
}

}  // namespace tpc
