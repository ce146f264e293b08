// Cellular-automaton part of the tracker (paper, Abstract: track finding by
// a cellular automaton): per-hit best neighbour pair, mutual-link cleaning
// and start hits of the resulting chains.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

constexpr int kNfThreads = 256;

__device__ __forceinline__ float nf_metric(float yd, float zd, float yu, float zu, float yh, float zh,
                                           float f, float wy, float wz) {
  const float dy = yd + (yu - yd) * f - yh;
  const float dz = zd + (zu - zd) * f - zh;
  return dy * dy * wy + dz * dz * wz;
}

// Running argmin of the pair metric: smaller m, ties to the smaller
// (id_d, id_u).
struct PairBest {
  bool have = false;
  float m = 0.0f;
  uint32_t id_d = 0, id_u = 0;
  int32_t d = -1, u = -1;
  __device__ __forceinline__ void offer(float mm, uint32_t idd, uint32_t idu, int32_t pd, int32_t pu) {
    const bool better = !have || mm < m || (mm == m && (idd < id_d || (idd == id_d && idu < id_u)));
    if (better) {
      have = true;
      m = mm;
      id_d = idd;
      id_u = idu;
      d = pd;
      u = pu;
    }
  }
};

constexpr int kNfCand = 32;      // up-row candidates listed per hit before a nested scan

// a3: for each hit h of row r (1..157), the
// pair (d in row r-1, u in row r+1) inside the origin-pointing windows
// |y - y_h x_r'/x_r| <= W, |z - z_h x_r'/x_r| <= W whose straight line passes
// closest to h, measured by m = dy^2 / (1.5 sy^2) + dz^2 / (1.5 sz^2);
// ties go to the smaller (id_d, id_u); the pair is kept if m <= m_max.
// Rows 0 and 158 get no links.
// One lane per hit.  The up-row candidates are listed once in LDS
// (thread-minor, so a wave's accesses fall in distinct banks) and paired
// with every down-row candidate as it is read; a hit with more than kNfCand
// up candidates scans the up window again per down candidate.  Both rows
// are read through the caches with the batched window reads (measured
// faster than staging the rows in LDS, and than holding the candidates in
// registers, whose fixed-length pairing loop costs more than it saves).
// This function: sorted hit h, `my` the thread's candidate slots in LDS;
// WB hit records are read per memory round trip (a tuning knob).
template <int WB>
__device__ __forceinline__ void nf_hit(const Slot& S, const DevConst& K, uint32_t h, uint32_t* my) {
  const int sr = (int)S.hit_sr[h];
  const int g = sr / kRows;
  const int row = sr - g * kRows;
  if (row == 0 || row == kRows - 1) {
    S.up[h] = -1;
    S.dn[h] = -1;
    return;
  }
  const RowBins Bd = S.bins[sr - 1], Bu = S.bins[sr + 1];
  const Hit x = S.hit[h];
  const uint32_t* bod = S.bin_off + Bd.base;
  const uint32_t* bou = S.bin_off + Bu.base;
  const float xr = K.row_x[row];
  const float rho_d = K.row_x[row - 1] / xr;
  const float rho_u = K.row_x[row + 1] / xr;
  const float f = (xr - K.row_x[row - 1]) / (K.row_x[row + 1] - K.row_x[row - 1]);
  const float W = K.nf_w;
  const float yh = x.y, zh = x.z;
  const float ypu = yh * rho_u, zpu = zh * rho_u;
  const float ypd = yh * rho_d, zpd = zh * rho_d;
  int nu = 0;
  for_window_hits<WB>(Bu, bou, S.hit, ypu, zpu, W, W, [&](uint32_t u, const Hit& c) {
    if (!(fabsf(c.y - ypu) <= W && fabsf(c.z - zpu) <= W)) return;
    if (nu < kNfCand) my[nu * kNfThreads] = u;
    ++nu;
  });
  PairBest best;
  if (nu > 0) {
    const float sy = sigma_y(K, zh), sz = sigma_z(K, zh);
    const float wy = 1.0f / (1.5f * (sy * sy));
    const float wz = 1.0f / (1.5f * (sz * sz));
    for_window_hits<WB>(Bd, bod, S.hit, ypd, zpd, W, W, [&](uint32_t d, const Hit& xd) {
      if (!(fabsf(xd.y - ypd) <= W && fabsf(xd.z - zpd) <= W)) return;
      if (nu <= kNfCand) {
        // the listed up hits, WB records per memory round trip
        for (int k0 = 0; k0 < nu; k0 += WB) {
          uint32_t uu[WB];
          Hit xu[WB];
#pragma unroll
          for (int v = 0; v < WB; ++v)
            if (k0 + v < nu) {
              uu[v] = my[(k0 + v) * kNfThreads];
              xu[v] = S.hit[uu[v]];
            }
#pragma unroll
          for (int v = 0; v < WB; ++v)
            if (k0 + v < nu)
              best.offer(nf_metric(xd.y, xd.z, xu[v].y, xu[v].z, yh, zh, f, wy, wz), xd.id,
                         xu[v].id, (int32_t)d, (int32_t)uu[v]);
        }
      } else {
        for_window_hits<WB>(Bu, bou, S.hit, ypu, zpu, W, W, [&](uint32_t u, const Hit& c) {
          if (!(fabsf(c.y - ypu) <= W && fabsf(c.z - zpu) <= W)) return;
          best.offer(nf_metric(xd.y, xd.z, c.y, c.z, yh, zh, f, wy, wz), xd.id, c.id,
                     (int32_t)d, (int32_t)u);
        });
      }
    });
  }
  const bool ok = best.have && best.m <= K.nf_mmax;
  S.up[h] = ok ? best.u : -1;
  S.dn[h] = ok ? best.d : -1;
}

// The hits of sectors [g0, g0 + ns) as one flat sequence (lane per hit, so
// every wave is full whatever the rows' sizes): blocks are dealt
// round-robin over the 8 XCDs, and the blocks of XCD x stride over the x-th
// contiguous eighth of the hits, so the rows r-1, r+1 its lanes read stay
// in its L2.
template <int WB>
__global__ void __launch_bounds__(kNfThreads) k_neighbours(Slot S, DevConst K, int g0, int ns) {
  __shared__ uint32_t cand[kNfCand * kNfThreads];
  const uint32_t h_begin = S.row_off[g0 * kRows];
  const uint32_t h_end = S.row_off[(g0 + ns) * kRows];
  const uint32_t x = blockIdx.x % 8u, nbx = gridDim.x / 8u;
  const uint32_t per = (h_end - h_begin + 7u) / 8u;
  const uint32_t c0 = h_begin + x * per;
  const uint32_t c1 = min(h_end, c0 + per);
  for (uint32_t h = c0 + (blockIdx.x / 8u) * kNfThreads + threadIdx.x; h < c1; h += nbx * kNfThreads)
    nf_hit<WB>(S, K, h, cand + threadIdx.x);
}

void launch_neighbours(int wb, int blocks, hipStream_t st, const Slot& S, const DevConst& K, int g0,
                       int ns) {
  switch (wb) {
    case 2: k_neighbours<2><<<blocks, kNfThreads, 0, st>>>(S, K, g0, ns); break;
    case 8: k_neighbours<8><<<blocks, kNfThreads, 0, st>>>(S, K, g0, ns); break;
    default: k_neighbours<4><<<blocks, kNfThreads, 0, st>>>(S, K, g0, ns); break;
  }
}

// Head of a cleaned chain of >= n_min_chain hits (no cleaned down link; the
// cleaned up links from h reach n_min_chain hits in all), from the links of
// a3 only: a link is cleaned when it is mutual.
__device__ __forceinline__ bool is_start(const Slot& S, uint32_t h, int n_min_chain, int32_t& uc,
                                         int32_t& dc) {
  const int32_t u = S.up[h], d = S.dn[h];
  uc = (u >= 0 && S.dn[u] == (int32_t)h) ? u : -1;
  dc = (d >= 0 && S.up[d] == (int32_t)h) ? d : -1;
  if (uc < 0 || dc >= 0) return false;
  int n = 2;
  for (int32_t k = uc; n < n_min_chain; ++n) {
    const int32_t kk = S.up[k];
    if (kk < 0 || S.dn[kk] != k) break;
    k = kk;
  }
  return n >= n_min_chain;
}

// a4: keep a link only if it is mutual; count the start hits of each row.
// Also clears the hit weights used by the tracklet selection.  One wave per
// row (rows hold ~100 hits), 64 hits at a time.
__global__ void __launch_bounds__(256) k_clean_rows(Slot S, int g0, int ns, int n_min_chain) {
  const int lane = threadIdx.x & 63;
  const int nwaves = (int)(gridDim.x * blockDim.x / 64);
  const int nr = ns * kRows;
  for (int v = (int)((blockIdx.x * blockDim.x + threadIdx.x) / 64); v < nr; v += nwaves) {
    const int sr = g0 * kRows + v;
    const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
    uint32_t count = 0;
    for (uint32_t base = h0; base < h1; base += 64) {
      const uint32_t h = base + lane;
      bool start = false;
      if (h < h1) {
        int32_t uc, dc;
        start = is_start(S, h, n_min_chain, uc, dc);
        S.hit[h].upc = uc;
        S.dnc[h] = dc;
        S.weight[h] = 0u;
      }
      count += (uint32_t)__popcll(__ballot(start));
    }
    if (lane == 0) S.row_nstart[sr] = count;
  }
}

// a4: write the start hits in (sector, row, position) order at the offsets
// given by the scan of the per-row counts over the launched sector range.
// One wave per row, as in k_clean_rows.
__global__ void __launch_bounds__(256) k_start_write(Slot S, int g0, int ns, int n_min_chain) {
  const int lane = threadIdx.x & 63;
  const int nwaves = (int)(gridDim.x * blockDim.x / 64);
  const int nr = ns * kRows;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int v = (int)((blockIdx.x * blockDim.x + threadIdx.x) / 64); v < nr; v += nwaves) {
    const int sr = g0 * kRows + v;
    const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
    uint32_t out = S.tl_base[g0] + S.row_nstart[sr];
    for (uint32_t base = h0; base < h1; base += 64) {
      const uint32_t h = base + lane;
      bool start = false;
      if (h < h1) {
        int32_t uc, dc;
        start = is_start(S, h, n_min_chain, uc, dc);
      }
      const unsigned long long m = __ballot(start);
      if (start) {
        const uint32_t k = out + (uint32_t)__popcll(m & below);
        S.start_hit[k] = (int32_t)h;
        S.start_sr[k] = sr;
      }
      out += (uint32_t)__popcll(m);
    }
  }
}

}  // namespace tpc
