// Cellular-automaton part of the tracker (paper, Abstract: track finding by
// a cellular automaton): per-hit best neighbour pair, mutual-link cleaning
// and start hits of the resulting chains.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

// Visit the sorted hits of row `sr` that can lie inside
// [yc - w, yc + w] x [zc - w, zc + w] (a superset: every bin the window
// touches, with a small margin so that rounding cannot hide a hit).
template <class Fn>
__device__ __forceinline__ void for_window(const Slot& S, int sr, float yc, float zc, float wy,
                                           float wz, Fn&& fn) {
  const RowBins b = S.bins[sr];
  const float eps = 1e-3f;
  const int iy0 = bin_y(b, yc - wy - eps), iy1 = bin_y(b, yc + wy + eps);
  const int iz0 = bin_z(b, zc - wz - eps), iz1 = bin_z(b, zc + wz + eps);
  for (int iz = iz0; iz <= iz1; ++iz) {
    const int first = b.base + iz * b.ny;
    const uint32_t p0 = S.bin_off[first + iy0];
    const uint32_t p1 = S.bin_off[first + iy1 + 1];
    for (uint32_t p = p0; p < p1; ++p) fn(p);
  }
}

// a3: one block per (sector, row).  For each hit h of row r (1..157), the
// pair (d in row r-1, u in row r+1) inside the origin-pointing windows
// |y - y_h x_r'/x_r| <= W, |z - z_h x_r'/x_r| <= W whose straight line passes
// closest to h, measured by m = dy^2 / (1.5 sy^2) + dz^2 / (1.5 sz^2);
// ties go to the smaller (id_d, id_u); the pair is kept if m <= m_max.
// Rows 0 and 158 get no links.  Also clears the per-sector counters.
__global__ void __launch_bounds__(256) k_neighbours(Slot S, DevConst K, int g0) {
  const int row = blockIdx.x;
  const int g = g0 + blockIdx.y;
  const int sr = g * kRows + row;
  const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
  if (row == 0 && threadIdx.x == 0) {
    S.n_start[g] = 0;
    S.n_track[g] = 0;
  }
  if (row == 0 || row == kRows - 1) {
    for (uint32_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
      S.up[h] = -1;
      S.dn[h] = -1;
    }
    return;
  }
  const float xr = K.row_x[row];
  const float rho_d = K.row_x[row - 1] / xr;
  const float rho_u = K.row_x[row + 1] / xr;
  const float f = (xr - K.row_x[row - 1]) / (K.row_x[row + 1] - K.row_x[row - 1]);
  const float W = K.nf_w;
  for (uint32_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
    const float yh = S.hy[h], zh = S.hz[h];
    const float ypd = yh * rho_d, zpd = zh * rho_d;
    const float ypu = yh * rho_u, zpu = zh * rho_u;
    const float sy = sigma_y(K, zh), sz = sigma_z(K, zh);
    const float wy = 1.0f / (1.5f * (sy * sy));
    const float wz = 1.0f / (1.5f * (sz * sz));
    bool have = false;
    float best = 0.0f;
    uint32_t bid_d = 0, bid_u = 0;
    int32_t bd = -1, bu = -1;
    for_window(S, sr - 1, ypd, zpd, W, W, [&](uint32_t d) {
      const float yd = S.hy[d], zd = S.hz[d];
      if (!(fabsf(yd - ypd) <= W && fabsf(zd - zpd) <= W)) return;
      const uint32_t idd = S.hid[d];
      for_window(S, sr + 1, ypu, zpu, W, W, [&](uint32_t u) {
        const float yu = S.hy[u], zu = S.hz[u];
        if (!(fabsf(yu - ypu) <= W && fabsf(zu - zpu) <= W)) return;
        const uint32_t idu = S.hid[u];
        const float dy = yd + (yu - yd) * f - yh;
        const float dz = zd + (zu - zd) * f - zh;
        const float m = dy * dy * wy + dz * dz * wz;
        const bool better = !have || m < best ||
                            (m == best && (idd < bid_d || (idd == bid_d && idu < bid_u)));
        if (better) {
          have = true;
          best = m;
          bid_d = idd;
          bid_u = idu;
          bd = (int32_t)d;
          bu = (int32_t)u;
        }
      });
    });
    const bool ok = have && best <= K.nf_mmax;
    S.up[h] = ok ? bu : -1;
    S.dn[h] = ok ? bd : -1;
  }
}

// a4: keep a link only if it is mutual (reading the links of a3 only), and
// collect the start hits: first hit of a cleaned chain of >= 3 hits.  Start
// hits go to the sector's region with a wave-aggregated atomic.  Also
// clears the hit weights used by the tracklet selection.
__global__ void __launch_bounds__(256) k_clean_start(Slot S, int g0) {
  const int row = blockIdx.x;
  const int g = g0 + blockIdx.y;
  const int sr = g * kRows + row;
  const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
  const uint32_t cap = S.tl_base[g + 1] - S.tl_base[g];
  for (uint32_t base = h0; base < h1; base += blockDim.x) {
    const uint32_t h = base + threadIdx.x;
    bool start = false;
    if (h < h1) {
      const int32_t u = S.up[h], d = S.dn[h];
      const int32_t uc = (u >= 0 && S.dn[u] == (int32_t)h) ? u : -1;
      const int32_t dc = (d >= 0 && S.up[d] == (int32_t)h) ? d : -1;
      S.upc[h] = uc;
      S.dnc[h] = dc;
      S.weight[h] = 0u;
      if (uc >= 0 && dc < 0) {
        const int32_t uu = S.up[uc];
        start = uu >= 0 && S.dn[uu] == uc;
      }
    }
    const unsigned long long m = __ballot(start);
    if (m) {
      const int lane = threadIdx.x & 63;
      const int leader = __ffsll((long long)m) - 1;
      uint32_t first = 0;
      if (lane == leader) first = atomicAdd(&S.n_start[g], (uint32_t)__popcll(m));
      first = __shfl(first, leader, 64);
      if (start) {
        const uint32_t k = first + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (k < cap) S.start_hit[S.tl_base[g] + k] = (int32_t)h;
        else atomicAdd(&S.err[2], 1u);
      }
    }
  }
}

// Prefix sums of a per-sector count over the launched sector range, so that
// a flat work index can be mapped to (sector, item).  One block.
__global__ void __launch_bounds__(1024) k_flatten(const uint32_t* cnt, uint32_t* flat, int g0, int ns) {
  __shared__ uint32_t w[64];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ns; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < ns ? cnt[g0 + i] : 0u;
    uint32_t tot;
    // wave scan then block scan
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t t = __shfl_up(x, d, 64);
      if (lane >= d) x += t;
    }
    if (lane == 63) w[wv] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
      uint32_t s = threadIdx.x < (blockDim.x >> 6) ? w[threadIdx.x] : 0u;
      for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(s, d, 64);
        if ((int)threadIdx.x >= d) s += t;
      }
      if (threadIdx.x < (blockDim.x >> 6)) w[32 + threadIdx.x] = s;
    }
    __syncthreads();
    tot = w[32 + (blockDim.x >> 6) - 1];
    const uint32_t before = wv ? w[32 + wv - 1] : 0u;
    if (i < ns) flat[i] = carry + before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) flat[ns] = carry;
}

}  // namespace tpc
