// Cellular-automaton part of the tracker (paper, Abstract: track finding by
// a cellular automaton): per-hit best neighbour pair, mutual-link cleaning
// and start hits of the resulting chains.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

constexpr int kNfThreads = 256;

// Visit the hits of one row that can lie inside [yc - wy, yc + wy] x
// [zc - wz, zc + wz]: every bin the window touches (plus a small margin so
// rounding cannot hide a hit); the caller applies the exact window test.
// `bins` is indexed by the row's bin number and holds hit positions in the
// numbering of whatever `fn` receives.
template <class BinPtr, class Fn>
__device__ __forceinline__ void for_window(const RowBins& b, BinPtr bins, float yc, float zc,
                                           float wy, float wz, Fn&& fn) {
  const float eps = 1e-3f;
  const int iy0 = bin_y(b, yc - wy - eps), iy1 = bin_y(b, yc + wy + eps);
  const int iz0 = bin_z(b, zc - wz - eps), iz1 = bin_z(b, zc + wz + eps);
  for (int iz = iz0; iz <= iz1; ++iz) {
    const int first = iz * b.ny;
    const uint32_t p0 = bins[first + iy0];
    const uint32_t p1 = bins[first + iy1 + 1];
    for (uint32_t p = p0; p < p1; ++p) fn(p);
  }
}

// A neighbour row seen through global memory (Hit records, absolute bin
// offsets); `add` turns the numbering into sorted-hit indices.
struct RowGlobal {
  const Hit* hit;
  const uint32_t* bins;
  uint32_t add;
  __device__ float2 yz(uint32_t p) const {
    const Hit x = hit[p];
    return make_float2(x.y, x.z);
  }
  __device__ uint32_t id(uint32_t p) const { return hit[p].id; }
};
__device__ __forceinline__ float nf_metric(float yd, float zd, float yu, float zu, float yh, float zh,
                                           float f, float wy, float wz) {
  const float dy = yd + (yu - yd) * f - yh;
  const float dz = zd + (zu - zd) * f - zh;
  return dy * dy * wy + dz * dz * wz;
}

// Best (down, up) pair of one hit by a nested scan of the two windows.
template <class RD, class RU>
__device__ void nested_pair(const DevConst& K, float yh, float zh, int row, const RowBins& Bd,
                            const RD& rd, const RowBins& Bu, const RU& ru, int32_t& out_up,
                            int32_t& out_dn) {
  const float xr = K.row_x[row];
  const float rho_d = K.row_x[row - 1] / xr;
  const float rho_u = K.row_x[row + 1] / xr;
  const float f = (xr - K.row_x[row - 1]) / (K.row_x[row + 1] - K.row_x[row - 1]);
  const float W = K.nf_w;
  const float ypd = yh * rho_d, zpd = zh * rho_d;
  const float ypu = yh * rho_u, zpu = zh * rho_u;
  const float sy = sigma_y(K, zh), sz = sigma_z(K, zh);
  const float wy = 1.0f / (1.5f * (sy * sy));
  const float wz = 1.0f / (1.5f * (sz * sz));
  bool have = false;
  float best = 0.0f;
  uint32_t bid_d = 0, bid_u = 0;
  int32_t bd_i = -1, bu_i = -1;
  for_window(Bd, rd.bins, ypd, zpd, W, W, [&](uint32_t d) {
    const float2 a = rd.yz(d);
    if (!(fabsf(a.x - ypd) <= W && fabsf(a.y - zpd) <= W)) return;
    const uint32_t idd = rd.id(d);
    for_window(Bu, ru.bins, ypu, zpu, W, W, [&](uint32_t u) {
      const float2 b = ru.yz(u);
      if (!(fabsf(b.x - ypu) <= W && fabsf(b.y - zpu) <= W)) return;
      const uint32_t idu = ru.id(u);
      const float m = nf_metric(a.x, a.y, b.x, b.y, yh, zh, f, wy, wz);
      const bool better =
          !have || m < best || (m == best && (idd < bid_d || (idd == bid_d && idu < bid_u)));
      if (better) {
        have = true;
        best = m;
        bid_d = idd;
        bid_u = idu;
        bd_i = (int32_t)(d + rd.add);
        bu_i = (int32_t)(u + ru.add);
      }
    });
  });
  const bool ok = have && best <= K.nf_mmax;
  out_up = ok ? bu_i : -1;
  out_dn = ok ? bd_i : -1;
}

constexpr int kNfCand = 32;      // up-row candidates kept per hit before a nested scan

// a3: one block per (sector, row).  For each hit h of row r (1..157), the
// pair (d in row r-1, u in row r+1) inside the origin-pointing windows
// |y - y_h x_r'/x_r| <= W, |z - z_h x_r'/x_r| <= W whose straight line passes
// closest to h, measured by m = dy^2 / (1.5 sy^2) + dz^2 / (1.5 sz^2);
// ties go to the smaller (id_d, id_u); the pair is kept if m <= m_max.
// Rows 0 and 158 get no links.
// One lane per hit; the up-row candidates are listed once (LDS,
// thread-minor so a wave's accesses fall in distinct banks) and paired with
// every down-row candidate; a hit with more than kNfCand up candidates takes
// a nested scan.  The neighbour rows are read through the caches rather than
// staged: the small LDS footprint keeps enough waves resident to hide the
// load latency (measured faster than staging both rows in LDS).
__global__ void __launch_bounds__(kNfThreads) k_neighbours(Slot S, DevConst K, int g0) {
  __shared__ uint32_t cand[kNfCand * kNfThreads];
  const int row = blockIdx.x;
  const int g = g0 + blockIdx.y;
  const int sr = g * kRows + row;
  const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
  if (row == 0 || row == kRows - 1) {
    for (uint32_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
      S.up[h] = -1;
      S.dn[h] = -1;
    }
    return;
  }
  const RowBins Bd = S.bins[sr - 1], Bu = S.bins[sr + 1];
  const RowGlobal rd{S.hit, S.bin_off + Bd.base, 0u}, ru{S.hit, S.bin_off + Bu.base, 0u};
  const float xr = K.row_x[row];
  const float rho_d = K.row_x[row - 1] / xr;
  const float rho_u = K.row_x[row + 1] / xr;
  const float f = (xr - K.row_x[row - 1]) / (K.row_x[row + 1] - K.row_x[row - 1]);
  const float W = K.nf_w;
  uint32_t* my = cand + threadIdx.x;
  for (uint32_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
    const Hit x = S.hit[h];
    const float yh = x.y, zh = x.z;
    const float ypu = yh * rho_u, zpu = zh * rho_u;
    int nu = 0;
    for_window(Bu, ru.bins, ypu, zpu, W, W, [&](uint32_t u) {
      const float2 c = ru.yz(u);
      if (!(fabsf(c.x - ypu) <= W && fabsf(c.y - zpu) <= W)) return;
      if (nu < kNfCand) my[nu * kNfThreads] = u;
      ++nu;
    });
    int32_t up = -1, dn = -1;
    if (nu > kNfCand) {
      nested_pair(K, yh, zh, row, Bd, rd, Bu, ru, up, dn);
    } else if (nu > 0) {
      const float ypd = yh * rho_d, zpd = zh * rho_d;
      const float sy = sigma_y(K, zh), sz = sigma_z(K, zh);
      const float wy = 1.0f / (1.5f * (sy * sy));
      const float wz = 1.0f / (1.5f * (sz * sz));
      bool have = false;
      float best = 0.0f;
      uint32_t bid_d = 0, bid_u = 0;
      for_window(Bd, rd.bins, ypd, zpd, W, W, [&](uint32_t d) {
        const Hit xd = S.hit[d];
        if (!(fabsf(xd.y - ypd) <= W && fabsf(xd.z - zpd) <= W)) return;
        for (int k = 0; k < nu; ++k) {
          const uint32_t u = my[k * kNfThreads];
          const Hit xu = S.hit[u];
          const float m = nf_metric(xd.y, xd.z, xu.y, xu.z, yh, zh, f, wy, wz);
          const bool better =
              !have || m < best || (m == best && (xd.id < bid_d || (xd.id == bid_d && xu.id < bid_u)));
          if (better) {
            have = true;
            best = m;
            bid_d = xd.id;
            bid_u = xu.id;
            dn = (int32_t)d;
            up = (int32_t)u;
          }
        }
      });
      if (!(have && best <= K.nf_mmax)) {
        up = -1;
        dn = -1;
      }
    }
    S.up[h] = up;
    S.dn[h] = dn;
  }
}

// Start of a cleaned chain of >= 3 hits, from the links of a3 only.
__device__ __forceinline__ bool is_start(const Slot& S, uint32_t h, int32_t& uc, int32_t& dc) {
  const int32_t u = S.up[h], d = S.dn[h];
  uc = (u >= 0 && S.dn[u] == (int32_t)h) ? u : -1;
  dc = (d >= 0 && S.up[d] == (int32_t)h) ? d : -1;
  if (uc < 0 || dc >= 0) return false;
  const int32_t uu = S.up[uc];
  return uu >= 0 && S.dn[uu] == uc;
}

// a4: keep a link only if it is mutual; count the start hits of each row.
// Also clears the hit weights used by the tracklet selection.
__global__ void __launch_bounds__(256) k_clean_rows(Slot S, int g0) {
  __shared__ uint32_t count;
  const int row = blockIdx.x;
  const int g = g0 + blockIdx.y;
  const int sr = g * kRows + row;
  const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (uint32_t base = h0; base < h1; base += blockDim.x) {
    const uint32_t h = base + threadIdx.x;
    bool start = false;
    if (h < h1) {
      int32_t uc, dc;
      start = is_start(S, h, uc, dc);
      S.hit[h].upc = uc;
      S.dnc[h] = dc;
      S.weight[h] = 0u;
    }
    const unsigned long long m = __ballot(start);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&count, (uint32_t)__popcll(m));
  }
  __syncthreads();
  if (threadIdx.x == 0) S.row_nstart[sr] = count;
}

// a4: write the start hits in (sector, row, position) order at the offsets
// given by the scan of the per-row counts over the launched sector range.
__global__ void __launch_bounds__(256) k_start_write(Slot S, int g0) {
  __shared__ uint32_t wcount[4];
  __shared__ uint32_t running;
  const int row = blockIdx.x;
  const int g = g0 + blockIdx.y;
  const int sr = g * kRows + row;
  const uint32_t h0 = S.row_off[sr], h1 = S.row_off[sr + 1];
  const uint32_t base_out = S.tl_base[g0] + S.row_nstart[sr];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) running = 0;
  __syncthreads();
  for (uint32_t base = h0; base < h1; base += blockDim.x) {
    const uint32_t h = base + threadIdx.x;
    bool start = false;
    if (h < h1) {
      int32_t uc, dc;
      start = is_start(S, h, uc, dc);
    }
    const unsigned long long m = __ballot(start);
    if (lane == 0) wcount[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = running, tot = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      if (i < w) before += wcount[i];
      tot += wcount[i];
    }
    if (start) {
      const uint32_t k = base_out + before + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      S.start_hit[k] = (int32_t)h;
      S.start_sr[k] = sr;
    }
    __syncthreads();
    if (threadIdx.x == 0) running += tot;
    __syncthreads();
  }
}

}  // namespace tpc
