// Cellular-automaton part of the tracker (paper, Abstract: track finding by
// a cellular automaton): per-hit best neighbour pair, mutual-link cleaning
// and start hits of the resulting chains.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

constexpr int kNfRowCap = 1024;   // hits of a neighbour row staged in LDS
constexpr int kNfCand = 16;       // up-row candidates kept per hit
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

// Best (down, up) pair of one hit.  hd/bd (hu/bu): hits and bin offsets of
// row r-1 (r+1) in a common numbering; add_d/add_u turn that numbering into
// sorted-hit indices.
template <class HitPtr, class BinPtr>
__device__ __forceinline__ void best_pair(const DevConst& K, const Hit hh, int row,
                                          const RowBins& Bd, HitPtr hd, BinPtr bd, uint32_t add_d,
                                          const RowBins& Bu, HitPtr hu, BinPtr bu, uint32_t add_u,
                                          uint32_t* cand, int32_t& out_up, int32_t& out_dn) {
  // cand[k * kNfThreads]: this thread's k-th candidate (thread-minor layout,
  // so a wave's accesses fall in distinct LDS banks)
  const float xr = K.row_x[row];
  const float rho_d = K.row_x[row - 1] / xr;
  const float rho_u = K.row_x[row + 1] / xr;
  const float f = (xr - K.row_x[row - 1]) / (K.row_x[row + 1] - K.row_x[row - 1]);
  const float W = K.nf_w;
  const float yh = hh.y, zh = hh.z;
  const float ypd = yh * rho_d, zpd = zh * rho_d;
  const float ypu = yh * rho_u, zpu = zh * rho_u;
  const float sy = sigma_y(K, zh), sz = sigma_z(K, zh);
  const float wy = 1.0f / (1.5f * (sy * sy));
  const float wz = 1.0f / (1.5f * (sz * sz));
  // up-row candidates inside the exact window
  int nu = 0;
  bool overflow = false;
  for_window(Bu, bu, ypu, zpu, W, W, [&](uint32_t u) {
    const Hit x = hu[u];
    if (!(fabsf(x.y - ypu) <= W && fabsf(x.z - zpu) <= W)) return;
    if (nu < kNfCand) cand[nu * kNfThreads] = u;
    else overflow = true;
    ++nu;
  });
  out_up = -1;
  out_dn = -1;
  if (nu == 0) return;
  bool have = false;
  float best = 0.0f;
  uint32_t bid_d = 0, bid_u = 0;
  int32_t bd_i = -1, bu_i = -1;
  auto pair = [&](uint32_t d, const Hit& xd, uint32_t u, const Hit& xu) {
    const float dy = xd.y + (xu.y - xd.y) * f - yh;
    const float dz = xd.z + (xu.z - xd.z) * f - zh;
    const float m = dy * dy * wy + dz * dz * wz;
    const bool better =
        !have || m < best || (m == best && (xd.id < bid_d || (xd.id == bid_d && xu.id < bid_u)));
    if (better) {
      have = true;
      best = m;
      bid_d = xd.id;
      bid_u = xu.id;
      bd_i = (int32_t)(d + add_d);
      bu_i = (int32_t)(u + add_u);
    }
  };
  for_window(Bd, bd, ypd, zpd, W, W, [&](uint32_t d) {
    const Hit xd = hd[d];
    if (!(fabsf(xd.y - ypd) <= W && fabsf(xd.z - zpd) <= W)) return;
    if (!overflow) {
      for (int k = 0; k < nu; ++k) {
        const uint32_t u = cand[k * kNfThreads];
        pair(d, xd, u, hu[u]);
      }
    } else {
      for_window(Bu, bu, ypu, zpu, W, W, [&](uint32_t u) {
        const Hit xu = hu[u];
        if (!(fabsf(xu.y - ypu) <= W && fabsf(xu.z - zpu) <= W)) return;
        pair(d, xd, u, xu);
      });
    }
  });
  if (have && best <= K.nf_mmax) {
    out_up = bu_i;
    out_dn = bd_i;
  }
}

// a3: one block per (sector, row).  For each hit h of row r (1..157), the
// pair (d in row r-1, u in row r+1) inside the origin-pointing windows
// |y - y_h x_r'/x_r| <= W, |z - z_h x_r'/x_r| <= W whose straight line passes
// closest to h, measured by m = dy^2 / (1.5 sy^2) + dz^2 / (1.5 sz^2);
// ties go to the smaller (id_d, id_u); the pair is kept if m <= m_max.
// Rows r-1 and r+1 (hits and bin offsets) are staged in LDS when they hold
// at most kNfRowCap hits; otherwise read from global memory.  Rows 0 and 158
// get no links.
__global__ void __launch_bounds__(kNfThreads) k_neighbours(Slot S, DevConst K, int g0) {
  __shared__ Hit sh_d[kNfRowCap];
  __shared__ Hit sh_u[kNfRowCap];
  __shared__ uint32_t sb_d[kNfRowCap + 1];
  __shared__ uint32_t sb_u[kNfRowCap + 1];
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
  if (h0 == h1) return;
  const uint32_t od = S.row_off[sr - 1], nd = h0 - od;
  const uint32_t ou = h1, nu = S.row_off[sr + 2] - h1;
  const RowBins Bd = S.bins[sr - 1], Bu = S.bins[sr + 1];
  const int nbd = Bd.ny * Bd.nz, nbu = Bu.ny * Bu.nz;
  uint32_t* my = cand + threadIdx.x;
  if (nd <= (uint32_t)kNfRowCap && nu <= (uint32_t)kNfRowCap) {
    for (uint32_t j = threadIdx.x; j < nd; j += blockDim.x) sh_d[j] = S.hit[od + j];
    for (uint32_t j = threadIdx.x; j < nu; j += blockDim.x) sh_u[j] = S.hit[ou + j];
    for (int j = threadIdx.x; j <= nbd; j += blockDim.x) sb_d[j] = S.bin_off[Bd.base + j] - od;
    for (int j = threadIdx.x; j <= nbu; j += blockDim.x) sb_u[j] = S.bin_off[Bu.base + j] - ou;
    __syncthreads();
    for (uint32_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
      int32_t up, dn;
      best_pair(K, S.hit[h], row, Bd, (const Hit*)sh_d, (const uint32_t*)sb_d, od, Bu,
                (const Hit*)sh_u, (const uint32_t*)sb_u, ou, my, up, dn);
      S.up[h] = up;
      S.dn[h] = dn;
    }
  } else {
    for (uint32_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
      int32_t up, dn;
      best_pair(K, S.hit[h], row, Bd, (const Hit*)S.hit, (const uint32_t*)(S.bin_off + Bd.base), 0u,
                Bu, (const Hit*)S.hit, (const uint32_t*)(S.bin_off + Bu.base), 0u, my, up, dn);
      S.up[h] = up;
      S.dn[h] = dn;
    }
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
