// a6 hit ownership and tracklet selection, a7 output refit.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
  return v;
}

// Rows are walked RB at a time (a tuning knob): the hit-list entries of a
// batch are loaded together, then the weights of their hits, so a batch
// costs two memory round trips instead of two per row.

// hv[u] = the tracklet's hit in row r0+u if that row is inside [rin, rout]
// of an active lane, else -1 (rows outside are not read); gr = the
// tracklet's sector times the rows per sector.
template <int RB>
__device__ __forceinline__ void load_row_batch(const Slot& S, const TlList& hits, int gr, int r0,
                                               bool active, int rin, int rout,
                                               int32_t (&hv)[RB]) {
  uint32_t e[RB], f[RB];
#pragma unroll
  for (int u = 0; u < RB; ++u) {
    const int r = r0 + u;
    const bool in = active && r >= rin && r <= rout;
    e[u] = in ? hits.at(r) : (uint32_t)kNoEntry;
    f[u] = in ? (uint32_t)S.row_off[gr + r] : 0u;
  }
#pragma unroll
  for (int u = 0; u < RB; ++u) hv[u] = entry_hit(e[u], f[u]);
}

template <int RB>
__device__ __forceinline__ void load_weights(const Slot& S, const int32_t (&hv)[RB],
                                             uint32_t (&wv)[RB]) {
#pragma unroll
  for (int u = 0; u < RB; ++u) wv[u] = hv[u] >= 0 ? S.weight[hv[u]] : 0u;
}

// a6: a valid tracklet becomes a track if it owns (holds the maximal weight
// of) at least n_min_track of its hits.  Writes 1/0 per tracklet of the
// range; the scan of these flags places the tracks.
// Lane per tracklet; a wave walks the rows its 64 consecutive tracklets
// span together, so each row's hit-list reads are contiguous (tile layout).
// The tracklets are in sector order: each XCD (blocks are dispatched
// round-robin over the 8; the grid is a multiple of 8) walks a contiguous
// chunk of them, a whole number of waves, so a sector's hit lists and
// weights are read through one XCD's L2.  Wave-aligned start of this
// wave's first group of 64, the chunk's end, and the stride.
struct XcdChunk {
  uint32_t first, end, stride;
};
__device__ __forceinline__ XcdChunk xcd_chunk(uint32_t total) {
  constexpr uint32_t kXcd = 8;
  const uint32_t xcd = blockIdx.x % kXcd, jb = blockIdx.x / kXcd;
  const uint32_t nbx = gridDim.x / kXcd;
  const uint32_t chunk = ((total + kXcd - 1) / kXcd + 63u) & ~63u;
  const uint32_t c0 = min(total, xcd * chunk);
  XcdChunk x;
  x.first = c0 + ((jb * blockDim.x + threadIdx.x) & ~63u);
  x.end = min(total, c0 + chunk);
  x.stride = nbx * blockDim.x;
  return x;
}

template <int RB>
__global__ void __launch_bounds__(256) k_select(Slot S, DevConst K, int g0) {
  const uint32_t total = S.range_cnt[0];
  const uint32_t base = S.tl_base[g0];
  const uint32_t lane = threadIdx.x & 63;
  const XcdChunk xc = xcd_chunk(total);
  for (uint32_t tb = xc.first; tb < xc.end; tb += xc.stride) {
    const uint32_t t = tb + lane;
    const uint32_t T = base + t;
    bool valid = false;
    int rin = 1, rout = 0;
    uint32_t w = 0;
    int gr = 0;
    if (t < total) {
      const int32_t* info = S.tl_info + (size_t)T * 4;
      valid = info[3] != 0;
      if (valid) {
        rin = info[1];
        rout = info[2];
        w = S.tl_weight[T];
        gr = S.start_sr[T] / kRows * kRows;
      }
    }
    const int lo = wave_min(valid ? rin : kRows), hi = wave_max(valid ? rout : -1);
    const TlList hits = tl_list(S, T);
    int cnt = 0;
    for (int r0 = lo; r0 <= hi; r0 += RB) {
      int32_t hv[RB];
      load_row_batch(S, hits, gr, r0, valid, rin, rout, hv);
      uint32_t wv[RB];
      load_weights(S, hv, wv);
#pragma unroll
      for (int u = 0; u < RB; ++u) cnt += (hv[u] >= 0 && wv[u] == w) ? 1 : 0;
    }
    if (t < total) S.tl_sel[t] = valid && cnt >= K.n_min_track ? 1u : 0u;
  }
}

// Selected tracklets -> tracks of the range (in tracklet order), each with
// its owned hits compacted (ascending row).  Lane per tracklet, rows walked
// together by the wave as in k_select.  The range's track region holds
// every track its hits allow (each owns >= n_min_track hits of its own); a
// position beyond it is not written and raises the capacity error.
template <int RB>
__global__ void __launch_bounds__(256) k_track_write(Slot S, int g0, int ns) {
  const uint32_t total = S.range_cnt[0];
  const uint32_t ntk = S.range_cnt[1];
  const uint32_t tl0 = S.tl_base[g0], tk0 = S.tk_base[g0];
  const uint32_t tk_room = S.tk_base[g0 + ns] - tk0;
  const uint32_t lane = threadIdx.x & 63;
  const XcdChunk xc = xcd_chunk(total);
  for (uint32_t tb = xc.first; tb < xc.end; tb += xc.stride) {
    const uint32_t t = tb + lane;
    const uint32_t T = tl0 + t;
    bool sel = false;
    uint32_t k = 0, w = 0;
    int rin = 1, rout = 0;
    int gr = 0;
    if (t < total) {
      const uint32_t pos = S.tl_sel[t];
      const uint32_t next = t + 1 < total ? S.tl_sel[t + 1] : ntk;
      sel = next != pos;
      if (sel && pos >= tk_room) {
        atomicOr(&S.err[2], 1u);
        sel = false;
      }
      if (sel) {
        k = tk0 + pos;
        const int32_t* info = S.tl_info + (size_t)T * 4;
        rin = info[1];
        rout = info[2];
        w = S.tl_weight[T];
        gr = S.start_sr[T] / kRows * kRows;
      }
    }
    const int lo = wave_min(sel ? rin : kRows), hi = wave_max(sel ? rout : -1);
    const TlList hits = tl_list(S, T);
    int32_t* own = S.tk_own + (size_t)k * kRows;
    uint8_t* own_row = S.tk_own_row + (size_t)k * kRows;
    int cnt = 0;
    for (int r0 = lo; r0 <= hi; r0 += RB) {
      int32_t hv[RB];
      load_row_batch(S, hits, gr, r0, sel, rin, rout, hv);
      uint32_t wv[RB];
      load_weights(S, hv, wv);
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        if (hv[u] >= 0 && wv[u] == w) {
          own[cnt] = hv[u];
          own_row[cnt] = (uint8_t)(r0 + u);
          ++cnt;
        }
      }
    }
    if (sel) {
      S.tk_tracklet[k] = (int32_t)T;
      S.tk_nown[k] = cnt;
    }
  }
}

void launch_select(int rb, int blocks, hipStream_t st, const Slot& S, const DevConst& K, int g0) {
  switch (rb) {
    case 4: k_select<4><<<blocks, 256, 0, st>>>(S, K, g0); break;
    case 16: k_select<16><<<blocks, 256, 0, st>>>(S, K, g0); break;
    default: k_select<8><<<blocks, 256, 0, st>>>(S, K, g0); break;
  }
}

void launch_track_write(int rb, int blocks, hipStream_t st, const Slot& S, int g0, int ns) {
  switch (rb) {
    case 4: k_track_write<4><<<blocks, 256, 0, st>>>(S, g0, ns); break;
    case 16: k_track_write<16><<<blocks, 256, 0, st>>>(S, g0, ns); break;
    default: k_track_write<8><<<blocks, 256, 0, st>>>(S, g0, ns); break;
  }
}

struct PassOut {
  Helix<double> st;
  int rlast, jlast, n;
  double chi2;
};

// One inward pass over the owned hits own[jmin .. n-1] (ascending rows):
// state reset to the outermost hit with the prior covariance, transport row
// by row, update with every owned hit (no gate).  A failed transport ends
// the pass.  Memory reads are issued ahead of their use.
__device__ __forceinline__ void refit_pass(const Slot& S, const DevConst& K, const int32_t* own,
                           const uint8_t* own_row, int n, int jmin, double s0, double t0,
                           double q0, PassOut& o) {
  const Hit xo = S.hit[own[n - 1]];
  Helix<double> st;
  st.y = (double)xo.y;
  st.z = (double)xo.z;
  st.s = s0;
  st.t = t0;
  st.q = q0;
  const double sy0 = K.sy0, sy1z = K.sy1zd, sz0 = K.sz0, sz1z = K.sz1zd;
  {
    const double sy = sy0 + sy1z * fabs(st.z), sz = sz0 + sz1z * fabs(st.z);
    reset_cov(st, sy * sy, sz * sz, (double)K.cs0, (double)K.ct0, (double)K.cq0);
  }
  o.st = st;
  o.rlast = own_row[n - 1];
  o.jlast = n - 1;
  o.n = 1;
  o.chi2 = 0.0;
  const double smax = K.smax, chi2max = K.chi2max;
  // row-synchronous walk (every lane moves one row per iteration).  Every
  // memory read of a step is issued at its top and used after the
  // transport: the radius of the next row, the record of the next owned
  // hit (own[j]) and the list entry after it (own[j - 1]); indices clamped
  // into [jmin, n) and row 0 so the reads stay inside the lists.
  int j = n - 2;
  int rn = j >= jmin ? (int)own_row[j] : -1;
  int32_t pn = own[max(j, jmin)];
  const int rstop = j >= jmin ? (int)own_row[jmin] : o.rlast;
  double x_hi = (double)K.row_x[o.rlast];
  float x_next = K.row_x[max(o.rlast - 1, 0)];
  for (int r = o.rlast - 1; r >= rstop; --r) {
    const double x_lo = (double)x_next;
    x_next = K.row_x[max(r - 1, 0)];
    const Hit xh = S.hit[pn];
    const int ja = max(j - 1, jmin);
    const int32_t p_after = own[ja];
    const int r_after = own_row[ja];
    if (!transport(st, x_lo - x_hi, K.bd, smax, K.kkd, K.m2d)) break;
    x_hi = x_lo;
    if (r != rn) continue;
    const double sy = sy0 + sy1z * fabs(st.z), sz = sz0 + sz1z * fabs(st.z);
    double ch = 0.0;
    kalman_update(st, (double)xh.y, (double)xh.z, sy * sy, sz * sz, chi2max, smax, false, &ch);
    o.chi2 = o.chi2 + ch;
    o.n += 1;
    o.st = st;
    o.rlast = r;
    o.jlast = j;
    --j;
    pn = p_after;
    rn = j >= jmin ? r_after : -1;
  }
}

// a7: refit of each track over its owned hits, in double, three inward
// passes.  Pass 1 starts from the tracklet's inner (s, T, Q) with s carried
// to the outermost owned row along the circle (sin phi is linear in x);
// each later pass starts from the previous pass's result carried back the
// same way, so the Jacobians are evaluated along the fitted track.  Output
// at the innermost fitted hit; its cluster is marked for the canonical
// ordering.
__global__ void __launch_bounds__(256) k_refit(Slot S, DevConst K, int g0, int ns) {
  const uint32_t tk0 = S.tk_base[g0];
  // tracks past the region were not written (capacity error raised)
  const uint32_t total = min(S.range_cnt[1], S.tk_base[g0 + ns] - tk0);
  // each XCD (blocks are dispatched round-robin over the 8) a contiguous
  // chunk of the tracks, which are in sector order: a sector's hits are read
  // through one XCD's L2
  constexpr uint32_t kXcd = 8;
  const uint32_t xcd = blockIdx.x % kXcd, jb = blockIdx.x / kXcd;
  const uint32_t nbx = (gridDim.x - xcd + kXcd - 1) / kXcd;
  const uint32_t chunk = (total + kXcd - 1) / kXcd;
  const uint32_t c0 = min(total, xcd * chunk);
  const uint32_t c1 = min(total, c0 + chunk);
  unsigned nfit = 0;
  for (uint32_t t = c0 + jb * blockDim.x + threadIdx.x; t < c1; t += nbx * blockDim.x) {
    ++nfit;
    const uint32_t k = tk0 + t;
    const int32_t T = S.tk_tracklet[k];
    const int n = S.tk_nown[k];
    const int32_t* own = S.tk_own + (size_t)k * kRows;
    const uint8_t* own_row = S.tk_own_row + (size_t)k * kRows;
    int32_t* out = S.tk_info + (size_t)k * 4;
    out[0] = 0;
    if (n < 1) continue;
    const int ro = own_row[n - 1];
    const int rin_tl = S.tl_info[(size_t)T * 4 + 1];
    const float* sv = S.tl_state + (size_t)T * 5;
    const double smax = K.smax;
    PassOut o;
    bool ok = true;
    {
      const double sin_ = sv[2], tin = sv[3], qin = sv[4];
      const double s0 = sin_ + (K.bd * qin) * ((double)K.row_x[ro] - (double)K.row_x[rin_tl]);
      if (!(fabs(s0) <= smax)) ok = false;
      else refit_pass(S, K, own, own_row, n, 0, s0, tin, qin, o);
    }
    for (int pass = 1; ok && pass < 3; ++pass) {
      const double sin_ = o.st.s, tin = o.st.t, qin = o.st.q;
      const double s0 = sin_ + (K.bd * qin) * ((double)K.row_x[ro] - (double)K.row_x[o.rlast]);
      if (!(fabs(s0) <= smax)) ok = false;
      else refit_pass(S, K, own, own_row, n, o.jlast, s0, tin, qin, o);
    }
    if (!ok || o.n < K.n_min_track) continue;
    out[0] = 1;
    out[1] = o.n;
    out[2] = o.rlast;
    out[3] = ro;
    double* par = S.tk_par + (size_t)k * 5;
    par[0] = o.st.y;
    par[1] = o.st.z;
    par[2] = o.st.s;
    par[3] = o.st.t;
    par[4] = o.st.q;
    double* cov = S.tk_cov + (size_t)k * 15;
#pragma unroll
    for (int i = 0; i < 15; ++i) cov[i] = o.st.c[i];
    S.tk_chi2[k] = o.chi2;
    S.tmap[S.hit[own[o.jlast]].id] = (int32_t)k;
  }
  wave_add_u64(&S.stats[3], nfit);
}

}  // namespace tpc
