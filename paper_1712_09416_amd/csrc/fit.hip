// a6 hit ownership and tracklet selection, a7 output refit.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

__device__ __forceinline__ int flat_find_f(const uint32_t* flat, int ns, uint32_t t) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (flat[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// a6: every hit keeps the largest weight (n << 24 | 0xFFFFFF - start ID) of
// the valid tracklets that contain it.
__global__ void __launch_bounds__(64) k_weights(Slot S, int g0, int ns) {
  const uint32_t total = S.flat_tl[ns];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int gi = flat_find_f(S.flat_tl, ns, t);
    const uint32_t T = S.tl_base[g0 + gi] + (t - S.flat_tl[gi]);
    const int32_t* info = S.tl_info + (size_t)T * 4;
    if (!info[3]) continue;
    const uint32_t w = S.tl_weight[T];
    const int32_t* hits = S.tl_hits + (size_t)T * kRows;
    for (int r = info[1]; r <= info[2]; ++r) {
      const int32_t h = hits[r];
      if (h >= 0) atomicMax(&S.weight[h], w);
    }
  }
}

// a6: a valid tracklet becomes a track if it owns (holds the maximal weight
// of) at least n_min_track of its hits.
__global__ void __launch_bounds__(64) k_select(Slot S, DevConst K, int g0, int ns) {
  const uint32_t total = S.flat_tl[ns];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int gi = flat_find_f(S.flat_tl, ns, t);
    const int g = g0 + gi;
    const uint32_t T = S.tl_base[g] + (t - S.flat_tl[gi]);
    const int32_t* info = S.tl_info + (size_t)T * 4;
    if (!info[3]) continue;
    const uint32_t w = S.tl_weight[T];
    const int32_t* hits = S.tl_hits + (size_t)T * kRows;
    int cnt = 0;
    for (int r = info[1]; r <= info[2]; ++r) {
      const int32_t h = hits[r];
      cnt += (h >= 0 && S.weight[h] == w) ? 1 : 0;
    }
    if (cnt < K.n_min_track) continue;
    const uint32_t k = atomicAdd(&S.n_track[g], 1u);
    if (k < S.tk_base[g + 1] - S.tk_base[g]) S.tk_tracklet[S.tk_base[g] + k] = (int32_t)T;
    else atomicAdd(&S.err[2], 1u);
  }
}

struct PassOut {
  Helix<double> st;
  int rlast, n;
  double chi2;
};

// owned hit of the tracklet at row r, or -1
__device__ __forceinline__ int32_t owned_at(const Slot& S, const int32_t* hits, uint32_t w, int r) {
  const int32_t h = hits[r];
  return (h >= 0 && S.weight[h] == w) ? h : -1;
}

// One inward pass from the outermost owned row ro down to rmin: state reset
// to the hit at ro with the prior covariance, then transport row by row and
// update with every owned hit (no gate).  A failed transport ends the pass.
__device__ void refit_pass(const Slot& S, const DevConst& K, const int32_t* hits, uint32_t w, int ro,
                           int rmin, double s0, double t0, double q0, PassOut& o) {
  const int32_t ho = hits[ro];
  Helix<double> st;
  st.y = (double)S.hy[ho];
  st.z = (double)S.hz[ho];
  st.s = s0;
  st.t = t0;
  st.q = q0;
  const double sy0 = K.sy0, sy1 = K.sy1, sz0 = K.sz0, sz1 = K.sz1, zmax = K.z_max;
  {
    const double sy = sy0 + sy1 * fabs(st.z) / zmax, sz = sz0 + sz1 * fabs(st.z) / zmax;
    reset_cov(st, sy * sy, sz * sz, (double)K.cs0, (double)K.ct0, (double)K.cq0);
  }
  o.st = st;
  o.rlast = ro;
  o.n = 1;
  o.chi2 = 0.0;
  const double smax = K.smax, chi2max = K.chi2max;
  for (int r = ro - 1; r >= rmin; --r) {
    if (!transport(st, (double)K.row_x[r] - (double)K.row_x[r + 1], K.bd, smax)) break;
    const int32_t h = owned_at(S, hits, w, r);
    if (h < 0) continue;
    const double sy = sy0 + sy1 * fabs(st.z) / zmax, sz = sz0 + sz1 * fabs(st.z) / zmax;
    double ch = 0.0;
    kalman_update(st, (double)S.hy[h], (double)S.hz[h], sy * sy, sz * sz, chi2max, smax, false, &ch);
    o.chi2 = o.chi2 + ch;
    o.n += 1;
    o.st = st;
    o.rlast = r;
  }
}

// a7: refit of each selected tracklet over its owned hits, in double, three
// inward passes.  Pass 1 starts from the tracklet's inner (s, T, Q) with s
// carried to the outermost owned row along the circle (sin phi is linear in
// x); each later pass starts from the previous pass's result carried back
// the same way, so the Jacobians are evaluated along the fitted track.
// Output at the innermost fitted hit; the innermost hit's cluster is marked
// for the canonical ordering.
__global__ void __launch_bounds__(64) k_refit(Slot S, DevConst K, int g0, int ns) {
  const uint32_t total = S.flat_tk[ns];
  const uint32_t stride = gridDim.x * blockDim.x;
  unsigned nfit = 0;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    ++nfit;
    const int gi = flat_find_f(S.flat_tk, ns, t);
    const int g = g0 + gi;
    const uint32_t k = S.tk_base[g] + (t - S.flat_tk[gi]);
    const int32_t T = S.tk_tracklet[k];
    const int32_t* info = S.tl_info + (size_t)T * 4;
    const int32_t* hits = S.tl_hits + (size_t)T * kRows;
    const uint32_t w = S.tl_weight[T];
    int32_t* out = S.tk_info + (size_t)k * 4;
    out[0] = 0;
    int ro = -1, rmin = kRows;
    for (int r = info[1]; r <= info[2]; ++r)
      if (owned_at(S, hits, w, r) >= 0) {
        ro = r;
        rmin = r < rmin ? r : rmin;
      }
    if (ro < 0) continue;
    const float* sv = S.tl_state + (size_t)T * 5;
    const double smax = K.smax;
    PassOut o;
    bool ok = true;
    {
      const double sin_ = sv[2], tin = sv[3], qin = sv[4];
      const double s0 = sin_ + (K.bd * qin) * ((double)K.row_x[ro] - (double)K.row_x[info[1]]);
      if (!(fabs(s0) <= smax)) ok = false;
      else refit_pass(S, K, hits, w, ro, rmin, s0, tin, qin, o);
    }
    for (int pass = 1; ok && pass < 3; ++pass) {
      const double sin_ = o.st.s, tin = o.st.t, qin = o.st.q;
      const double s0 = sin_ + (K.bd * qin) * ((double)K.row_x[ro] - (double)K.row_x[o.rlast]);
      if (!(fabs(s0) <= smax)) ok = false;
      else refit_pass(S, K, hits, w, ro, o.rlast, s0, tin, qin, o);
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
    S.tmap[S.hid[hits[o.rlast]]] = (int32_t)k;
  }
  wave_add_u64(&S.stats[3], nfit);
}

}  // namespace tpc
