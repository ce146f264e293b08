// Device-side building blocks of the TPC sector tracker for gfx950:
// slot layout, pad-row bin geometry and the Kalman-filter transport/update.
//
// Method (paper, Abstract and Section 2): track finding by a cellular
// automaton over pad-row hits followed by Kalman-filter track following.
// The paper gives no formulas; the arithmetic below is the project's written
// definition of those steps (helix in the local sector frame, state
// (y, z, sin phi, tan lambda, q/pT) at the pad-row x).  Float decisions are
// bit-reproducible against a CPU evaluation in the same operation order:
// every kernel is built with -ffp-contract=off and correctly rounded
// division and square root, and each expression below is evaluated left to
// right exactly as written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpcca.h"

namespace tpc {

constexpr int kRows = 159;
constexpr int kSectorsPerEvent = 36;
constexpr int kMaxRowHits = 4096;         // LDS sort capacity of one pad row
constexpr int kBinsPerHit = 2;            // a row has at most this many bins per hit
constexpr uint32_t kNoHit = 0xFFFFFFFFu;
constexpr int kRowBlocks = (kRows + 7) / 8;   // a tracklet's hit list in blocks of 8 rows
constexpr uint16_t kNoEntry = 0xFFFFu;        // hit-list entry of a row without hit

// ---------------------------------------------------------------------------
// constants handed to every kernel by value
// ---------------------------------------------------------------------------
struct DevConst {
  float row_x[kRows + 1];
  float tanh_half;
  float z_max;
  float sy0, sy1, sz0, sz1;
  // error model sigma(z) = sigma_0 + sigma_1 |z| / z_max with sigma_1 / z_max
  // formed once, in float and in double
  float sy1z, sz1z;
  double sy1zd, sz1zd;
  float b;          // curvature per unit q/pT, float
  double bd;        // same, double (refit)
  float nf_w, nf_mmax, chi2max, kwin, wmax, smax, cs0, ct0, cq0, medge, mz;
  int n_gap, n_min_tracklet, n_min_track, n_min_chain;
  float bin_target;  // clusters per grid bin aimed at
  float bin_min_edge;
  float kk, m2;             // scattering law k^2/X0 and mass^2 (0: no scattering), float
  double kkd, m2d;          // the same in double (refit, merger)
};

// per (sector, row) grid description
struct RowBins {
  float y0, z0, iby, ibz;   // lower edges and inverse bin sizes
  int32_t ny, nz;           // bins in y and z
  int32_t base;             // first entry of this row in bin_off
  int32_t first;            // the row's first sorted hit
};

// A sorted hit: coordinates, global cluster index, cleaned up-link (sorted
// index of the next hit of its chain, -1 none).  16 bytes: one load.
struct alignas(16) Hit {
  float y, z;
  uint32_t id;
  int32_t upc;
};

// One slot: a batch of events whose clusters are concatenated; sector g of
// the slot is sector g % 36 of event g / 36.
struct Slot {
  // input (caller device memory, or the slot's own copy)
  const uint8_t* sector;
  const uint8_t* row;
  const float* y;
  const float* z;
  int64_t* ev_off;          // [E+1] cluster offsets of the events
  int32_t n_events;
  int32_t n_sectors;        // 36 * n_events
  int64_t n;                // clusters
  // grid
  uint32_t* row_cnt;        // [SR]
  uint32_t* row_off;        // [SR+1] first sorted hit of each (sector, row)
  RowBins* bins;            // [SR]
  uint32_t* row_bin;        // [SR+1] bins per row, then the rows' first bin
  uint32_t* bin_off;        // [2 (n + SR) + SR + 1] per row: its bins' first hits, then the end
  uint32_t* rank;           // [n]
  Hit* hit;                 // [n] sorted by (sector, row, bin, id)
  uint32_t* hit_sr;         // [n] (sector, row) of each sorted hit (slot-wide index)
  // links (sorted-hit indices, -1 none); the cleaned up-link lives in hit[].upc
  int32_t* up;
  int32_t* dn;
  int32_t* dnc;
  // per-sector regions (used by per-sector launches; contiguous for a range)
  uint32_t* tl_base;        // [S+1] tracklet region of each sector
  uint32_t* tk_base;        // [S+1] track region of each sector
  uint32_t* row_nstart;     // [SR+1] start hits per row, then their offsets
  uint32_t* range_cnt;      // [16]: tracklets, tracks of the launched range; rows > 1024 hits
  uint32_t* big_rows;       // [n / 1024 + 1] (sector, row) of the rows over 1024 hits
  int32_t* start_hit;       // [tl capacity] sorted index of the start hit
  int32_t* start_sr;        // [tl capacity] (sector, row) of the start hit
  // tracklets
  uint16_t* tl_hits;        // [tl capacity / 64][kRowBlocks][64][8] per row: the hit's offset in its row, kNoEntry none
  int32_t* tl_info;         // [tl capacity][4]: n, row_in, row_out, valid
  uint32_t* tl_weight;      // [tl capacity]
  float* tl_state;          // [tl capacity][5] inner state (y, z, s, T, Q)
  uint32_t* tl_sel;         // [tl capacity+1] selected flag, then track positions
  uint32_t* weight;         // [n] per sorted hit, 0 = unowned
  // tracks (per-sector regions)
  int32_t* tk_tracklet;     // [tk capacity]
  int32_t* tk_own;          // [tk capacity][kRows] owned hits (sorted index), ascending row
  uint8_t* tk_own_row;      // [tk capacity][kRows] their rows
  int32_t* tk_nown;         // [tk capacity]
  int32_t* tk_info;         // [tk capacity][4]: ok, n, row_in, row_out
  double* tk_par;           // [tk capacity][5]
  double* tk_cov;           // [tk capacity][15]
  double* tk_chi2;          // [tk capacity]
  // canonical order
  int32_t* tmap;            // [n] per global cluster: temp track whose innermost hit it is
  uint32_t* scan_a;         // [n+1] scratch for the device scans
  uint32_t* scan_b;         // [block partials]
  uint32_t* out_count;      // [2]: tracks, hits of the slot
  uint32_t* out_ntk;        // [tk capacity+1] hit counts in canonical order, then offsets
  int32_t* out_order;       // [tk capacity] temporary track of each canonical position
  tpc_track* out_tracks;    // [tk capacity]
  int32_t* out_hits;        // [n]
  uint32_t* ev_track_off;   // [E+1]
  uint32_t* ev_hit_off;     // [E+1]
  uint32_t* err;            // [4]: invalid clusters, dense rows, overflow, spare
  unsigned long long* stats; // [8] work counters
  // capacities
  int64_t cap_n;
  int64_t cap_tl;
  int64_t cap_tk;
  int32_t cap_e;
};

// Row-indexed hit list of tracklet T: per row the hit's offset from its
// row's first sorted hit (rows hold at most 4096 hits), kNoEntry if none.
// Stored in tiles of 64 tracklets; inside a tile, blocks of 8 rows, and in
// a block the 8 entries of each tracklet together (16 bytes): a tracklet
// reads or writes 8 rows with one access, and the lanes of a wave
// (consecutive tracklets) touch one contiguous kilobyte per block.
struct TlList {
  uint16_t* p;              // this tracklet's entries of row block 0
  __device__ __forceinline__ uint4 load_block(int b) const {
    return *reinterpret_cast<const uint4*>(p + (size_t)b * 512);
  }
  __device__ __forceinline__ void store_block(int b, const uint4& v) const {
    *reinterpret_cast<uint4*>(p + (size_t)b * 512) = v;
  }
  __device__ __forceinline__ uint16_t at(int r) const { return p[(size_t)(r >> 3) * 512 + (r & 7)]; }
};
__device__ __forceinline__ TlList tl_list(const Slot& S, uint32_t T) {
  return TlList{S.tl_hits + ((size_t)(T >> 6) * kRowBlocks * 64 + (T & 63u)) * 8};
}
// entry k (0..7) of a block held in registers as two 64-bit halves (a
// shift and a two-way select: no indexed access, which the compiler would
// place in scratch memory)
__device__ __forceinline__ uint32_t block_get(const uint4& v, int k) {
  const uint64_t h = k < 4 ? ((uint64_t)v.y << 32 | v.x) : ((uint64_t)v.w << 32 | v.z);
  return (uint32_t)(h >> ((k & 3) * 16)) & 0xFFFFu;
}
__device__ __forceinline__ void block_set(uint4& v, int k, uint32_t e) {
  const bool lo = k < 4;
  uint64_t h = lo ? ((uint64_t)v.y << 32 | v.x) : ((uint64_t)v.w << 32 | v.z);
  const int sh = (k & 3) * 16;
  h = (h & ~(0xFFFFull << sh)) | ((uint64_t)(e & 0xFFFFu) << sh);
  const uint32_t a = (uint32_t)h, b = (uint32_t)(h >> 32);
  v.x = lo ? a : v.x;
  v.y = lo ? b : v.y;
  v.z = lo ? v.z : a;
  v.w = lo ? v.w : b;
}
__device__ __forceinline__ uint4 block_empty() {
  return make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
}
// sorted-hit index of an entry of the row whose first hit is `first`
__device__ __forceinline__ int32_t entry_hit(uint32_t e, uint32_t first) {
  return e == kNoEntry ? -1 : (int32_t)(first + e);
}

// ---------------------------------------------------------------------------
// pad-row bins: monotone in y and z, identical in every kernel
// ---------------------------------------------------------------------------
// (a NaN coordinate maps to bin 0: every index stays inside the row)
__device__ __forceinline__ int bin_y(const RowBins& b, float y) {
  const float f = (y - b.y0) * b.iby;
  return f >= 0.0f ? (int)fminf(f, (float)(b.ny - 1)) : 0;
}
__device__ __forceinline__ int bin_z(const RowBins& b, float z) {
  const float f = (z - b.z0) * b.ibz;
  return f >= 0.0f ? (int)fminf(f, (float)(b.nz - 1)) : 0;
}

// Hits of one row that can lie inside [yc - wy, yc + wy] x [zc - wz, zc + wz]:
// every bin the window touches, plus a small margin so rounding cannot hide
// a hit; the caller applies the exact window test.  `bo` is the row's bin
// offset table (sorted-hit positions).  The bin ranges of up to four z rows
// are read together, then their hits four at a time across the ranges, so
// a query waits for a few memory round trips rather than one per hit or
// per range.  fn(p, hit) runs in ascending p within a range, ranges in
// ascending z.  WB: hit records read per round trip (a tuning knob).
template <int WB, class Fn>
__device__ __forceinline__ void for_window_hits(const RowBins& b, const uint32_t* bo, const Hit* hit,
                                                float yc, float zc, float wy, float wz, Fn&& fn) {
  const float eps = 1e-3f;
  const int iy0 = bin_y(b, yc - wy - eps), iy1 = bin_y(b, yc + wy + eps);
  const int iz0 = bin_z(b, zc - wz - eps), iz1 = bin_z(b, zc + wz + eps);
  for (int izb = iz0; izb <= iz1; izb += 4) {
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = 0u;
      hi[k] = 0u;
      if (izb + k <= iz1) {
        const int first = (izb + k) * b.ny;
        lo[k] = bo[first + iy0];
        hi[k] = bo[first + iy1 + 1];
      }
    }
    // the four ranges as one sequence (same order), read WB hits at a
    // time whichever ranges they fall in
    const uint32_t c0 = hi[0] - lo[0];
    const uint32_t c1 = c0 + (hi[1] - lo[1]);
    const uint32_t c2 = c1 + (hi[2] - lo[2]);
    const uint32_t c3 = c2 + (hi[3] - lo[3]);
    for (uint32_t f = 0; f < c3; f += WB) {
      uint32_t p[WB];
      Hit x[WB];
#pragma unroll
      for (int u = 0; u < WB; ++u) {
        const uint32_t q = f + u;
        p[u] = q < c0 ? lo[0] + q : q < c1 ? lo[1] + (q - c0) : q < c2 ? lo[2] + (q - c1) : lo[3] + (q - c2);
        if (q < c3) x[u] = hit[p[u]];
      }
#pragma unroll
      for (int u = 0; u < WB; ++u)
        if (f + u < c3) fn(p[u], x[u]);
    }
  }
}

__device__ __forceinline__ float sigma_y(const DevConst& k, float z) {
  return k.sy0 + k.sy1z * fabsf(z);
}
__device__ __forceinline__ float sigma_z(const DevConst& k, float z) {
  return k.sz0 + k.sz1z * fabsf(z);
}

// ---------------------------------------------------------------------------
// Kalman filter on the helix state.  Template over float (tracklet phases,
// which take decisions) and double (the output refit).
// Covariance packed as the lower triangle of (y, z, s, T, Q):
//   0:yy 1:zy 2:zz 3:sy 4:sz 5:ss 6:Ty 7:Tz 8:Ts 9:TT 10:Qy 11:Qz 12:Qs 13:QT 14:QQ
// ---------------------------------------------------------------------------
// sum over the wave, then one atomic per wave (all 64 lanes must call)
__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, unsigned long long v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

template <class F>
struct Helix {
  F y, z, s, t, q;
  F c[15];
};

template <class F> __device__ __forceinline__ F fabs_(F v);
template <> __device__ __forceinline__ float fabs_(float v) { return fabsf(v); }
template <> __device__ __forceinline__ double fabs_(double v) { return fabs(v); }
template <class F> __device__ __forceinline__ F sqrt_(F v);
template <> __device__ __forceinline__ float sqrt_(float v) { return sqrtf(v); }
template <> __device__ __forceinline__ double sqrt_(double v) { return sqrt(v); }
// a*b + c rounded once.  Every sum of products of the filter is a chain of
// these in a fixed order (the CPU checker uses the same chains), so results
// stay bit-identical with contraction switched off for everything else.
template <class F> __device__ __forceinline__ F fma_(F a, F b, F c);
template <> __device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }

// Move the state by dx along the circle of curvature b*q.  sin(phi) grows
// linearly with x; y advances by dx times the tangent of the mid-angle
// (N/D below); z advances by T times the arc, the arc being the chord
// times asin(u)/u = 1 + u^2/6 + 3u^4/40 (u = half chord * curvature).
// Returns false, leaving the state untouched, if |sin phi| would pass smax.
// kCov = false moves the parameters only (the same arithmetic for them),
// for callers that discard the covariance.
template <class F, bool kCov = true>
__device__ __forceinline__ bool transport(Helix<F>& h, F dx, F b, F smax, F kk = F(0),
                                          F m2 = F(0)) {
  const F one = F(1), half = F(0.5), two = F(2);
  const F bq = b * h.q;
  const F s1 = fma_(bq, dx, h.s);
  if (!(fabs_(s1) <= smax)) return false;
  const F s0 = h.s;
  const F c0 = sqrt_(fma_(-s0, s0, one));
  const F c1 = sqrt_(fma_(-s1, s1, one));
  const F N = s0 + s1;
  const F D = c0 + c1;
  // one division: the reciprocals of D, c0 and c1 are products with
  // 1/(c0 c1 D)
  const F c01 = c0 * c1;
  const F inv = one / (c01 * D);
  const F iD = c01 * inv;
  const F ic0 = (c1 * D) * inv;
  const F ic1 = (c0 * D) * inv;
  const F tmid = N * iD;
  const F chord = fabs_(dx) * sqrt_(fma_(tmid, tmid, one));
  const F u = half * bq * chord;
  const F u2 = u * u;
  F arc = chord * fma_(u2, fma_(u2, F(3) / F(40), one / F(6)), one);
  if (dx < F(0)) arc = -arc;

  // Jacobian; dz/dQ to leading order, 2 T b N dx^2 / D^3 (the mid-angle
  // cosine taken as D/2)
  const F iD2 = iD * iD;
  const F r0 = s0 * ic0;
  const F r1 = s1 * ic1;
  const F dy_ds = dx * fma_(N, r0 + r1, two * D) * iD2;
  const F dy_dq = b * dx * dx * fma_(N, r1, D) * iD2;
  const F dz_ds = h.t * dx * N * (ic0 * ic1 * iD);
  const F dz_dt = arc;
  const F dz_dq = two * h.t * b * N * dx * dx * (iD2 * iD);
  const F ds_dq = b * dx;

  h.y = fma_(dx, tmid, h.y);
  h.z = fma_(h.t, arc, h.z);
  h.s = s1;
  if (!kCov) return true;

  F* c = h.c;
  const F yy = c[0], zy = c[1], zz = c[2], sy = c[3], sz = c[4], ss = c[5];
  const F ty = c[6], tz = c[7], ts = c[8], tt = c[9];
  const F qy = c[10], qz = c[11], qs = c[12], qt = c[13], qq = c[14];

  // rows y, z, s of J*C (the columns that the product below reads)
  const F jy_y = fma_(dy_dq, qy, fma_(dy_ds, sy, yy));
  const F jy_s = fma_(dy_dq, qs, fma_(dy_ds, ss, sy));
  const F jy_q = fma_(dy_dq, qq, fma_(dy_ds, qs, qy));
  const F jz_y = fma_(dz_dq, qy, fma_(dz_dt, ty, fma_(dz_ds, sy, zy)));
  const F jz_z = fma_(dz_dq, qz, fma_(dz_dt, tz, fma_(dz_ds, sz, zz)));
  const F jz_s = fma_(dz_dq, qs, fma_(dz_dt, ts, fma_(dz_ds, ss, sz)));
  const F jz_t = fma_(dz_dq, qt, fma_(dz_dt, tt, fma_(dz_ds, ts, tz)));
  const F jz_q = fma_(dz_dq, qq, fma_(dz_dt, qt, fma_(dz_ds, qs, qz)));
  const F js_y = fma_(ds_dq, qy, sy);
  const F js_z = fma_(ds_dq, qz, sz);
  const F js_s = fma_(ds_dq, qs, ss);
  const F js_t = fma_(ds_dq, qt, ts);
  const F js_q = fma_(ds_dq, qq, qs);

  // (J*C)*J^T, lower triangle; TT, QT, QQ unchanged
  c[0] = fma_(dy_dq, jy_q, fma_(dy_ds, jy_s, jy_y));
  c[1] = fma_(dy_dq, jz_q, fma_(dy_ds, jz_s, jz_y));
  c[2] = fma_(dz_dq, jz_q, fma_(dz_dt, jz_t, fma_(dz_ds, jz_s, jz_z)));
  c[3] = fma_(dy_dq, js_q, fma_(dy_ds, js_s, js_y));
  c[4] = fma_(dz_dq, js_q, fma_(dz_dt, js_t, fma_(dz_ds, js_s, js_z)));
  c[5] = fma_(ds_dq, js_q, js_s);
  c[6] = fma_(dy_dq, qt, fma_(dy_ds, ts, ty));
  c[7] = fma_(dz_dq, qt, fma_(dz_dt, tt, fma_(dz_ds, ts, tz)));
  c[8] = fma_(ds_dq, qt, ts);
  c[10] = fma_(dy_dq, qq, fma_(dy_ds, qs, qy));
  c[11] = fma_(dz_dq, qq, fma_(dz_dt, qt, fma_(dz_ds, qs, qz)));
  c[12] = fma_(ds_dq, qq, qs);

  // multiple scattering at the end of the step (kk = k^2/X0 > 0):
  // theta0^2 = kk L (a + m^2 a^2), a = Q^2/(1+T^2), L = |arc| sqrt(1+T^2);
  // var(phi) = theta0^2 (1+T^2), var(lambda) = theta0^2, dQ = Q T dlambda,
  // dT = (1+T^2) dlambda
  if (kk > F(0)) {
    const F t2 = fma_(h.t, h.t, one);
    const F L = fabs_(arc) * sqrt_(t2);
    const F a = (h.q * h.q) / t2;
    const F th2 = kk * L * fma_(m2, a * a, a);
    c[5] = fma_(fma_(-s1, s1, one), th2 * t2, c[5]);
    c[9] = fma_(th2, t2 * t2, c[9]);
    c[13] = fma_(th2, h.q * h.t * t2, c[13]);
    c[14] = fma_(th2, h.q * h.q * (h.t * h.t), c[14]);
  }
  return true;
}

// Inverse of the 2x2 residual covariance S = C_(y,z) + diag(vy, vz).
template <class F>
struct Resid {
  F w00, w01, w11, s00, s11;
};

template <class F>
__device__ __forceinline__ Resid<F> resid_weights(const Helix<F>& h, F vy, F vz) {
  Resid<F> r;
  const F s00 = h.c[0] + vy;
  const F s01 = h.c[1];
  const F s11 = h.c[2] + vz;
  const F det = fma_(s00, s11, -(s01 * s01));
  const F inv = F(1) / det;
  r.w00 = s11 * inv;
  r.w01 = -s01 * inv;
  r.w11 = s00 * inv;
  r.s00 = s00;
  r.s11 = s11;
  return r;
}

template <class F>
__device__ __forceinline__ F chi2_of(const Resid<F>& w, F ry, F rz) {
  return fma_(ry, fma_(w.w00, ry, w.w01 * rz), rz * fma_(w.w01, ry, w.w11 * rz));
}

// Kalman update with the measurement (my, mz).  gated: refuse (state
// untouched) when chi2 > chi2max, a variance would not stay positive or
// |sin phi| would reach smax.
template <class F>
__device__ __forceinline__ bool kalman_update(Helix<F>& h, F my, F mz, F vy, F vz, F chi2max,
                                              F smax, bool gated, F* chi2_out) {
  const Resid<F> w = resid_weights(h, vy, vz);
  const F ry = my - h.y;
  const F rz = mz - h.z;
  const F chi2 = chi2_of(w, ry, rz);
  *chi2_out = chi2;
  if (gated && !(chi2 <= chi2max)) return false;
  const F* c = h.c;
  // covariance column of each state entry with y and with z
  const F cy[5] = {c[0], c[1], c[3], c[6], c[10]};
  const F cz[5] = {c[1], c[2], c[4], c[7], c[11]};
  F ky[5], kz[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    ky[i] = fma_(cy[i], w.w00, cz[i] * w.w01);
    kz[i] = fma_(cy[i], w.w01, cz[i] * w.w11);
  }
  Helix<F> o;
  o.y = fma_(ky[0], ry, fma_(kz[0], rz, h.y));
  o.z = fma_(ky[1], ry, fma_(kz[1], rz, h.z));
  o.s = fma_(ky[2], ry, fma_(kz[2], rz, h.s));
  o.t = fma_(ky[3], ry, fma_(kz[3], rz, h.t));
  o.q = fma_(ky[4], ry, fma_(kz[4], rz, h.q));
  int k = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j, ++k) o.c[k] = fma_(-ky[i], cy[j], fma_(-kz[i], cz[j], c[k]));
  }
  if (gated) {
    if (!(o.c[0] > F(0) && o.c[2] > F(0) && o.c[5] > F(0) && o.c[9] > F(0) && o.c[14] > F(0) &&
          fabs_(o.s) < smax))
      return false;
  }
  h = o;
  return true;
}

// Prior covariance: measurement variances in y and z at the hit, wide
// diagonal for the angles and the curvature.
template <class F>
__device__ __forceinline__ void reset_cov(Helix<F>& h, F vy, F vz, F cs0, F ct0, F cq0) {
#pragma unroll
  for (int i = 0; i < 15; ++i) h.c[i] = F(0);
  h.c[0] = vy;
  h.c[2] = vz;
  h.c[5] = cs0;
  h.c[9] = ct0;
  h.c[14] = cq0;
}

// From x to xt in equal steps of at most step_max (refused beyond 1000 cm,
// longer than any path in the chamber, which also bounds the step count).
template <bool kCov = true>
__device__ __forceinline__ bool transport_to_x(Helix<double>& h, double x, double xt, double b,
                                               double smax, double step_max, double kk = 0.0,
                                               double m2 = 0.0) {
  const double d = xt - x;
  if (!(fabs(d) <= 1000.0)) return false;
  const int n = max(1, (int)ceil(fabs(d) / step_max));
  const double dx = d / (double)n;
  for (int i = 0; i < n; ++i)
    if (!transport<double, kCov>(h, dx, b, smax, kk, m2)) return false;
  return true;
}

}  // namespace tpc
