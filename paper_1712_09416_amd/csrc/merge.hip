// Cross-sector merger: a particle that crosses the boundary between two
// neighbouring sectors of one side, or the central membrane between the two
// sectors of one azimuth, leaves one track segment in each; the
// per-sector tracker fits them separately.  This step (the continuation of
// the per-sector tracking the paper's tracker chain performs next) joins
// such segments and refits the joined hit list across the sector frames.
//
//  M1 each track's state at its outermost hit: one outward Kalman pass over
//     its hits, seeded with its fitted parameters at the innermost hit and
//     the prior covariance (lane per track);
//  M2 pairs (A, B) of one event, B in a neighbouring sector of A's side or
//     in the sector across the membrane (same frame, no turn),
//     0 < B.row_in - A.row_out <= row_gap: A's outer state turned into B's
//     frame and transported to B's innermost row is compared with B's
//     fitted state, chi2 = d^T (C_A + C_B)^-1 d over the 5 parameters.
//     T and Q do not change under rotation or transport and d_i^2 / S_ii
//     never exceeds the chi2, so pairs failing the cut on them alone are
//     skipped before any transport.  Each A's best outer partner and each
//     B's best inner partner, ties to the smaller track position, from the
//     pairs evaluated in parallel (a pass for the smallest chi2s, a second
//     for the partners reaching them);
//  M3 a pair is linked if each is the other's best; links form chains;
//  M4 each chain of >= 2 segments is refitted inward over all its hits, in
//     passes (the first seeded with the outermost segment's outer state,
//     each later one with the previous result carried out to the outermost
//     hit), turning frames at the boundaries (lane per chain);
//  then the output: merged chains in place of their segments, canonical
//  order (event, innermost cluster ID) kept.
//
// Frame rotation: the frame of the neighbouring sector is turned by the
// angle a with cosine ca and sine sa; x' = x ca + y sa, y' = -x sa + y ca,
// sin phi' = sin(phi - a); the covariance is carried to the new x' along
// the track, C' = J C J^T with J(y', y) = ca - sa tan phi',
// J(z', y) = -sa T / cos phi', J(s', y) = -b Q sa, J(s', s) = cos phi' / cos phi
// (dense products in index order, so the result is reproducible bit for bit).
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

constexpr int kMaxChain = 16;    // segments of one chain (each holds >= 10 of the 159 rows)

__device__ __forceinline__ double xrow(const DevConst& K, int r) { return (double)K.row_x[r]; }

__device__ __forceinline__ void prior_d(const DevConst& K, Helix<double>& st, double zv) {
  const double sy = (double)K.sy0 + K.sy1zd * fabs(zv);
  const double sz = (double)K.sz0 + K.sz1zd * fabs(zv);
  reset_cov(st, sy * sy, sz * sz, (double)K.cs0, (double)K.ct0, (double)K.cq0);
}

// ungated update with a measured (y, z); returns its chi2
__device__ __forceinline__ double update_yz(const DevConst& K, Helix<double>& st, float y,
                                            float z) {
  const double sy = (double)K.sy0 + K.sy1zd * fabs(st.z);
  const double sz = (double)K.sz0 + K.sz1zd * fabs(st.z);
  double ch = 0.0;
  kalman_update(st, (double)y, (double)z, sy * sy, sz * sz, (double)K.chi2max, (double)K.smax,
                false, &ch);
  return ch;
}

__device__ __forceinline__ double update_hit(const Slot& S, const DevConst& K, Helix<double>& st,
                                             int64_t gid) {
  return update_yz(K, st, S.y[gid], S.z[gid]);
}

// a cluster's pad row and coordinates, loaded together
struct HitRec {
  int row;
  float y, z;
};
__device__ __forceinline__ HitRec load_hit(const Slot& S, int64_t gid) {
  HitRec h;
  h.row = S.row[gid];
  h.y = S.y[gid];
  h.z = S.z[gid];
  return h;
}

// kCov = false turns the parameters only (the same arithmetic for them).
template <bool kCov = true>
__device__ bool rotate_frame(Helix<double>& h, double& x, double ca, double sa, double b,
                             double smax) {
  const double y = h.y, s = h.s, tl = h.t, q = h.q;
  const double c = sqrt(1.0 - s * s);
  const double s1 = s * ca - c * sa;
  if (!(fabs(s1) <= smax)) return false;
  const double x1 = x * ca + y * sa;
  const double y1 = -x * sa + y * ca;
  if (!kCov) {
    h.y = y1;
    h.s = s1;
    x = x1;
    return true;
  }
  const double c1 = sqrt(1.0 - s1 * s1);
  double J[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) J[i][j] = i == j ? 1.0 : 0.0;
  J[0][0] = ca - sa * (s1 / c1);
  J[1][0] = -sa * tl / c1;
  J[2][0] = -(b * q) * sa;
  J[2][2] = c1 / c;
  double Cf[5][5];
#pragma unroll
  for (int i = 0, k = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++k) Cf[i][j] = Cf[j][i] = h.c[k];
  double A[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) a = a + J[i][k] * Cf[k][l];
      A[i][l] = a;
    }
#pragma unroll
  for (int i = 0, k = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++k) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < 5; ++l) v = v + A[i][l] * J[j][l];
      h.c[k] = v;
    }
  h.y = y1;
  h.s = s1;
  x = x1;
  return true;
}

// d^T S^-1 d by Cholesky (S packed like the covariance); false if S is not
// positive definite
__device__ bool chi2_5(const double* S, const double* d, double& chi2) {
  double L[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) L[i][j] = 0.0;
#pragma unroll
  for (int i = 0, k = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++k) L[i][j] = S[k];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double v = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) v = v - L[j][k] * L[j][k];
    if (!(v > 0.0)) return false;
    const double ljj = sqrt(v);
    L[j][j] = ljj;
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      double w = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) w = w - L[i][k] * L[j][k];
      L[i][j] = w / ljj;
    }
  }
  double yv[5];
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double w = d[i];
#pragma unroll
    for (int k = 0; k < i; ++k) w = w - L[i][k] * yv[k];
    yv[i] = w / L[i][i];
    sum = sum + yv[i] * yv[i];
  }
  chi2 = sum;
  return true;
}

// +1 if sector b (0..35 of one event) is the next one counter-clockwise of
// a on the same side, -1 the previous one, kMembrane if b is across the
// central membrane from a (same azimuth: the same frame), 0 otherwise
constexpr int kMembrane = 2;
__device__ __forceinline__ int neighbour(int a, int b) {
  const int ka = a % 18, kb = b % 18;
  if (a / 18 != b / 18) return ka == kb ? kMembrane : 0;
  if (kb == (ka + 1) % 18) return 1;
  if (ka == (kb + 1) % 18) return -1;
  return 0;
}

// the state in the frame of sector b from that of sector a, dir =
// neighbour(a, b) != 0 (no turn across the membrane)
template <bool kCov = true>
__device__ __forceinline__ bool turn_frame(Helix<double>& st, double& x, int dir, const DevConst& K,
                                           const MergeConst& C) {
  if (dir == kMembrane) return true;
  return rotate_frame<kCov>(st, x, C.ca, (double)dir * C.sa, K.bd, C.smax);
}

__device__ __forceinline__ const int32_t* track_hits(const Slot& S, const tpc_track& t) {
  return S.out_hits + S.ev_hit_off[t.event] + t.hit_off;
}

// M1
__global__ void __launch_bounds__(256) k_mg_outer(Slot S, DevConst K, MergeSlot M, MergeConst C) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const tpc_track t = S.out_tracks[a];
    const int64_t ev0 = S.ev_off[t.event];
    const int32_t* h = track_hits(S, t);
    Helix<double> st;
    st.y = t.par[0];
    st.z = t.par[1];
    st.s = t.par[2];
    st.t = t.par[3];
    st.q = t.par[4];
    prior_d(K, st, st.z);
    bool ok = true;
    // outward over rows row_in+1 .. row_out, updating with hits h[1..]
    // (one per row, rows ascending).  Every read of a step is issued at its
    // top and used after the transport: the next row's radius (the current
    // one carried in a register), the next hit's coordinates, the row of the
    // hit after it and the list entry after that (indices clamped to the
    // last hit).
    const int nlast = t.n_hits - 1;
    int k = 1;
    int64_t gn = ev0 + h[min(k, nlast)];
    int rn = k <= nlast ? (int)S.row[gn] : -1;
    int32_t h_after = h[min(k + 1, nlast)];
    double x_lo = xrow(K, t.row_in);
    float x_next = K.row_x[min(t.row_in + 1, kRows - 1)];
    for (int r = t.row_in + 1; r <= t.row_out; ++r) {
      const double x_hi = (double)x_next;
      x_next = K.row_x[min(r + 1, kRows - 1)];
      const float hy = S.y[gn], hz = S.z[gn];
      const int64_t g_after = ev0 + h_after;
      const int r_after = S.row[g_after];
      const int32_t h_after2 = h[min(k + 2, nlast)];
      if (!transport(st, x_hi - x_lo, K.bd, C.smax, K.kkd, K.m2d)) {
        ok = false;
        break;
      }
      x_lo = x_hi;
      if (r != rn) continue;
      update_yz(K, st, hy, hz);
      ++k;
      gn = g_after;
      rn = k <= nlast ? r_after : -1;
      h_after = h_after2;
    }
    M.ok[a] = ok ? 1 : 0;
    double* op = M.op + (size_t)a * 5;
    op[0] = st.y;
    op[1] = st.z;
    op[2] = st.s;
    op[3] = st.t;
    op[4] = st.q;
    double* oc = M.oc + (size_t)a * 15;
    for (int i = 0; i < 15; ++i) oc[i] = st.c[i];
  }
}

// track positions grouped by (event, sector, first row) and by (event,
// sector, last row); the order inside a group does not matter (ties are
// broken by track position)
__global__ void k_mg_count(Slot S, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const tpc_track& t = S.out_tracks[a];
    const int g = t.event * kSectorsPerEvent + t.sector;
    atomicAdd(&M.in_off[g * kRows + t.row_in], 1u);
    atomicAdd(&M.out_off[g * kRows + t.row_out], 1u);
  }
}

__global__ void k_mg_scatter(Slot S, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const tpc_track& t = S.out_tracks[a];
    const int g = t.event * kSectorsPerEvent + t.sector;
    const int gi = g * kRows + t.row_in, go = g * kRows + t.row_out;
    M.in_list[M.in_off[gi] + atomicAdd(&M.in_cur[gi], 1u)] = (int32_t)a;
    M.out_list[M.out_off[go] + atomicAdd(&M.out_cur[go], 1u)] = (int32_t)a;
  }
}

// M2 for the pair (A with outer state st0, B); false if incompatible
__device__ bool pair_chi2(const DevConst& K, const MergeConst& C, const tpc_track& A,
                          const double* op, const double* oc, const tpc_track& B, double& chi2) {
  const int dir = neighbour(A.sector, B.sector);
  if (dir == 0) return false;
  if (!(B.row_in > A.row_out && B.row_in - A.row_out <= C.row_gap)) return false;
  const double cut = C.chi2_max;
  const double dT = op[3] - B.par[3], dQ = op[4] - B.par[4];
  if (dT * dT > cut * (oc[9] + B.cov[9])) return false;
  if (dQ * dQ > cut * (oc[14] + B.cov[14])) return false;
  Helix<double> st;
  st.y = op[0];
  st.z = op[1];
  st.s = op[2];
  st.t = op[3];
  st.q = op[4];
  for (int i = 0; i < 15; ++i) st.c[i] = oc[i];
  double x = xrow(K, A.row_out);
  if (!turn_frame(st, x, dir, K, C)) return false;
  if (!transport_to_x(st, x, xrow(K, B.row_in), K.bd, C.smax, C.step_max, K.kkd, K.m2d)) return false;
  double d[5], Sm[15];
  d[0] = st.y - B.par[0];
  d[1] = st.z - B.par[1];
  d[2] = st.s - B.par[2];
  d[3] = st.t - B.par[3];
  d[4] = st.q - B.par[4];
  for (int i = 0; i < 15; ++i) Sm[i] = st.c[i] + B.cov[i];
  if (!chi2_5(Sm, d, chi2)) return false;
  return chi2 <= cut;
}

constexpr int kPairLanes = 16;   // lanes walking one track's candidates

// A pair (A, B) of the candidate walk: if compatible, its chi2 lowers A's
// and B's smallest chi2 (kFinal = false; the bit pattern of a non-negative
// double orders like its value) and the pair is listed for the second pass
// (in the block's segment of the list, up to pair_cap pairs each, slots
// taken a wave at a time); or, once those are
// known, it offers B as A's best outer partner and A as B's best inner
// partner where it reaches them (kFinal = true; the smaller track position
// wins a tie).  Called by every active lane of the wave together.
template <bool kFinal>
__device__ __forceinline__ void pair_eval(const Slot& S, const DevConst& K, const MergeSlot& M,
                                          const MergeConst& C, int32_t a, int32_t b) {
  double ch = 0.0;
  const bool ok = pair_chi2(K, C, S.out_tracks[a], M.op + (size_t)a * 5,
                            M.oc + (size_t)a * 15, S.out_tracks[b], ch);
  const unsigned long long key = (unsigned long long)__double_as_longlong(ch);
  if (kFinal) {
    if (ok && key == M.out_key[a]) atomicMin(&M.best_out[a], b);
    if (ok && key == M.in_key[b]) atomicMin(&M.best_in[b], a);
    return;
  }
  if (ok) {
    atomicMin(&M.out_key[a], key);
    atomicMin(&M.in_key[b], key);
  }
  const unsigned long long m = __ballot(ok);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  const uint32_t seg = blockIdx.x % kPairSegs;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(M.pair_n + seg * kPairPad, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  const uint32_t idx = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
  if (ok && idx < M.pair_cap) {
    const size_t at = (size_t)seg * M.pair_cap + idx;
    M.pair_a[at] = a;
    M.pair_b[at] = b;
    M.pair_key[at] = key;
  }
}

// The pair count of segment (lane of the wave), read once per lane; every
// lane of the wave must call (one segment per lane).
static_assert(kPairSegs == 64, "one pair-list segment per lane of a wave");
__device__ __forceinline__ uint32_t pair_seg_count(const MergeSlot& M) {
  return M.pair_n[(threadIdx.x & 63) * kPairPad];
}

// M2 + M3 over every pair the sector and row conditions admit: the tracks
// of A's event in the two neighbouring sectors of its side and in the
// sector across the membrane whose first row lies in (A.row_out,
// A.row_out + row_gap], three runs of in_list.  Each A is walked by
// kPairLanes lanes of a one-wave block; the pairs that pass the cuts on T
// and Q (a few in a hundred) queue in LDS, and the wave evaluates them 64
// at a time, so the frame turn, transport and chi2 run on full waves.  Run
// twice (kFinal false, then true); the results do not depend on the order
// in which pairs are met.
template <bool kFinal>
__global__ void __launch_bounds__(64) k_mg_pairs(Slot S, DevConst K, MergeSlot M, MergeConst C) {
  __shared__ int32_t qa[128], qb[128];
  constexpr int kPerWave = 64 / kPairLanes;
  // the second pass walks the candidates again only if the first pass's
  // pair list overflowed (k_mg_pair_best has the pairs otherwise)
  if (kFinal && !__any(pair_seg_count(M) > M.pair_cap)) return;
  const uint32_t ntk = S.out_count[0];
  const int lane = threadIdx.x;
  const int gl = lane % kPairLanes;
  const unsigned long long below = (1ull << lane) - 1ull;
  const double cut = C.chi2_max;
  int qn = 0;   // queued pairs (the same in every lane)
  for (uint32_t base = blockIdx.x * kPerWave; base < ntk; base += gridDim.x * kPerWave) {
    const uint32_t a = base + lane / kPairLanes;
    uint32_t s0 = 0, s1 = 0, s2 = 0;
    int c1 = 0, c2 = 0, c3 = 0;
    double oT = 0.0, oQ = 0.0, vT = 0.0, vQ = 0.0;
    if (a < ntk && M.ok[a]) {
      const tpc_track& A = S.out_tracks[a];
      const int r_lo = A.row_out + 1, r_hi = min(A.row_out + C.row_gap, kRows - 1);
      if (r_lo <= r_hi) {
        const int side = A.sector / 18, k = A.sector % 18;
        const int g = A.event * kSectorsPerEvent;
        const uint32_t* off = M.in_off;
        const int ga = (g + side * 18 + (k + 1) % 18) * kRows;
        const int gb = (g + side * 18 + (k + 17) % 18) * kRows;
        const int gc = (g + (1 - side) * 18 + k) * kRows;
        s0 = off[ga + r_lo];
        s1 = off[gb + r_lo];
        s2 = off[gc + r_lo];
        c1 = (int)(off[ga + r_hi + 1] - s0);
        c2 = c1 + (int)(off[gb + r_hi + 1] - s1);
        c3 = c2 + (int)(off[gc + r_hi + 1] - s2);
        oT = M.op[(size_t)a * 5 + 3];
        oQ = M.op[(size_t)a * 5 + 4];
        vT = M.oc[(size_t)a * 15 + 9];
        vQ = M.oc[(size_t)a * 15 + 14];
      }
    }
    for (int i0 = 0; __any(i0 < c3); i0 += kPairLanes) {
      const int i = i0 + gl;
      bool pass = false;
      int32_t b = 0;
      if (i < c3) {
        const uint32_t idx = i < c1 ? s0 + i : i < c2 ? s1 + (i - c1) : s2 + (i - c2);
        b = M.in_list[idx];
        const tpc_track& B = S.out_tracks[b];
        // the cuts of pair_chi2 on T and Q, in its arithmetic
        const double dT = oT - B.par[3], dQ = oQ - B.par[4];
        pass = !(dT * dT > cut * (vT + B.cov[9])) && !(dQ * dQ > cut * (vQ + B.cov[14]));
      }
      const unsigned long long m = __ballot(pass);
      if (pass) {
        const int pos = qn + __popcll(m & below);
        qa[pos] = (int32_t)a;
        qb[pos] = b;
      }
      qn += __popcll(m);
      if (qn >= 64) {
        __syncthreads();
        qn -= 64;
        pair_eval<kFinal>(S, K, M, C, qa[qn + lane], qb[qn + lane]);
        __syncthreads();
      }
    }
  }
  __syncthreads();
  if (lane < qn) pair_eval<kFinal>(S, K, M, C, qa[lane], qb[lane]);
}

template __global__ void k_mg_pairs<false>(Slot, DevConst, MergeSlot, MergeConst);
template __global__ void k_mg_pairs<true>(Slot, DevConst, MergeSlot, MergeConst);

// The second pass over the pairs the first one listed (when they all fit):
// a pair reaching A's (B's) smallest chi2 offers B (A) as its best partner.
__device__ __forceinline__ void offer_listed(const MergeSlot& M, size_t at) {
  const int32_t a = M.pair_a[at], b = M.pair_b[at];
  const unsigned long long key = M.pair_key[at];
  if (key == M.out_key[a]) atomicMin(&M.best_out[a], b);
  if (key == M.in_key[b]) atomicMin(&M.best_in[b], a);
}

// Waves are dealt to the segments (with 64 waves or more, the waves w = s
// mod 64 share segment s, lane by lane; with fewer, each wave takes whole
// segments), so every pair is read by one lane in one round.
__global__ void k_mg_pair_best(MergeSlot M) {
  const uint32_t cnt = pair_seg_count(M);
  if (__any(cnt > M.pair_cap)) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
  if (n_waves >= (uint32_t)kPairSegs) {
    const uint32_t s = wave % kPairSegs, per = n_waves / kPairSegs;
    const uint32_t n = __shfl(cnt, (int)s, 64);
    if (wave >= per * kPairSegs) return;
    for (uint32_t i = (wave / kPairSegs) * 64 + lane; i < n; i += per * 64)
      offer_listed(M, (size_t)s * M.pair_cap + i);
  } else {
    for (uint32_t s = wave; s < (uint32_t)kPairSegs; s += n_waves) {
      const uint32_t n = __shfl(cnt, (int)s, 64);
      for (uint32_t i = lane; i < n; i += 64) offer_listed(M, (size_t)s * M.pair_cap + i);
    }
  }
}

// a track without a compatible partner: -1 and chi2 0
__global__ void k_mg_final(Slot S, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const unsigned long long ki = M.in_key[a], ko = M.out_key[a];
    M.chi_in[a] = ki == ~0ull ? 0.0 : __longlong_as_double((long long)ki);
    if (ki == ~0ull) M.best_in[a] = -1;
    M.chi_out[a] = ko == ~0ull ? 0.0 : __longlong_as_double((long long)ko);
    if (ko == ~0ull) M.best_out[a] = -1;
  }
}

// M3: mutual best pairs (link_in filled with -1 before)
__global__ void k_mg_link(Slot S, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const int32_t b = M.best_out[a];
    const bool linked = b >= 0 && M.best_in[b] == (int32_t)a;
    M.link_out[a] = linked ? b : -1;
    if (linked) M.link_in[b] = (int32_t)a;
  }
}

// A chain's segments, innermost first: where each one's hit list starts in
// out_hits, its hit count, sector and first and last pad rows (the rows of
// its first and last hit).  Read once per chain; every pass walks these.
struct Chain {
  int n;
  int64_t ev0;                   // the event's first cluster
  int64_t hoff[kMaxChain];
  int32_t nh[kMaxChain];
  uint8_t sec[kMaxChain], rin[kMaxChain], rout[kMaxChain];
};

// One inward pass over the chain, seeded with (s0, t0, q0) at the
// outermost hit.  The pass is one flat loop of transport steps, each a row
// step inside a segment or one of the equal steps from a turned frame to
// the next segment's outermost hit, followed by an update where the step
// ends on a hit.  The lanes of a wave thus stay in step through segment
// changes, which fall at different rows for different chains (a loop over
// segments with a row loop inside would hold every lane of a wave in each
// segment until the longest one of the wave ends).
__device__ bool chain_pass(const Slot& S, const DevConst& K, const MergeConst& C, const Chain& ch,
                           double s0, double t0, double q0, Helix<double>& out, double& chi2,
                           int& n) {
  const int64_t ev0 = ch.ev0;
  int j = ch.n - 1;
  const int32_t* h = S.out_hits + ch.hoff[j];
  int k = ch.nh[j] - 1;
  int sector = ch.sec[j];
  int cur_row = ch.rout[j];
  Helix<double> st;
  {
    const int64_t go = ev0 + h[k];
    st.y = (double)S.y[go];
    st.z = (double)S.z[go];
  }
  st.s = s0;
  st.t = t0;
  st.q = q0;
  prior_d(K, st, st.z);
  chi2 = 0.0;
  n = 1;
  --k;
  // the row walk through the segment's hits h[k..0] below cur_row (one hit
  // per row, rows strictly descending).  Every read of a step is issued at
  // its top and used after the transport: the radius of the next row (the
  // current one carried in a register), the next hit's coordinates, the row
  // of the hit after it and the list entry after that (indices clamped to
  // h[0]).
  int r, rn, rstop;
  int64_t gn;
  int32_t h_after;
  double x_hi;
  float x_next;
  auto walk_from = [&](int row) {
    r = row - 1;
    x_hi = xrow(K, row);
    x_next = K.row_x[max(row - 1, 0)];
    const int kk = max(k, 0);
    gn = ev0 + h[kk];
    rn = k >= 0 ? (int)S.row[gn] : -1;
    h_after = h[max(k - 1, 0)];
    rstop = k >= 0 ? (int)ch.rin[j] : row;
  };
  walk_from(cur_row);
  // equal steps left to the outermost hit of the segment entered last
  int sub = 0;
  double dxb = 0.0;
  float by = 0.f, bz = 0.f;
  for (;;) {
    if (sub == 0 && r < rstop) {
      // segment done: turn into the next segment's frame and aim at its
      // outermost hit in steps of at most step_max
      if (j == 0) break;
      --j;
      const int dir = neighbour(sector, ch.sec[j]);
      sector = ch.sec[j];
      double x = xrow(K, cur_row);
      if (!turn_frame(st, x, dir, K, C)) return false;
      h = S.out_hits + ch.hoff[j];
      k = ch.nh[j] - 1;
      const int64_t g = ev0 + h[k];
      by = S.y[g];
      bz = S.z[g];
      const int rb = ch.rout[j];
      const double d = xrow(K, rb) - x;
      if (!(fabs(d) <= 1000.0)) return false;
      sub = max(1, (int)ceil(fabs(d) / C.step_max));
      dxb = d / (double)sub;
      // after the update at that hit, the walk continues below its row
      cur_row = rb;
      --k;
      walk_from(rb);
    }
    double dx;
    float hy, hz;
    bool upd;
    int64_t g_after = 0;
    int r_after = 0;
    int32_t h_after2 = 0;
    const bool walking = sub == 0;
    if (walking) {
      const double x_lo = (double)x_next;
      x_next = K.row_x[max(r - 1, 0)];
      hy = S.y[gn];
      hz = S.z[gn];
      g_after = ev0 + h_after;
      r_after = S.row[g_after];
      h_after2 = h[max(k - 2, 0)];
      dx = x_lo - x_hi;
      x_hi = x_lo;
      upd = r == rn;
    } else {
      dx = dxb;
      hy = by;
      hz = bz;
      upd = --sub == 0;
    }
    if (!transport(st, dx, K.bd, C.smax, K.kkd, K.m2d)) return false;
    if (upd) {
      chi2 = chi2 + update_yz(K, st, hy, hz);
      ++n;
    }
    if (walking) {
      if (upd) {
        cur_row = r;
        --k;
        gn = g_after;
        rn = k >= 0 ? r_after : -1;
        h_after = h_after2;
      }
      --r;
    }
  }
  out = st;
  return true;
}

// The inner result of a pass carried out to the outermost hit (the next
// pass resets the covariance, so only its parameters matter): through each
// segment to its last row in equal steps of at most step_max, turning
// frames between segments; one flat loop of steps, as the pass.
__device__ bool carry_out(const DevConst& K, const MergeConst& C, const Chain& ch,
                          Helix<double> st, double& s0, double& t0, double& q0) {
  double x = xrow(K, ch.rin[0]);
  int j = 0;
  double xo = xrow(K, ch.rout[0]);
  double d = xo - x;
  if (!(fabs(d) <= 1000.0)) return false;
  int sub = max(1, (int)ceil(fabs(d) / C.step_max));
  double dxs = d / (double)sub;
  for (;;) {
    if (!transport<double, false>(st, dxs, K.bd, C.smax, K.kkd, K.m2d)) return false;
    if (--sub > 0) continue;
    x = xo;
    if (++j == ch.n) break;
    const int dir = neighbour(ch.sec[j - 1], ch.sec[j]);
    if (!turn_frame<false>(st, x, dir, K, C)) return false;
    xo = xrow(K, ch.rout[j]);
    d = xo - x;
    if (!(fabs(d) <= 1000.0)) return false;
    sub = max(1, (int)ceil(fabs(d) / C.step_max));
    dxs = d / (double)sub;
  }
  s0 = st.s;
  t0 = st.t;
  q0 = st.q;
  return true;
}

// M4: refit of each chain (lane per chain head)
__global__ void __launch_bounds__(256) k_mg_chain(Slot S, DevConst K, MergeSlot M, MergeConst C) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    M.head_ok[a] = 0;
    if (M.link_in[a] >= 0 || M.link_out[a] < 0) continue;     // not the head of a chain
    Chain ch;
    ch.n = 0;
    bool fits = true;
    int32_t last = (int32_t)a;
    for (int32_t p = (int32_t)a; p >= 0; p = M.link_out[p]) {
      if (ch.n == kMaxChain) {
        fits = false;
        break;
      }
      const tpc_track& T = S.out_tracks[p];
      if (ch.n == 0) ch.ev0 = S.ev_off[T.event];
      ch.hoff[ch.n] = (int64_t)S.ev_hit_off[T.event] + T.hit_off;
      ch.nh[ch.n] = T.n_hits;
      ch.sec[ch.n] = (uint8_t)T.sector;
      ch.rin[ch.n] = (uint8_t)T.row_in;
      ch.rout[ch.n] = (uint8_t)T.row_out;
      ++ch.n;
      last = p;
    }
    bool good = fits && M.ok[last] != 0;
    double s0 = M.op[(size_t)last * 5 + 2], t0 = M.op[(size_t)last * 5 + 3],
           q0 = M.op[(size_t)last * 5 + 4];
    Helix<double> res;
    double chi2 = 0.0;
    int nh = 0;
    for (int pass = 0; pass < C.passes && good; ++pass) {
      if (pass > 0) good = carry_out(K, C, ch, res, s0, t0, q0);
      if (good) good = chain_pass(S, K, C, ch, s0, t0, q0, res, chi2, nh);
    }
    if (!good) continue;
    M.head_ok[a] = 1;
    M.nseg[a] = ch.n;
    M.nfit[a] = nh;
    double* par = M.par + (size_t)a * 5;
    par[0] = res.y;
    par[1] = res.z;
    par[2] = res.s;
    par[3] = res.t;
    par[4] = res.q;
    double* cov = M.cov + (size_t)a * 15;
    for (int i = 0; i < 15; ++i) cov[i] = res.c[i];
    M.chi2[a] = chi2;
  }
}

__device__ __forceinline__ int32_t chain_head(const MergeSlot& M, int32_t a) {
  int32_t h = a;
  while (M.link_in[h] >= 0) h = M.link_in[h];
  return h;
}

// output items: a refitted chain replaces its segments (at its head's
// position), every other track stays
__global__ void k_mg_emit(Slot S, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const int32_t h = chain_head(M, (int32_t)a);
    uint32_t e = 1, n = (uint32_t)S.out_tracks[a].n_hits;
    if (M.head_ok[h]) {
      e = h == (int32_t)a ? 1u : 0u;
      n = h == (int32_t)a ? (uint32_t)M.nfit[h] : 0u;
    }
    M.emit[a] = e;
    M.nh[a] = n;
  }
}

__global__ void k_mg_event_off(Slot S, MergeSlot M) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > S.n_events) return;
  const uint32_t k = S.ev_track_off[e];
  M.ev_track_off[e] = M.emit[k];
  M.ev_hit_off[e] = M.nh[k];
}

// n hit IDs from src to dst, eight loads in flight before their stores
__device__ __forceinline__ void copy_hits(int32_t* dst, const int32_t* src, int n) {
  for (int i0 = 0; i0 < n; i0 += 8) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = i0 + u < n ? src[i0 + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < n) dst[i0 + u] = v[u];
  }
}

__global__ void __launch_bounds__(256) k_mg_write(Slot S, DevConst K, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const int32_t h = chain_head(M, (int32_t)a);
    const bool merged = M.head_ok[h] != 0;
    const int32_t src = merged ? h : (int32_t)a;
    M.into[a] = (int32_t)M.emit[src];
    if (merged && h != (int32_t)a) continue;
    const uint32_t pos = M.emit[a];
    const uint32_t hpos = M.nh[a];
    tpc_track o = S.out_tracks[a];
    const int e = o.event;
    int32_t* dst = M.hits + hpos;
    if (merged) {
      int32_t last = h;
      int nh = 0;
      for (int32_t p = h; p >= 0; p = M.link_out[p]) {
        const tpc_track T = S.out_tracks[p];
        const int32_t* src_h = track_hits(S, T);
        copy_hits(dst + nh, src_h, T.n_hits);
        nh += T.n_hits;
        last = p;
      }
      o.n_hits = M.nfit[h];
      o.row_out = S.out_tracks[last].row_out;
      o.ndf = 2 * o.n_hits - 5;
      for (int i = 0; i < 5; ++i) o.par[i] = M.par[(size_t)h * 5 + i];
      for (int i = 0; i < 15; ++i) o.cov[i] = M.cov[(size_t)h * 15 + i];
      o.chi2 = M.chi2[h];
      M.out_nseg[pos] = M.nseg[h];
    } else {
      const int32_t* src_h = track_hits(S, o);
      copy_hits(dst, src_h, o.n_hits);
      M.out_nseg[pos] = 1;
    }
    o.hit_off = (int64_t)(hpos - M.ev_hit_off[e]);
    M.tracks[pos] = o;
  }
}

}  // namespace tpc
