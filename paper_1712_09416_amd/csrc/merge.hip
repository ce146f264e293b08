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
//     skipped before any transport.  Lane per A (best outer partner) and
//     lane per B (best inner partner), ties to the smaller track position;
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

// Candidates of a track among the tracks of the two neighbouring sectors
// of its side and of the sector across the membrane, in its event, those
// whose row (`off` indexes first rows, or last rows) lies in [r_lo, r_hi]:
// every pair the sector and row conditions of M2 admit.
template <class Fn>
__device__ __forceinline__ void for_neighbours(const uint32_t* off, const int32_t* list,
                                               const tpc_track& t, int r_lo, int r_hi, Fn&& fn) {
  r_lo = max(r_lo, 0);
  r_hi = min(r_hi, kRows - 1);
  if (r_lo > r_hi) return;
  const int side = t.sector / 18, k = t.sector % 18;
  const int nb[3] = {side * 18 + (k + 1) % 18, side * 18 + (k + 17) % 18, (1 - side) * 18 + k};
  for (int u = 0; u < 3; ++u) {
    const int g = t.event * kSectorsPerEvent + nb[u];
    const uint32_t i1 = off[g * kRows + r_hi + 1];
    for (uint32_t i = off[g * kRows + r_lo]; i < i1; ++i) fn(list[i]);
  }
}

// M2 + M3: best outer partner of each A.  Every compatible pair is
// evaluated here once: its chi2 also lowers B's smallest chi2 (the bit
// pattern of a non-negative double orders like its value), and the first
// kMgPairs pairs of A are kept for the pass that picks B's best A.
__global__ void __launch_bounds__(256) k_mg_best_out(Slot S, DevConst K, MergeSlot M,
                                                    MergeConst C) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    int32_t best = -1;
    double bc = 0.0;
    int32_t np = 0;
    if (M.ok[a]) {
      const tpc_track& A = S.out_tracks[a];
      const double* op = M.op + (size_t)a * 5;
      const double* oc = M.oc + (size_t)a * 15;
      for_neighbours(M.in_off, M.in_list, A, A.row_out + 1, A.row_out + C.row_gap, [&](int32_t b) {
        double ch;
        if (!pair_chi2(K, C, A, op, oc, S.out_tracks[b], ch)) return;
        atomicMin(&M.in_key[b], (unsigned long long)__double_as_longlong(ch));
        if (np < kMgPairs) {
          M.pr_b[(size_t)a * kMgPairs + np] = b;
          M.pr_chi[(size_t)a * kMgPairs + np] = ch;
        }
        ++np;
        if (best < 0 || ch < bc || (ch == bc && b < best)) {
          best = b;
          bc = ch;
        }
      });
    }
    M.best_out[a] = best;
    M.chi_out[a] = bc;
    M.pr_n[a] = np;
  }
}

// M2 + M3: best inner partner of each B: among the A whose pair reaches B's
// smallest chi2, the smaller track position (lane per A, over the pairs the
// previous pass kept; an A with more than kMgPairs pairs evaluates them again).
__global__ void __launch_bounds__(256) k_mg_best_in(Slot S, DevConst K, MergeSlot M,
                                                   MergeConst C) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const int32_t np = M.pr_n[a];
    if (np == 0) continue;
    auto offer = [&](int32_t b, double ch) {
      if ((unsigned long long)__double_as_longlong(ch) == M.in_key[b])
        atomicMin(&M.best_in[b], (int32_t)a);
    };
    if (np <= kMgPairs) {
      for (int k = 0; k < np; ++k)
        offer(M.pr_b[(size_t)a * kMgPairs + k], M.pr_chi[(size_t)a * kMgPairs + k]);
    } else {
      const tpc_track& A = S.out_tracks[a];
      const double* op = M.op + (size_t)a * 5;
      const double* oc = M.oc + (size_t)a * 15;
      for_neighbours(M.in_off, M.in_list, A, A.row_out + 1, A.row_out + C.row_gap, [&](int32_t b) {
        double ch;
        if (pair_chi2(K, C, A, op, oc, S.out_tracks[b], ch)) offer(b, ch);
      });
    }
  }
}

// B without a compatible A: -1 and chi2 0
__global__ void k_mg_in_final(Slot S, MergeSlot M) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < ntk; b += stride) {
    const unsigned long long key = M.in_key[b];
    const bool none = key == ~0ull;
    M.chi_in[b] = none ? 0.0 : __longlong_as_double((long long)key);
    if (none) M.best_in[b] = -1;
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

struct Chain {
  int n;
  int32_t pos[kMaxChain];
};

// one inward pass over the chain, seeded with (s0, t0, q0) at the
// outermost hit
__device__ bool chain_pass(const Slot& S, const DevConst& K, const MergeConst& C, const Chain& ch,
                           double s0, double t0, double q0, Helix<double>& out, double& chi2,
                           int& n) {
  const tpc_track L = S.out_tracks[ch.pos[ch.n - 1]];
  const int64_t evL = S.ev_off[L.event];
  const int32_t* hl = track_hits(S, L);
  const int64_t go = evL + hl[L.n_hits - 1];
  Helix<double> st;
  st.y = (double)S.y[go];
  st.z = (double)S.z[go];
  st.s = s0;
  st.t = t0;
  st.q = q0;
  prior_d(K, st, st.z);
  chi2 = 0.0;
  n = 1;
  int cur_row = S.row[go];
  for (int j = ch.n - 1; j >= 0; --j) {
    const tpc_track T = S.out_tracks[ch.pos[j]];
    const int64_t ev0 = S.ev_off[T.event];
    const int32_t* h = track_hits(S, T);
    int k = T.n_hits - 1;
    if (j == ch.n - 1) {
      --k;
    } else {
      // from the outer segment's frame to this one's
      const int dir = neighbour(S.out_tracks[ch.pos[j + 1]].sector, T.sector);
      double x = xrow(K, cur_row);
      if (!turn_frame(st, x, dir, K, C)) return false;
      const int64_t g = ev0 + h[k];
      const int r = S.row[g];
      if (!transport_to_x(st, x, xrow(K, r), K.bd, C.smax, C.step_max, K.kkd, K.m2d)) return false;
      chi2 = chi2 + update_hit(S, K, st, g);
      ++n;
      cur_row = r;
      --k;
    }
    // the segment's remaining hits h[k..0], inward (one hit per row, rows
    // strictly descending), as a walk of row steps.  Every read of a step
    // is issued at its top and used after the transport: the radius of the
    // next row (the current one carried in a register), the next hit's
    // coordinates, the row of the hit after it and the list entry after
    // that (indices clamped to h[0]).
    if (k >= 0) {
      int64_t gn = ev0 + h[k];
      int rn = S.row[gn];
      int32_t h_after = h[max(k - 1, 0)];
      const int rstop = S.row[ev0 + h[0]];
      double x_hi = xrow(K, cur_row);
      float x_next = K.row_x[max(cur_row - 1, 0)];
      for (int r = cur_row - 1; r >= rstop; --r) {
        const double x_lo = (double)x_next;
        x_next = K.row_x[max(r - 1, 0)];
        const float hy = S.y[gn], hz = S.z[gn];
        const int64_t g_after = ev0 + h_after;
        const int r_after = S.row[g_after];
        const int32_t h_after2 = h[max(k - 2, 0)];
        if (!transport(st, x_lo - x_hi, K.bd, C.smax, K.kkd, K.m2d)) return false;
        x_hi = x_lo;
        if (r != rn) continue;
        chi2 = chi2 + update_yz(K, st, hy, hz);
        ++n;
        cur_row = r;
        --k;
        gn = g_after;
        rn = k >= 0 ? r_after : -1;
        h_after = h_after2;
      }
    }
  }
  out = st;
  return true;
}

// the inner result of a pass carried out to the outermost hit (the next
// pass resets the covariance, so only its parameters matter)
__device__ bool carry_out(const Slot& S, const DevConst& K, const MergeConst& C, const Chain& ch,
                          Helix<double> st, double& s0, double& t0, double& q0) {
  const tpc_track F = S.out_tracks[ch.pos[0]];
  double x = xrow(K, S.row[S.ev_off[F.event] + track_hits(S, F)[0]]);
  for (int j = 0; j < ch.n; ++j) {
    const tpc_track T = S.out_tracks[ch.pos[j]];
    const double xo = xrow(K, S.row[S.ev_off[T.event] + track_hits(S, T)[T.n_hits - 1]]);
    if (!transport_to_x<false>(st, x, xo, K.bd, C.smax, C.step_max, K.kkd, K.m2d)) return false;
    x = xo;
    if (j + 1 < ch.n) {
      const int dir = neighbour(T.sector, S.out_tracks[ch.pos[j + 1]].sector);
      if (!turn_frame<false>(st, x, dir, K, C)) return false;
    }
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
    for (int32_t p = (int32_t)a; p >= 0; p = M.link_out[p]) {
      if (ch.n == kMaxChain) {
        fits = false;
        break;
      }
      ch.pos[ch.n++] = p;
    }
    const int32_t last = ch.pos[ch.n - 1];
    bool good = fits && M.ok[last] != 0;
    double s0 = M.op[(size_t)last * 5 + 2], t0 = M.op[(size_t)last * 5 + 3],
           q0 = M.op[(size_t)last * 5 + 4];
    Helix<double> res;
    double chi2 = 0.0;
    int nh = 0;
    for (int pass = 0; pass < C.passes && good; ++pass) {
      if (pass > 0) good = carry_out(S, K, C, ch, res, s0, t0, q0);
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
