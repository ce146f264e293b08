// a5: tracklet construction (paper, Abstract: Kalman-filter track
// following).  One lane per start hit, float arithmetic; the lane's state
// and the decisions of its current block of 8 rows live in registers, its
// hit list in global memory (row-indexed, a block written when the lane
// leaves it).
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

// Stop rules after a transport to the row at radius xr: left the sector
// sideways, crossed the membrane, or left the drift volume.
__device__ __forceinline__ bool inside(const DevConst& K, const Helix<float>& h, float xr, bool side_c) {
  if (!(fabsf(h.y) <= xr * K.tanh_half + K.medge)) return false;
  if (!(fabsf(h.z) <= K.z_max + K.mz)) return false;
  if (side_c ? (h.z > K.mz) : (h.z < -K.mz)) return false;
  return true;
}

// Best hit of row sr for the predicted state: inside
// |r_y| <= min(k sqrt(S_yy), w_max), |r_z| <= min(k sqrt(S_zz), w_max),
// smallest chi2, ties to the smaller cluster ID.  -1 if none; the hit record
// is returned in `out`.  WB: hit records read per round trip.
template <int WB>
__device__ __forceinline__ int32_t search_row(const Slot& S, const DevConst& K, const RowBins& rb,
                                              const Helix<float>& h, float vy, float vz,
                                              unsigned& examined, Hit& out) {
  const Resid<float> w = resid_weights(h, vy, vz);
  float wy = K.kwin * sqrtf(w.s00);
  if (wy > K.wmax) wy = K.wmax;
  float wz = K.kwin * sqrtf(w.s11);
  if (wz > K.wmax) wz = K.wmax;
  const float yc = h.y, zc = h.z;
  int32_t best = -1;
  float bchi = 0.0f;
  uint32_t bid = 0;
  for_window_hits<WB>(rb, S.bin_off + rb.base, S.hit, yc, zc, wy, wz, [&](uint32_t p, const Hit& x) {
    const float ry = x.y - yc, rz = x.z - zc;
    if (!(fabsf(ry) <= wy && fabsf(rz) <= wz)) return;
    ++examined;                 // hits inside the window (independent of the binning)
    const float ch = chi2_of(w, ry, rz);
    const uint32_t id = x.id;
    if (best < 0 || ch < bchi || (ch == bchi && id < bid)) {
      best = (int32_t)p;
      bchi = ch;
      bid = id;
      out = x;
    }
  });
  return best;
}

__device__ __forceinline__ bool try_hit(const DevConst& K, Helix<float>& h, const Hit& x, float vy,
                                        float vz, unsigned& tries) {
  float ch;
  ++tries;
  return kalman_update(h, x.y, x.z, vy, vz, K.chi2max, K.smax, true, &ch);
}

// For each start hit h0 (row r0) with cleaned up-link h1:
//  seed  (y, z) = h0, sin phi and tan lambda from h0 -> h1, q/pT = 0, prior
//        covariance (hit variances, wide angles and curvature);
//  out   rows r0+1..158: transport, stop rules; follow the cleaned chain while
//        its hits pass the gate, then (for good) take the best-chi2 hit of
//        each row's window; stop after n_gap consecutive rows without hit;
//  in    restart at the outermost hit with the prior covariance and the
//        outward (s, T, Q); rows down to 0: re-confirm the outward hit, else
//        search; same gap rule.  The inward hits form the tracklet.
template <int WB>
__global__ void __launch_bounds__(256) k_tracklets(Slot S, DevConst K, int g0) {
  // Tracklets are ordered by (sector, row): give each XCD (blocks are
  // dispatched round-robin over the 8 XCDs) one contiguous chunk, so the
  // hits a chunk's lanes read stay in that XCD's L2.
  const uint32_t total = S.range_cnt[0];
  const uint32_t base = S.tl_base[g0];
  constexpr uint32_t kXcd = 8;
  const uint32_t xcd = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
  const uint32_t nbx = (gridDim.x - xcd + kXcd - 1) / kXcd;
  const uint32_t chunk = (total + kXcd - 1) / kXcd;
  const uint32_t c0 = xcd * chunk;
  const uint32_t c1 = min(total, c0 + chunk);
  unsigned visits = 0, examined = 0, done = 0, tl_hits = 0, tries = 0;
  for (uint32_t t = c0 + j * blockDim.x + threadIdx.x; t < c1; t += nbx * blockDim.x) {
    ++done;
    const uint32_t T = base + t;
    const int sr0 = S.start_sr[T];
    const int g = sr0 / kRows;
    const int r0 = sr0 - g * kRows;
    const bool side_c = (g % kSectorsPerEvent) >= kSectorsPerEvent / 2;
    const int64_t ev0 = S.ev_off[g / kSectorsPerEvent];
    const int32_t p0 = S.start_hit[T];
    const Hit x0 = S.hit[p0];
    const Hit x1 = S.hit[x0.upc];
    const TlList hits = tl_list(S, T);
    const uint32_t first0 = S.row_off[sr0];

    // radii of the start row and the next one (r0 <= 157: a start hit has
    // an up link)
    const float x_r0 = K.row_x[r0], x_r1 = K.row_x[r0 + 1];
    Helix<float> st;
    {
      const float dx = x_r1 - x_r0;
      const float dy = x1.y - x0.y;
      const float dz = x1.z - x0.z;
      const float L = sqrtf(dx * dx + dy * dy);
      st.y = x0.y;
      st.z = x0.z;
      st.s = dy / L;
      st.t = dz / L;
      st.q = 0.0f;
      const float sy = sigma_y(K, st.z), sz = sigma_z(K, st.z);
      reset_cov(st, sy * sy, sz * sz, K.cs0, K.ct0, K.cq0);
    }
    // the hit list's block of the current row, in registers
    int cb = r0 >> 3;
    uint4 blk = block_empty();
    block_set(blk, r0 & 7, (uint32_t)p0 - first0);

    // outward
    Helix<float> last = st;
    int rout = r0;
    float x_rout = x_r0;
    int32_t next = x0.upc;     // cleaned chain link of the last accepted hit
    int32_t p_out = p0;        // the outermost accepted hit
    bool chain = true;
    int miss = 0;
    // row radii: the current one carried in a register, the next one read
    // a step ahead (index clamped to the last row); both start from values
    // the seed has used, so no read before the loop is waited for inside it
    float x_prev = x_r0;
    float x_ahead = x_r1;
    for (int r = r0 + 1; r < kRows; ++r) {
      ++visits;
      const float xr = x_ahead;
      x_ahead = K.row_x[min(r + 1, kRows - 1)];
      // reads independent of the state, issued before the transport: the
      // row's bin range and the hit the chain link points to
      const RowBins rb = S.bins[g * kRows + r];
      Hit xnext;
      if (chain && next >= 0) xnext = S.hit[next];
      if ((r & 7) == 0) {          // into the next block of rows
        hits.store_block(cb, blk);
        cb = r >> 3;
        blk = block_empty();
      }
      if (!transport(st, xr - x_prev, K.b, K.smax, K.kk, K.m2)) break;
      x_prev = xr;
      if (!inside(K, st, xr, side_c)) break;
      const float sy = sigma_y(K, st.z), sz = sigma_z(K, st.z);
      const float vy = sy * sy, vz = sz * sz;
      int32_t got = -1;
      Hit xg;
      if (chain) {
        if (next >= 0) {
          xg = xnext;
          if (try_hit(K, st, xg, vy, vz, tries)) got = next;
        }
        if (got < 0) chain = false;
      }
      if (got < 0) {
        const int32_t bh = search_row<WB>(S, K, rb, st, vy, vz, examined, xg);
        if (bh >= 0 && try_hit(K, st, xg, vy, vz, tries)) got = bh;
      }
      if (got >= 0) {
        block_set(blk, r & 7, (uint32_t)got - (uint32_t)rb.first);
        next = xg.upc;
        p_out = got;
        miss = 0;
        last = st;
        rout = r;
        x_rout = xr;
      } else if (++miss >= K.n_gap) {
        break;
      }
    }
    hits.store_block(cb, blk);

    // inward, covariance reset at the outermost hit
    const Hit xo = S.hit[p_out];
    st = last;
    st.y = xo.y;
    st.z = xo.z;
    {
      const float sy = sigma_y(K, st.z), sz = sigma_z(K, st.z);
      reset_cov(st, sy * sy, sz * sz, K.cs0, K.ct0, K.cq0);
    }
    int n = 1;
    int rin = rout;
    last = st;
    miss = 0;
    // the blocks of the current row and of the one below, in registers (the
    // outward decisions, rewritten as the inward ones are taken; a block is
    // stored back only if an entry changed); the outward hit of the next
    // row down loaded one step ahead, the first hit of the row below it two
    // steps ahead
    const int gr = g * kRows;
    cb = (rout - 1) >> 3;
    blk = hits.load_block(cb);
    uint4 blk_dn = cb > 0 ? hits.load_block(cb - 1) : block_empty();
    bool dirty = false;
    const uint32_t f_a = rout - 1 >= r0 ? (uint32_t)S.row_off[gr + rout - 1] : 0u;
    uint32_t f_next = rout - 2 >= r0 ? (uint32_t)S.row_off[gr + rout - 2] : 0u;
    int32_t uh_next = rout - 1 >= r0 ? entry_hit(block_get(blk, (rout - 1) & 7), f_a) : -1;
    Hit xu_next;
    if (uh_next >= 0) xu_next = S.hit[uh_next];
    x_prev = x_rout;
    x_ahead = K.row_x[max(rout - 1, 0)];
    // wait for these reads here, once: a read still in flight at the loop's
    // entry would make the compiler wait inside every step
    asm volatile("" : "+v"(x_ahead), "+v"(f_next));
    for (int r = rout - 1; r >= 0; --r) {
      ++visits;
      const float xr = x_ahead;
      x_ahead = K.row_x[max(r - 1, 0)];
      const RowBins rb = S.bins[gr + r];
      const int32_t uh = uh_next;
      const Hit xu = xu_next;
      // row r-1: its outward entry (this block or the one below) and the
      // first hit of its row, read a step ago
      uh_next = -1;
      if (r - 1 >= r0)
        uh_next = entry_hit(block_get((r & 7) == 0 ? blk_dn : blk, (r - 1) & 7), f_next);
      if (uh_next >= 0) xu_next = S.hit[uh_next];
      if (r - 2 >= r0) f_next = (uint32_t)S.row_off[gr + r - 2];
      if (!transport(st, xr - x_prev, K.b, K.smax, K.kk, K.m2)) break;
      x_prev = xr;
      if (!inside(K, st, xr, side_c)) break;
      const float sy = sigma_y(K, st.z), sz = sigma_z(K, st.z);
      const float vy = sy * sy, vz = sz * sz;
      int32_t got = -1;
      if (uh >= 0 && try_hit(K, st, xu, vy, vz, tries)) got = uh;
      if (got < 0) {
        Hit xs;
        const int32_t bh = search_row<WB>(S, K, rb, st, vy, vz, examined, xs);
        if (bh >= 0 && try_hit(K, st, xs, vy, vz, tries)) got = bh;
      }
      {
        const uint32_t e = got >= 0 ? (uint32_t)got - (uint32_t)rb.first : (uint32_t)kNoEntry;
        if (block_get(blk, r & 7) != e) {
          block_set(blk, r & 7, e);
          dirty = true;
        }
      }
      if (got >= 0) {
        ++n;
        miss = 0;
        last = st;
        rin = r;
      } else if (++miss >= K.n_gap) {
        break;
      }
      if ((r & 7) == 0 && r > 0) {   // into the block below
        if (dirty) hits.store_block(cb, blk);
        dirty = false;
        --cb;
        blk = blk_dn;
        blk_dn = cb > 0 ? hits.load_block(cb - 1) : block_empty();
      }
    }
    if (dirty) hits.store_block(cb, blk);
    tl_hits += (unsigned)n;
    int32_t* info = S.tl_info + (size_t)T * 4;
    const bool valid = n >= K.n_min_tracklet;
    info[0] = n;
    info[1] = rin;
    info[2] = rout;
    info[3] = valid ? 1 : 0;
    const uint32_t id0 = (uint32_t)((int64_t)x0.id - ev0);
    const uint32_t w = ((uint32_t)n << 24) | (0xFFFFFFu - id0);
    S.tl_weight[T] = w;
    // a6 (ownership): every hit of a valid tracklet keeps the largest weight
    // of the tracklets holding it; issued here, so the atomics overlap the
    // other lanes' Kalman steps, and only where the weight read is smaller
    if (valid) {
      // the list is read back a block of eight rows per memory round trip
      for (int b = rin >> 3; b <= rout >> 3; ++b) {
        const uint4 v = hits.load_block(b);
        uint32_t f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) f[u] = (uint32_t)S.row_off[gr + min(8 * b + u, kRows - 1)];
        int32_t h[8];
        uint32_t cur[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = 8 * b + u;
          h[u] = (r >= rin && r <= rout) ? entry_hit(block_get(v, u), f[u]) : -1;
          cur[u] = h[u] >= 0 ? S.weight[h[u]] : 0xFFFFFFFFu;
        }
        // a weight already at least w stays so (the maximum only grows)
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (cur[u] < w) atomicMax(&S.weight[h[u]], w);
      }
    }
    float* sv = S.tl_state + (size_t)T * 5;
    sv[0] = last.y;
    sv[1] = last.z;
    sv[2] = last.s;
    sv[3] = last.t;
    sv[4] = last.q;
  }
  wave_add_u64(&S.stats[0], done);
  wave_add_u64(&S.stats[1], visits);
  wave_add_u64(&S.stats[2], examined);
  wave_add_u64(&S.stats[6], tl_hits);
  wave_add_u64(&S.stats[7], tries);
}

void launch_tracklets(int wb, int blocks, int threads, hipStream_t st, const Slot& S,
                      const DevConst& K, int g0) {
  switch (wb) {
    case 2: k_tracklets<2><<<blocks, threads, 0, st>>>(S, K, g0); break;
    case 8: k_tracklets<8><<<blocks, threads, 0, st>>>(S, K, g0); break;
    default: k_tracklets<4><<<blocks, threads, 0, st>>>(S, K, g0); break;
  }
}

}  // namespace tpc
