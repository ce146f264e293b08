// C ABI of the tracker: argument checks, workspace carving, launch order.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <array>
#include <vector>

#include "tpc_device.h"
#include "tpc_kernels.h"

using namespace tpc;

namespace {

constexpr int kScanTile = 1024;
constexpr int64_t kCountChunkHost = 4096;    // clusters per block of k_count

struct SlotHost {
  Slot d{};
  int state = 0;   // 0 empty, 1 staged, 2 grid built, 3 sectors tracked, 4 final
  int64_t n = 0;
  int n_events = 0;
  std::vector<int64_t> ev_off;
  hipEvent_t done = nullptr;          // recorded after the slot's last enqueued work
  hipGraphExec_t graph = nullptr;     // captured tracking sequence
  std::vector<int64_t> graph_ev_off;  // staged shape the graph was captured with
  const void* graph_in[4] = {};
  MergeSlot m{};                      // cross-sector merger buffers
  bool merged = false;                // merger output valid for the staged data
  uint8_t* own_sector = nullptr;
  uint8_t* own_row = nullptr;
  float* own_y = nullptr;
  float* own_z = nullptr;
  // clusters per sector of the built grid, read back for the per-sector
  // launch sequences (each launch sized by its own sector); empty until read
  std::vector<uint32_t> sec_n;
};

// __global__ helpers local to this file
__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

__global__ void k_kf_step(DevConst K, float* state, const float* dx, const float* meas, float* result,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float* st = state + i * 20;
  Helix<float> h;
  h.y = st[0];
  h.z = st[1];
  h.s = st[2];
  h.t = st[3];
  h.q = st[4];
  for (int k = 0; k < 15; ++k) h.c[k] = st[5 + k];
  int bits = 0;
  float chi2 = 0.0f;
  if (transport(h, dx[i], K.b, K.smax)) {
    bits = 1;
    const float* m = meas + i * 4;
    if (kalman_update(h, m[0], m[1], m[2], m[3], K.chi2max, K.smax, true, &chi2)) bits |= 2;
  }
  st[0] = h.y;
  st[1] = h.z;
  st[2] = h.s;
  st[3] = h.t;
  st[4] = h.q;
  for (int k = 0; k < 15; ++k) st[5 + k] = h.c[k];
  int* ri = reinterpret_cast<int*>(result + i * 2);
  ri[0] = bits;
  result[i * 2 + 1] = chi2;
}

// Links of one event as cluster IDs (diagnostics).
__global__ void k_links_out(Slot S, int e, int32_t* up, int32_t* dn, int32_t* upc, int32_t* dnc) {
  const uint32_t b = S.row_off[e * kSectorsPerEvent * kRows];
  const uint32_t t = S.row_off[(e + 1) * kSectorsPerEvent * kRows];
  const int64_t ev0 = S.ev_off[e];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = b + blockIdx.x * blockDim.x + threadIdx.x; p < t; p += stride) {
    const int64_t id = (int64_t)S.hit[p].id - ev0;
    const int32_t l[4] = {S.up[p], S.dn[p], S.hit[p].upc, S.dnc[p]};
    int32_t* o[4] = {up, dn, upc, dnc};
    for (int k = 0; k < 4; ++k)
      o[k][id] = l[k] >= 0 ? (int32_t)((int64_t)S.hit[l[k]].id - ev0) : -1;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

struct Carver {
  uint8_t* base;
  size_t off = 0;
  bool dry;
  template <class T>
  T* take(int64_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
    off += sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    return p;
  }
};

// Capacities of the tracklet and track regions: cleaned chains are
// disjoint and a start hit heads one of >= n_min_chain hits, so a sector of
// n hits has at most n/n_min_chain start hits; an output
// track owns >= n_min_track hits that no other track owns, so at most
// n/n_min_track tracks.  Each sector's region gets one entry more.
int64_t tracklet_cap(const tpc_params& p) {
  return p.max_clusters / p.n_min_chain + (int64_t)p.max_events * kSectorsPerEvent;
}
int64_t track_cap(const tpc_params& p) {
  return p.max_clusters / p.n_min_track + (int64_t)p.max_events * kSectorsPerEvent;
}

void carve_slot(Carver& c, const tpc_params& p, Slot& s, SlotHost* h) {
  const int64_t N = p.max_clusters;
  const int E = p.max_events;
  const int64_t S = (int64_t)E * kSectorsPerEvent;
  const int64_t SR = S * kRows;
  const int64_t cap_tl = tracklet_cap(p);
  const int64_t cap_tk = track_cap(p);
  uint8_t* own_sector = c.take<uint8_t>(N);
  uint8_t* own_row = c.take<uint8_t>(N);
  float* own_y = c.take<float>(N);
  float* own_z = c.take<float>(N);
  if (h) {
    h->own_sector = own_sector;
    h->own_row = own_row;
    h->own_y = own_y;
    h->own_z = own_z;
  }
  s.ev_off = c.take<int64_t>(E + 1);
  s.row_cnt = c.take<uint32_t>(SR);
  s.row_off = c.take<uint32_t>(SR + 1);
  s.bins = c.take<RowBins>(SR);
  s.row_bin = c.take<uint32_t>(SR + 1);
  // a row of n hits has at most kBinsPerHit * max(n, 1) bins, plus one end entry
  s.bin_off = c.take<uint32_t>(kBinsPerHit * (N + SR) + SR + 1);
  s.rank = c.take<uint32_t>(N);
  s.hit = c.take<Hit>(N);
  s.hit_sr = c.take<uint32_t>(N);
  s.up = c.take<int32_t>(N);
  s.dn = c.take<int32_t>(N);
  s.dnc = c.take<int32_t>(N);
  s.tl_base = c.take<uint32_t>(S + 1);
  s.tk_base = c.take<uint32_t>(S + 1);
  s.row_nstart = c.take<uint32_t>(SR + 1);
  s.range_cnt = c.take<uint32_t>(16);
  s.big_rows = c.take<uint32_t>(N / 1024 + 1);
  s.start_hit = c.take<int32_t>(cap_tl);
  s.start_sr = c.take<int32_t>(cap_tl);
  s.tl_hits = c.take<uint16_t>((cap_tl + 63) / 64 * 64 * kRowBlocks * 8);
  s.tl_info = c.take<int32_t>(cap_tl * 4);
  s.tl_weight = c.take<uint32_t>(cap_tl);
  s.tl_state = c.take<float>(cap_tl * 5);
  s.tl_sel = c.take<uint32_t>(cap_tl + 1);
  s.weight = c.take<uint32_t>(N);
  s.tk_tracklet = c.take<int32_t>(cap_tk);
  s.tk_own = c.take<int32_t>(cap_tk * kRows);
  s.tk_own_row = c.take<uint8_t>(cap_tk * kRows);
  s.tk_nown = c.take<int32_t>(cap_tk);
  s.tk_info = c.take<int32_t>(cap_tk * 4);
  s.tk_par = c.take<double>(cap_tk * 5);
  s.tk_cov = c.take<double>(cap_tk * 15);
  s.tk_chi2 = c.take<double>(cap_tk);
  s.tmap = c.take<int32_t>(N);
  s.scan_a = c.take<uint32_t>(N + 1);
  s.scan_b = c.take<uint32_t>(std::max<int64_t>(std::max<int64_t>(N, SR), cap_tl) / kScanTile + 4);
  s.out_count = c.take<uint32_t>(2);
  s.out_ntk = c.take<uint32_t>(cap_tk + 1);
  s.out_order = c.take<int32_t>(cap_tk);
  s.out_tracks = c.take<tpc_track>(cap_tk);
  s.out_hits = c.take<int32_t>(N);
  s.ev_track_off = c.take<uint32_t>(E + 1);
  s.ev_hit_off = c.take<uint32_t>(E + 1);
  s.err = c.take<uint32_t>(4);
  s.stats = c.take<unsigned long long>(8);
  MergeSlot m;
  m.in_off = c.take<uint32_t>(SR + 1);
  m.in_cur = c.take<uint32_t>(SR);
  m.in_list = c.take<int32_t>(cap_tk);
  m.out_off = c.take<uint32_t>(SR + 1);
  m.out_cur = c.take<uint32_t>(SR);
  m.out_list = c.take<int32_t>(cap_tk);
  m.op = c.take<double>(cap_tk * 5);
  m.oc = c.take<double>(cap_tk * 15);
  m.ok = c.take<int32_t>(cap_tk);
  m.best_out = c.take<int32_t>(cap_tk);
  m.chi_out = c.take<double>(cap_tk);
  m.best_in = c.take<int32_t>(cap_tk);
  m.chi_in = c.take<double>(cap_tk);
  m.in_key = c.take<unsigned long long>(cap_tk);
  m.out_key = c.take<unsigned long long>(cap_tk);
  // compatible pairs: two per track of capacity in all (a central event has
  // ~0.3), spread over the segments
  m.pair_cap = (uint32_t)std::min<int64_t>((2 * cap_tk + kPairSegs - 1) / kPairSegs, 0x7FFFFFFFll);
  m.pair_a = c.take<int32_t>((int64_t)m.pair_cap * kPairSegs);
  m.pair_b = c.take<int32_t>((int64_t)m.pair_cap * kPairSegs);
  m.pair_key = c.take<unsigned long long>((int64_t)m.pair_cap * kPairSegs);
  m.pair_n = c.take<uint32_t>(kPairSegs * kPairPad);
  m.link_out = c.take<int32_t>(cap_tk);
  m.link_in = c.take<int32_t>(cap_tk);
  m.head_ok = c.take<int32_t>(cap_tk);
  m.nseg = c.take<int32_t>(cap_tk);
  m.nfit = c.take<int32_t>(cap_tk);
  m.par = c.take<double>(cap_tk * 5);
  m.cov = c.take<double>(cap_tk * 15);
  m.chi2 = c.take<double>(cap_tk);
  m.emit = c.take<uint32_t>(cap_tk + 1);
  m.nh = c.take<uint32_t>(cap_tk + 1);
  m.into = c.take<int32_t>(cap_tk);
  m.tracks = c.take<tpc_track>(cap_tk);
  m.hits = c.take<int32_t>(N);
  m.out_nseg = c.take<int32_t>(cap_tk);
  m.ev_track_off = c.take<uint32_t>(E + 1);
  m.ev_hit_off = c.take<uint32_t>(E + 1);
  if (h) h->m = m;
  s.cap_n = N;
  s.cap_tl = cap_tl;
  s.cap_tk = cap_tk;
  s.cap_e = E;
}

// Per-stream copies of the only buffers that the per-sector launch sequence
// shares between sectors (start/track counters, scan partials, selection
// flags), so sectors on different streams never touch the same bytes.
constexpr int kMaxLanes = 8;
struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  uint32_t* range_cnt = nullptr;
  uint32_t* scan_b = nullptr;
  uint32_t* tl_sel = nullptr;
};

void carve_lanes(Carver& c, const tpc_params& p, Lane* lanes) {
  const int64_t N = p.max_clusters;
  const int64_t S = (int64_t)p.max_events * kSectorsPerEvent;
  const int64_t SR = S * kRows;
  const int64_t cap_tl = tracklet_cap(p);
  for (int i = 0; i < kMaxLanes; ++i) {
    uint32_t* a = c.take<uint32_t>(16);
    uint32_t* b = c.take<uint32_t>(std::max<int64_t>(std::max<int64_t>(N, SR), cap_tl) / kScanTile + 4);
    uint32_t* t = c.take<uint32_t>(cap_tl + 1);
    if (lanes) {
      lanes[i].range_cnt = a;
      lanes[i].scan_b = b;
      lanes[i].tl_sel = t;
    }
  }
}

bool params_ok(const tpc_params* p) {
  if (!p) return false;
  if (!(p->max_slots >= 1 && p->max_slots <= 1024)) return false;
  if (!(p->max_events >= 1 && p->max_events <= 4096)) return false;
  if (!(p->max_clusters >= 1 && p->max_clusters <= (int64_t)0x7FFFFFFF)) return false;
  if (!(p->n_gap >= 1 && p->n_min_tracklet >= 2 && p->n_min_track >= 3)) return false;
  if (!(p->n_min_chain >= 3 && p->n_min_chain <= kRows)) return false;
  if (!(p->tl_block == 64 || p->tl_block == 128 || p->tl_block == 256)) return false;
  if (!(p->win_batch == 2 || p->win_batch == 4 || p->win_batch == 8)) return false;
  if (!(p->row_batch == 4 || p->row_batch == 8 || p->row_batch == 16)) return false;
  if (!(p->s_max > 0.0f && p->s_max < 1.0f && p->chi2_max > 0.0f)) return false;
  if (!(p->nf_window > 0.0f && p->k_win > 0.0f && p->w_max > 0.0f)) return false;
  if (!(p->c_s0 > 0.0f && p->c_t0 > 0.0f && p->c_q0 > 0.0f)) return false;
  if (!(p->bin_target > 0.0f && p->bin_min_edge > 0.0f)) return false;
  if (!(p->x0_cm >= 0.0f && p->ms_mass >= 0.0f && std::isfinite(p->x0_cm) &&
        std::isfinite(p->ms_mass)))
    return false;
  return true;
}

// Why a geometry is refused (nullptr if it is valid).
const char* geometry_error(const tpc_geometry* g) {
  if (g->n_sectors != TPC_N_SECTORS || g->n_rows != TPC_N_ROWS)
    return "geometry must have 36 sectors of 159 pad rows";
  for (int r = 0; r < TPC_N_ROWS; ++r) {
    if (!(std::isfinite(g->row_x[r]) && g->row_x[r] > 0.0f) ||
        (r > 0 && !(g->row_x[r] > g->row_x[r - 1])))
      return "pad-row radii must be positive and increasing";
  }
  if (!(g->z_max > 0.0f && g->tan_half_angle > 0.0f && g->sigma_y0 > 0.0f && g->sigma_z0 > 0.0f &&
        g->sigma_y1 >= 0.0f && g->sigma_z1 >= 0.0f && std::isfinite(g->bz_tesla)))
    return "bad geometry constants";
  return nullptr;
}

// The constants every kernel receives, from a checked geometry and params.
void fill_constants(DevConst& k, const tpc_geometry* g, const tpc_params* p) {
  std::memset(&k, 0, sizeof(k));
  for (int r = 0; r < kRows; ++r) k.row_x[r] = g->row_x[r];
  k.tanh_half = g->tan_half_angle;
  k.z_max = g->z_max;
  k.sy0 = g->sigma_y0;
  k.sy1 = g->sigma_y1;
  k.sz0 = g->sigma_z0;
  k.sz1 = g->sigma_z1;
  k.sy1z = k.sy1 / k.z_max;
  k.sz1z = k.sz1 / k.z_max;
  k.sy1zd = (double)k.sy1 / (double)k.z_max;
  k.sz1zd = (double)k.sz1 / (double)k.z_max;
  // curvature per unit q/pT: d(phi)/dl = b q/pT, b = -c Bz, c = 0.00299792458 GeV/(T cm)
  k.bd = -0.00299792458 * (double)g->bz_tesla;
  k.b = (float)k.bd;
  k.nf_w = p->nf_window;
  k.nf_mmax = p->nf_mmax;
  k.chi2max = p->chi2_max;
  k.kwin = p->k_win;
  k.wmax = p->w_max;
  k.smax = p->s_max;
  k.cs0 = p->c_s0;
  k.ct0 = p->c_t0;
  k.cq0 = p->c_q0;
  k.medge = p->m_edge;
  k.mz = p->m_z;
  k.n_gap = p->n_gap;
  k.n_min_tracklet = p->n_min_tracklet;
  k.n_min_track = p->n_min_track;
  k.n_min_chain = p->n_min_chain;
  k.bin_target = p->bin_target;
  k.bin_min_edge = p->bin_min_edge;
  // scattering law: theta0^2 = (k^2 / X0) L / (beta p)^2 with
  // k = 13.6 MeV (1 + 0.038 ln(1 cm / X0)); computed in double on the host
  if (p->x0_cm > 0.0f) {
    const double x0 = (double)p->x0_cm;
    const double kms = 0.0136 * (1.0 + 0.038 * std::log(1.0 / x0));
    k.kkd = kms * kms / x0;
    k.m2d = (double)p->ms_mass * (double)p->ms_mass;
  } else {
    k.kkd = 0.0;
    k.m2d = 0.0;
  }
  k.kk = (float)k.kkd;
  k.m2 = (float)k.m2d;
}

thread_local std::string g_init_error;

}  // namespace

struct tpc_ctx {
  DevConst k;
  tpc_params p;
  tpc_geometry g;
  hipStream_t stream;
  uint8_t* ws;
  size_t ws_bytes;
  std::vector<SlotHost> slots;
  std::string err;
  bool prof = false;
  bool prof_valid = false;
  bool capturing = false;
  int prof_slot = -1;
  // stage-boundary events of the profiled steps, a ring of kProfRing steps
  std::vector<std::array<hipEvent_t, TPC_N_STAGES + 1>> prof_ev;
  int64_t prof_n = 0;         // profiled steps completed since profiling was switched on
  Lane lanes[kMaxLanes];
  hipEvent_t fork = nullptr;
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
};

#define TPC_HIP(call)                                                         \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return ctx->fail(TPC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TPC_LAUNCHED()                                                        \
  do {                                                                        \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess)                                                     \
      return ctx->fail(TPC_EDEVICE, std::string("launch: ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr int kProfRing = 256;

void mark(tpc_ctx* ctx, int i) {
  if (ctx->prof && !ctx->capturing)
    (void)hipEventRecord(ctx->prof_ev[(size_t)(ctx->prof_n % kProfRing)][i], ctx->stream);
}

int record_done(tpc_ctx* ctx, SlotHost& h) {
  if (!h.done) TPC_HIP(hipEventCreateWithFlags(&h.done, hipEventDisableTiming));
  TPC_HIP(hipEventRecord(h.done, ctx->stream));
  return TPC_OK;
}

int grid_stride_blocks(int64_t n, int threads, int cap = 4096) {
  const int64_t b = (n + threads - 1) / threads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// Exclusive scan in place of data[0, n) (n = *n_dev if given, else n_bound,
// which bounds it); the total goes to total_out and, with write_end, to
// data[n].
void scan_u32(hipStream_t st, uint32_t* data, const uint32_t* n_dev, int64_t n_bound,
              uint32_t* partial, uint32_t* total_out, bool write_end = true) {
  if (n_bound <= kSmallScanMax) {
    k_scan_small<<<1, 1024, 0, st>>>(data, n_dev, n_bound, total_out, write_end ? 1 : 0);
    return;
  }
  const int nb = (int)std::max<int64_t>(1, (n_bound + kScanTile - 1) / kScanTile);
  k_scan_tiles<<<nb, 256, 0, st>>>(data, n_dev, n_bound, partial);
  k_scan_partials<<<1, 1024, 0, st>>>(partial, nb, data, n_dev, n_bound, total_out,
                                      write_end ? 1 : 0);
  k_scan_apply<<<nb, 256, 0, st>>>(data, n_dev, n_bound, partial, data);
}



int build_grid(tpc_ctx* ctx, SlotHost& h) {
  Slot& s = h.d;
  hipStream_t st = ctx->stream;
  const int64_t SR = (int64_t)s.n_sectors * kRows;
  k_zero_u32<<<grid_stride_blocks(SR, 256), 256, 0, st>>>(s.row_cnt, SR);
  k_zero_u32<<<1, 64, 0, st>>>(s.err, 4);
  k_zero_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(s.stats), 16);
  int64_t max_ev = 1;
  for (int e = 0; e < h.n_events; ++e) max_ev = std::max<int64_t>(max_ev, h.ev_off[e + 1] - h.ev_off[e]);
  const unsigned chunks = (unsigned)((max_ev + kCountChunkHost - 1) / kCountChunkHost);
  k_count<<<dim3(chunks, h.n_events), 256, 0, st>>>(s);
  k_row_layout<<<grid_stride_blocks(SR, 256), 256, 0, st>>>(s, ctx->k);
  scan_u32(st, s.row_off, nullptr, SR, s.scan_b, nullptr);
  scan_u32(st, s.row_bin, nullptr, SR, s.scan_b, nullptr);
  k_row_finish<<<grid_stride_blocks(SR, 256), 256, 0, st>>>(s, ctx->p.n_min_chain, ctx->p.n_min_track);
  scan_u32(st, s.tl_base, nullptr, s.n_sectors, s.scan_b, nullptr);
  scan_u32(st, s.tk_base, nullptr, s.n_sectors, s.scan_b, nullptr);
  k_scatter<<<grid_stride_blocks(h.n, 256), 256, 0, st>>>(s);
  k_row_sort_tiny<<<(unsigned)SR, 64, 0, st>>>(s);
  k_row_sort_small<<<(unsigned)SR, 256, 0, st>>>(s);
  k_row_sort_large<<<64, 256, 0, st>>>(s);
  TPC_LAUNCHED();
  h.state = 2;
  return TPC_OK;
}

// Per-sector cluster counts of the slot's built grid, on the host (one
// synchronising read per staging; used only by the per-sector sequences).
int read_sector_counts(tpc_ctx* ctx, SlotHost& h) {
  if ((int64_t)h.sec_n.size() == (int64_t)h.d.n_sectors) return TPC_OK;
  const int ns = h.d.n_sectors;
  std::vector<uint32_t> ro((size_t)ns * kRows + 1);
  TPC_HIP(hipMemcpyAsync(ro.data(), h.d.row_off, ro.size() * sizeof(uint32_t),
                         hipMemcpyDeviceToHost, ctx->stream));
  TPC_HIP(hipStreamSynchronize(ctx->stream));
  h.sec_n.resize(ns);
  for (int g = 0; g < ns; ++g) h.sec_n[g] = ro[(size_t)(g + 1) * kRows] - ro[(size_t)g * kRows];
  return TPC_OK;
}

// Clusters of sectors [g0, g0 + ns): exact when the per-sector counts were
// read, else the slot's total (a bound).
int64_t range_clusters(const SlotHost& h, int g0, int ns) {
  if ((int64_t)h.sec_n.size() != (int64_t)h.d.n_sectors || ns == h.d.n_sectors) return h.n;
  int64_t n = 0;
  for (int g = g0; g < g0 + ns; ++g) n += h.sec_n[g];
  return n;
}

int track_range(tpc_ctx* ctx, SlotHost& h, int g0, int ns, const Lane* lane = nullptr) {
  Slot s = h.d;
  hipStream_t st = ctx->stream;
  if (lane) {
    s.range_cnt = lane->range_cnt;
    s.scan_b = lane->scan_b;
    s.tl_sel = lane->tl_sel;
    st = lane->st;
  }
  const bool marks = lane == nullptr;
  // host bounds for the grids, from the range's own clusters (the exact
  // counts live on the device; every kernel strides over them)
  const int64_t n_range = range_clusters(h, g0, ns);
  const int64_t tl_bound = std::min<int64_t>(s.cap_tl, n_range / ctx->p.n_min_chain + ns);
  const int tl_block = ctx->p.tl_block;
  const int nb_lane =
      std::max(8, grid_stride_blocks(tl_bound, tl_block, 16384 * 64 / tl_block) / 8 * 8);
  // a multiple of 8 blocks: each XCD walks its chunk of the tracklets
  const int nb_sel = (grid_stride_blocks(tl_bound, 256, 4096) + 7) / 8 * 8;
  // a lane per hit of the range (the grid from the host bound; the kernel
  // strides over the device count)
  launch_neighbours(ctx->p.win_batch, grid_stride_blocks(n_range, 256, 65536) / 8 * 8 + 8, st, s,
                    ctx->k, g0, ns);
  if (marks) mark(ctx, 2);
  // a wave per pad row
  const int nb_rows = grid_stride_blocks((int64_t)ns * kRows * 64, 256, 16384);
  k_clean_rows<<<nb_rows, 256, 0, st>>>(s, g0, ns, ctx->p.n_min_chain);
  scan_u32(st, s.row_nstart + (size_t)g0 * kRows, nullptr, (int64_t)ns * kRows, s.scan_b,
           s.range_cnt + 0, false);
  k_start_write<<<nb_rows, 256, 0, st>>>(s, g0, ns, ctx->p.n_min_chain);
  if (marks) mark(ctx, 3);
  launch_tracklets(ctx->p.win_batch, nb_lane, ctx->p.tl_block, st, s, ctx->k, g0);
  if (marks) mark(ctx, 4);
  launch_select(ctx->p.row_batch, nb_sel, st, s, ctx->k, g0);
  scan_u32(st, s.tl_sel, s.range_cnt + 0, tl_bound, s.scan_b, s.range_cnt + 1, false);
  launch_track_write(ctx->p.row_batch, nb_sel, st, s, g0, ns);
  if (marks) mark(ctx, 5);
  // four waves per block: a block's waves go to the four SIMDs of one CU,
  // so the few hundred working waves of an event do not share SIMDs
  // a multiple of 8 blocks: each XCD strides over its chunk of the tracks
  const int nb_ref = (grid_stride_blocks(std::max<int64_t>(1, tl_bound / 4), 256, 1024) + 7) / 8 * 8;
  k_refit<<<nb_ref, 256, 0, st>>>(s, ctx->k, g0, ns);
  if (marks) mark(ctx, 6);
  TPC_LAUNCHED();
  return TPC_OK;
}

int finalize(tpc_ctx* ctx, SlotHost& h) {
  Slot& s = h.d;
  hipStream_t st = ctx->stream;
  const int nbn = grid_stride_blocks(h.n, 256);
  k_flags<<<nbn, 256, 0, st>>>(s);
  scan_u32(st, s.scan_a, nullptr, h.n, s.scan_b, nullptr);
  k_order<<<std::max(nbn, (h.n_events + 256) / 256), 256, 0, st>>>(s);
  scan_u32(st, s.out_ntk, s.out_count, s.cap_tk, s.scan_b, s.out_count + 1);
  k_event_hits<<<(h.n_events + 1 + 255) / 256, 256, 0, st>>>(s);
  // 8 lanes per track (tracks <= clusters / 10 + sectors)
  k_write_out<<<grid_stride_blocks(std::max<int64_t>(1, h.n / 50) * 8, 256, 16384), 256, 0, st>>>(s, ctx->k);
  mark(ctx, 7);
  TPC_LAUNCHED();
  h.state = 4;
  return TPC_OK;
}

int stage(tpc_ctx* ctx, int slot, int n_events, const int64_t* offs, const uint8_t* sector,
          const uint8_t* row, const float* y, const float* z, int flags) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  if (n_events < 1 || n_events > ctx->p.max_events)
    return ctx->fail(TPC_EINVAL, "number of events out of range");
  if (!offs || offs[0] != 0) return ctx->fail(TPC_EINVAL, "event offsets must start at 0");
  for (int e = 0; e < n_events; ++e) {
    if (offs[e + 1] < offs[e]) return ctx->fail(TPC_EINVAL, "event offsets decrease");
    if (offs[e + 1] - offs[e] > (int64_t)(1 << 24))
      return ctx->fail(TPC_EINVAL, "more than 2^24 clusters in one event");
  }
  const int64_t n = offs[n_events];
  if (n > ctx->p.max_clusters) return ctx->fail(TPC_ENOMEM, "more clusters than max_clusters");
  if (n > 0 && (!sector || !row || !y || !z)) return ctx->fail(TPC_EINVAL, "null cluster array");
  if (flags != TPC_HOST && flags != TPC_DEVICE) return ctx->fail(TPC_EINVAL, "flags must be TPC_HOST or TPC_DEVICE");
  SlotHost& h = ctx->slots[slot];
  Slot& s = h.d;
  hipStream_t st = ctx->stream;
  h.n = n;
  h.n_events = n_events;
  h.merged = false;
  h.sec_n.clear();
  h.ev_off.assign(offs, offs + n_events + 1);
  s.n = n;
  s.n_events = n_events;
  s.n_sectors = n_events * kSectorsPerEvent;
  if (flags == TPC_DEVICE) {
    s.sector = sector;
    s.row = row;
    s.y = y;
    s.z = z;
  } else {
    TPC_HIP(hipMemcpyAsync(h.own_sector, sector, n, hipMemcpyHostToDevice, st));
    TPC_HIP(hipMemcpyAsync(h.own_row, row, n, hipMemcpyHostToDevice, st));
    TPC_HIP(hipMemcpyAsync(h.own_y, y, n * 4, hipMemcpyHostToDevice, st));
    TPC_HIP(hipMemcpyAsync(h.own_z, z, n * 4, hipMemcpyHostToDevice, st));
    s.sector = h.own_sector;
    s.row = h.own_row;
    s.y = h.own_y;
    s.z = h.own_z;
  }
  TPC_HIP(hipMemcpyAsync(s.ev_off, h.ev_off.data(), (n_events + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, st));
  h.state = 1;
  return record_done(ctx, h);
}

int track_slot_eager(tpc_ctx* ctx, int slot);

}  // namespace

extern "C" {

int tpc_params_default(tpc_params* p) {
  if (!p) return TPC_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->nf_window = 3.0f;
  p->nf_mmax = 16.0f;
  p->chi2_max = 16.0f;
  p->k_win = 4.0f;
  p->w_max = 5.0f;
  p->s_max = 0.95f;
  p->c_s0 = 1.0f;
  p->c_t0 = 1.0f;
  p->c_q0 = 100.0f;
  p->m_edge = 1.0f;
  p->m_z = 1.0f;
  p->n_gap = 6;
  p->n_min_tracklet = 10;
  p->n_min_track = 10;
  p->bin_target = 0.25f;
  p->bin_min_edge = 1.0f;
  p->max_slots = 1;
  p->max_events = 1;
  p->max_clusters = 4 << 20;
  p->x0_cm = 0.0f;
  p->ms_mass = 0.13957f;
  p->n_min_chain = 4;
  p->tl_block = 64;
  p->win_batch = 4;
  p->row_batch = 8;
  return TPC_OK;
}

size_t tpc_workspace_bytes(const tpc_params* p) {
  if (!params_ok(p)) return 0;
  Carver c{nullptr, 0, true};
  for (int i = 0; i < p->max_slots; ++i) {
    Slot s{};
    carve_slot(c, *p, s, nullptr);
  }
  carve_lanes(c, *p, nullptr);
  return c.off + 256;
}

int tpc_init_geometry(tpc_ctx** out, const tpc_geometry* g, const tpc_params* p, void* dev_workspace,
                      size_t ws_bytes, void* hip_stream) {
  g_init_error.clear();
  if (!out || !g || !p) {
    g_init_error = "null argument";
    return TPC_EINVAL;
  }
  *out = nullptr;
  const char* bad = geometry_error(g);
  if (bad) {
    g_init_error = bad;
    return TPC_EINVAL;
  }
  if (!params_ok(p)) {
    g_init_error = "bad params";
    return TPC_EINVAL;
  }
  const size_t need = tpc_workspace_bytes(p);
  if (!dev_workspace || ws_bytes < need) {
    g_init_error = "workspace too small: need " + std::to_string(need) + " bytes";
    return TPC_ENOMEM;
  }
  tpc_ctx* ctx = new tpc_ctx();
  ctx->p = *p;
  ctx->g = *g;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->ws = reinterpret_cast<uint8_t*>(dev_workspace);
  ctx->ws_bytes = ws_bytes;
  fill_constants(ctx->k, g, p);
  Carver c{ctx->ws, 0, false};
  ctx->slots.resize(p->max_slots);
  for (int i = 0; i < p->max_slots; ++i) carve_slot(c, *p, ctx->slots[i].d, &ctx->slots[i]);
  carve_lanes(c, *p, ctx->lanes);
  *out = ctx;
  return TPC_OK;
}

int tpc_load_clusters(tpc_ctx* ctx, int slot, const uint8_t* sector, const uint8_t* row,
                      const float* y, const float* z, const float* q, int64_t n, int flags) {
  (void)q;
  if (!ctx) return TPC_EINVAL;
  if (n < 0) return ctx->fail(TPC_EINVAL, "negative cluster count");
  const int64_t offs[2] = {0, n};
  return stage(ctx, slot, 1, offs, sector, row, y, z, flags);
}

int tpc_load_batch(tpc_ctx* ctx, int slot, int n_events, const int64_t* event_offsets,
                   const uint8_t* sector, const uint8_t* row, const float* y, const float* z,
                   const float* q, int flags) {
  (void)q;
  return stage(ctx, slot, n_events, event_offsets, sector, row, y, z, flags);
}

int tpc_track_sector(tpc_ctx* ctx, int slot, int sector) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (h.state < 1 || h.state == 4) return ctx->fail(TPC_ESTATE, "slot not staged or already final");
  if (sector < 0 || sector >= h.d.n_sectors) return ctx->fail(TPC_EINVAL, "sector out of range");
  if (h.state < 2) {
    const int rc = build_grid(ctx, h);
    if (rc) return rc;
  }
  int rc = read_sector_counts(ctx, h);
  if (rc) return rc;
  rc = track_range(ctx, h, sector, 1);
  if (rc) return rc;
  h.state = 3;
  return record_done(ctx, h);
}

int tpc_track_event(tpc_ctx* ctx, int slot) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (h.state < 1 || h.state >= 3) return ctx->fail(TPC_ESTATE, "slot not staged or already tracked");
  return track_slot_eager(ctx, slot);
}

int tpc_track_event_streams(tpc_ctx* ctx, int slot, int n_streams) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  if (n_streams < 1 || n_streams > kMaxLanes)
    return ctx->fail(TPC_EINVAL, "n_streams must be 1..8");
  if (ctx->capturing) return ctx->fail(TPC_ESTATE, "not available under capture");
  SlotHost& h = ctx->slots[slot];
  if (h.state < 1 || h.state >= 3) return ctx->fail(TPC_ESTATE, "slot not staged or already tracked");
  for (int i = 0; i < n_streams; ++i) {
    Lane& l = ctx->lanes[i];
    if (!l.st) TPC_HIP(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
    if (!l.done) TPC_HIP(hipEventCreateWithFlags(&l.done, hipEventDisableTiming));
  }
  if (!ctx->fork) TPC_HIP(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  if (h.state < 2) {
    const int rc = build_grid(ctx, h);
    if (rc) return rc;
  }
  {
    const int rc = read_sector_counts(ctx, h);
    if (rc) return rc;
  }
  TPC_HIP(hipEventRecord(ctx->fork, ctx->stream));
  for (int i = 0; i < n_streams; ++i) TPC_HIP(hipStreamWaitEvent(ctx->lanes[i].st, ctx->fork, 0));
  for (int g = 0; g < h.d.n_sectors; ++g) {
    const int rc = track_range(ctx, h, g, 1, &ctx->lanes[g % n_streams]);
    if (rc) return rc;
  }
  for (int i = 0; i < n_streams; ++i) {
    TPC_HIP(hipEventRecord(ctx->lanes[i].done, ctx->lanes[i].st));
    TPC_HIP(hipStreamWaitEvent(ctx->stream, ctx->lanes[i].done, 0));
  }
  const int rc = finalize(ctx, h);
  if (rc) return rc;
  return record_done(ctx, h);
}

int tpc_merge_params_default(tpc_merge_params* m) {
  if (!m) return TPC_EINVAL;
  m->chi2_max = 30.0f;
  m->row_gap = 12;
  m->step_max = 2.0f;
  m->passes = 3;
  m->s_max = 0.999f;
  return TPC_OK;
}

int tpc_merge(tpc_ctx* ctx, int slot, const tpc_merge_params* mp) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  if (!mp || !(mp->chi2_max > 0.0f) || mp->row_gap < 1 || !(mp->step_max >= 0.1f) ||
      mp->passes < 1 || mp->passes > 8 || !(mp->s_max > 0.0f && mp->s_max < 1.0f))
    return ctx->fail(TPC_EINVAL, "bad merge parameters");
  if (ctx->capturing) return ctx->fail(TPC_ESTATE, "not available under capture");
  SlotHost& h = ctx->slots[slot];
  if (h.state == 3) {
    const int rc = finalize(ctx, h);
    if (rc) return rc;
  }
  if (h.state != 4) return ctx->fail(TPC_ESTATE, "slot not tracked");
  MergeConst C;
  const double t = (double)ctx->g.tan_half_angle;
  C.ca = (1.0 - t * t) / (1.0 + t * t);
  C.sa = (2.0 * t) / (1.0 + t * t);
  C.chi2_max = (double)mp->chi2_max;
  C.step_max = (double)mp->step_max;
  C.smax = (double)mp->s_max;
  C.row_gap = mp->row_gap;
  C.passes = mp->passes;
  Slot& s = h.d;
  MergeSlot& m = h.m;
  hipStream_t st = ctx->stream;
  const int64_t K = s.cap_tk;
  const int64_t ns = s.n_sectors;
  // lane-per-track kernels in four-wave blocks: a block's waves go to the
  // four SIMDs of one CU, so the working waves do not share SIMDs
  const int nbt = grid_stride_blocks(K, 256, 2048);
  const int nb = grid_stride_blocks(K, 256);
  const int64_t nsr = ns * kRows;
  for (uint32_t* p : {m.in_off, m.out_off}) k_zero_u32<<<grid_stride_blocks(nsr + 1, 256), 256, 0, st>>>(p, nsr + 1);
  for (uint32_t* p : {m.in_cur, m.out_cur}) k_zero_u32<<<grid_stride_blocks(nsr, 256), 256, 0, st>>>(p, nsr);
  k_fill_i32<<<nb, 256, 0, st>>>(m.link_in, K, -1);
  // per track: smallest chi2 as inner and as outer partner (bit pattern;
  // all ones = none) and the partner reaching it
  for (unsigned long long* p : {m.in_key, m.out_key})
    k_fill_i32<<<grid_stride_blocks(2 * K, 256), 256, 0, st>>>(reinterpret_cast<int32_t*>(p),
                                                               2 * K, -1);
  for (int32_t* p : {m.best_in, m.best_out}) k_fill_i32<<<nb, 256, 0, st>>>(p, K, 0x7FFFFFFF);
  k_zero_u32<<<grid_stride_blocks(kPairSegs * kPairPad, 256), 256, 0, st>>>(m.pair_n, kPairSegs * kPairPad);
  k_mg_count<<<nb, 256, 0, st>>>(s, m);
  scan_u32(st, m.in_off, nullptr, nsr, s.scan_b, nullptr);
  scan_u32(st, m.out_off, nullptr, nsr, s.scan_b, nullptr);
  k_mg_scatter<<<nb, 256, 0, st>>>(s, m);
  k_mg_outer<<<nbt, 256, 0, st>>>(s, ctx->k, m, C);
  // one-wave blocks, four tracks each
  const int nbp = grid_stride_blocks((K + 3) / 4, 1, 16384);
  k_mg_pairs<false><<<nbp, 64, 0, st>>>(s, ctx->k, m, C);
  k_mg_pair_best<<<nb, 256, 0, st>>>(m);
  // walks the candidates again only if the list overflowed (a smaller grid:
  // its blocks return at once otherwise)
  k_mg_pairs<true><<<std::min(nbp, 1024), 64, 0, st>>>(s, ctx->k, m, C);
  k_mg_final<<<nb, 256, 0, st>>>(s, m);
  k_mg_link<<<nb, 256, 0, st>>>(s, m);
  k_mg_chain<<<nbt, 256, 0, st>>>(s, ctx->k, m, C);
  k_mg_emit<<<nb, 256, 0, st>>>(s, m);
  scan_u32(st, m.emit, s.out_count, K, s.scan_b, nullptr);
  scan_u32(st, m.nh, s.out_count, K, s.scan_b, nullptr);
  k_mg_event_off<<<(h.n_events + 1 + 255) / 256, 256, 0, st>>>(s, m);
  k_mg_write<<<nbt, 256, 0, st>>>(s, ctx->k, m);
  TPC_LAUNCHED();
  h.merged = true;
  return record_done(ctx, h);
}

int tpc_get_merged(tpc_ctx* ctx, int slot, int event, tpc_track* out, int64_t max_tracks,
                   int32_t* hit_ids, int64_t max_hits, int32_t* n_segments, int64_t* n_tracks,
                   int64_t* n_hits) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (event < 0 || event >= std::max(1, h.n_events)) return ctx->fail(TPC_EINVAL, "event out of range");
  if (max_tracks < 0 || max_hits < 0) return ctx->fail(TPC_EINVAL, "negative buffer size");
  if ((max_tracks > 0 && !out) || (max_hits > 0 && !hit_ids))
    return ctx->fail(TPC_EINVAL, "null output buffer");
  if (!h.merged || h.state != 4) return ctx->fail(TPC_ESTATE, "slot not merged");
  hipStream_t st = ctx->stream;
  uint32_t toff[2], hoff[2];
  TPC_HIP(hipMemcpyAsync(toff, h.m.ev_track_off + event, sizeof(toff), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(hoff, h.m.ev_hit_off + event, sizeof(hoff), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  const int64_t nt = (int64_t)toff[1] - toff[0];
  const int64_t nh = (int64_t)hoff[1] - hoff[0];
  if (n_tracks) *n_tracks = nt;
  if (n_hits) *n_hits = nh;
  if (nt > max_tracks || nh > max_hits) return ctx->fail(TPC_EOVERFLOW, "output buffers too small");
  if (nt) TPC_HIP(hipMemcpyAsync(out, h.m.tracks + toff[0], nt * sizeof(tpc_track), hipMemcpyDeviceToHost, st));
  if (nt && n_segments)
    TPC_HIP(hipMemcpyAsync(n_segments, h.m.out_nseg + toff[0], nt * 4, hipMemcpyDeviceToHost, st));
  if (nh) TPC_HIP(hipMemcpyAsync(hit_ids, h.m.hits + hoff[0], nh * 4, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  return TPC_OK;
}

int tpc_get_merge_links(tpc_ctx* ctx, int slot, int event, int32_t* link_out, int32_t* best_out,
                        double* best_chi2, int32_t* merged_into) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (event < 0 || event >= std::max(1, h.n_events)) return ctx->fail(TPC_EINVAL, "event out of range");
  if (!h.merged || h.state != 4) return ctx->fail(TPC_ESTATE, "slot not merged");
  hipStream_t st = ctx->stream;
  uint32_t toff[2], moff = 0;
  TPC_HIP(hipMemcpyAsync(toff, h.d.ev_track_off + event, sizeof(toff), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(&moff, h.m.ev_track_off + event, 4, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  const int64_t n = (int64_t)toff[1] - toff[0];
  if (n == 0) return TPC_OK;
  std::vector<int32_t> lo(n), bo(n), mi(n);
  std::vector<double> bc(n);
  TPC_HIP(hipMemcpyAsync(lo.data(), h.m.link_out + toff[0], n * 4, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(bo.data(), h.m.best_out + toff[0], n * 4, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(bc.data(), h.m.chi_out + toff[0], n * 8, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(mi.data(), h.m.into + toff[0], n * 4, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) {
    if (link_out) link_out[i] = lo[i] >= 0 ? lo[i] - (int32_t)toff[0] : -1;
    if (best_out) best_out[i] = bo[i] >= 0 ? bo[i] - (int32_t)toff[0] : -1;
    if (best_chi2) best_chi2[i] = bc[i];
    if (merged_into) merged_into[i] = mi[i] - (int32_t)moff;
  }
  return TPC_OK;
}

int tpc_calib_accumulate(tpc_ctx* ctx, int slot, uint32_t* hist, int n_bins, float z_lo,
                         float z_hi) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  if (!hist || n_bins < 1 || n_bins > (1 << 20) || !std::isfinite(z_lo) || !std::isfinite(z_hi) ||
      !(z_hi > z_lo))
    return ctx->fail(TPC_EINVAL, "bad histogram arguments");
  if (ctx->capturing) return ctx->fail(TPC_ESTATE, "not available under capture");
  SlotHost& h = ctx->slots[slot];
  if (h.state == 3) {
    const int rc = finalize(ctx, h);
    if (rc) return rc;
  }
  if (h.state != 4) return ctx->fail(TPC_ESTATE, "slot not tracked");
  const double w = ((double)z_hi - (double)z_lo) / (double)n_bins;
  k_cal_accumulate<<<grid_stride_blocks(h.d.cap_tk, 256, 1024), 256, 0, ctx->stream>>>(
      h.d, ctx->k, hist, n_bins, (double)z_lo, w);
  TPC_LAUNCHED();
  return record_done(ctx, h);
}

int tpc_calib_fit(const uint32_t* hist, int n_bins, float z_lo, float z_hi, float z_max,
                  double eps_tracked, double* out, void* hip_stream) {
  if (!hist || !out || n_bins < 1 || n_bins > (1 << 20) || !std::isfinite(z_lo) ||
      !std::isfinite(z_hi) || !(z_hi > z_lo) || !(z_max > 0.0f) || !std::isfinite(eps_tracked) ||
      !(std::fabs(eps_tracked) < 0.5))
    return TPC_EINVAL;
  const double w = ((double)z_hi - (double)z_lo) / (double)n_bins;
  k_cal_fit<<<1, 256, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(hist, n_bins, (double)z_lo, w,
                                                                       (double)z_max, eps_tracked, out);
  return hipGetLastError() == hipSuccess ? TPC_OK : TPC_EDEVICE;
}

int tpc_calib_correct_z(tpc_ctx* ctx, const uint8_t* sector, float* z, int64_t n, double eps) {
  if (!ctx) return TPC_EINVAL;
  if (n < 0 || (n > 0 && (!sector || !z))) return ctx->fail(TPC_EINVAL, "bad cluster arrays");
  if (!std::isfinite(eps) || !(std::fabs(eps) < 0.5)) return ctx->fail(TPC_EINVAL, "eps out of range");
  if (n == 0) return TPC_OK;
  k_cal_correct<<<grid_stride_blocks(n, 256), 256, 0, ctx->stream>>>(sector, z, n, eps,
                                                                    (double)ctx->g.z_max);
  TPC_LAUNCHED();
  return TPC_OK;
}

}  // extern "C"

namespace {

// The slot's graph was captured for its current staging (same inputs, same
// event offsets), so replaying it tracks what is staged now.
bool graph_matches(const SlotHost& h) {
  return h.graph && h.ev_off == h.graph_ev_off && h.graph_in[0] == h.d.sector &&
         h.graph_in[1] == h.d.row && h.graph_in[2] == h.d.y && h.graph_in[3] == h.d.z;
}

int capture_slot(tpc_ctx* ctx, SlotHost& h) {
  if (h.graph) {
    TPC_HIP(hipGraphExecDestroy(h.graph));
    h.graph = nullptr;
  }
  const int state0 = h.state;
  h.state = 1;                       // capture the grid build too
  ctx->capturing = true;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  int rc = TPC_OK;
  if (e == hipSuccess) {
    rc = build_grid(ctx, h);
    if (!rc) rc = track_range(ctx, h, 0, h.d.n_sectors);
    if (!rc) rc = finalize(ctx, h);
    e = hipStreamEndCapture(ctx->stream, &g);
  }
  ctx->capturing = false;
  h.state = state0;
  if (rc) return rc;
  if (e != hipSuccess) return ctx->fail(TPC_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&h.graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h.graph = nullptr;
    return ctx->fail(TPC_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e));
  }
  h.graph_ev_off = h.ev_off;
  h.graph_in[0] = h.d.sector;
  h.graph_in[1] = h.d.row;
  h.graph_in[2] = h.d.y;
  h.graph_in[3] = h.d.z;
  return TPC_OK;
}

int launch_slot_graph(tpc_ctx* ctx, SlotHost& h) {
  TPC_HIP(hipGraphLaunch(h.graph, ctx->stream));
  h.state = 4;
  return record_done(ctx, h);
}

// The one-launch-per-step sequence of a staged slot (tpc_track_event).
int track_slot_eager(tpc_ctx* ctx, int slot) {
  SlotHost& h = ctx->slots[slot];
  mark(ctx, 0);
  if (h.state < 2) {
    const int rc = build_grid(ctx, h);
    if (rc) return rc;
  }
  mark(ctx, 1);
  int rc = track_range(ctx, h, 0, h.d.n_sectors);
  if (rc) return rc;
  rc = finalize(ctx, h);
  if (rc) return rc;
  if (ctx->prof && !ctx->capturing) ++ctx->prof_n;
  ctx->prof_valid = ctx->prof;
  ctx->prof_slot = slot;
  return record_done(ctx, h);
}

}  // namespace

extern "C" {

int tpc_graph_capture(tpc_ctx* ctx, int slot) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (h.state < 1) return ctx->fail(TPC_ESTATE, "slot not staged");
  if (!ctx->stream) return ctx->fail(TPC_EINVAL, "graph capture needs a non-default stream");
  return capture_slot(ctx, h);
}

int tpc_graph_launch(tpc_ctx* ctx, int slot) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (!h.graph) return ctx->fail(TPC_ESTATE, "no graph captured for the slot");
  if (h.state < 1) return ctx->fail(TPC_ESTATE, "slot not staged");
  if (!graph_matches(h)) return ctx->fail(TPC_ESTATE, "slot staged with another shape than at capture");
  return launch_slot_graph(ctx, h);
}

int tpc_track_events(tpc_ctx* ctx, const int* slots, int n) {
  if (!ctx) return TPC_EINVAL;
  if (!slots || n < 1 || n > ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "bad slot list");
  if (!ctx->stream) return ctx->fail(TPC_EINVAL, "graph replay needs a non-default stream");
  if (ctx->capturing) return ctx->fail(TPC_ESTATE, "not available under capture");
  std::vector<char> seen(ctx->p.max_slots, 0);
  for (int i = 0; i < n; ++i) {
    if (slots[i] < 0 || slots[i] >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
    if (seen[slots[i]]) return ctx->fail(TPC_EINVAL, "slot listed twice");
    seen[slots[i]] = 1;
  }
  for (int i = 0; i < n; ++i)
    if (ctx->slots[slots[i]].state < 1) return ctx->fail(TPC_ESTATE, "slot not staged");
  for (int i = 0; i < n; ++i) {
    SlotHost& h = ctx->slots[slots[i]];
    if (!graph_matches(h)) {
      const int rc = capture_slot(ctx, h);
      if (rc) return rc;
    }
    const int rc = launch_slot_graph(ctx, h);
    if (rc) return rc;
  }
  return TPC_OK;
}

int tpc_submit(tpc_ctx* ctx, int slot) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  if (ctx->capturing) return ctx->fail(TPC_ESTATE, "not available under capture");
  SlotHost& h = ctx->slots[slot];
  if (h.state < 1) return ctx->fail(TPC_ESTATE, "slot not staged");
  if (graph_matches(h)) return launch_slot_graph(ctx, h);
  if (h.state >= 3) return ctx->fail(TPC_ESTATE, "slot already tracked");
  return track_slot_eager(ctx, slot);
}

int tpc_poll(tpc_ctx* ctx, int slot) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (!h.done) return TPC_OK;
  const hipError_t e = hipEventQuery(h.done);
  if (e == hipSuccess) return TPC_OK;
  if (e == hipErrorNotReady) return TPC_EBUSY;
  return ctx->fail(TPC_EDEVICE, std::string("poll: ") + hipGetErrorString(e));
}

int tpc_set_profiling(tpc_ctx* ctx, int enable) {
  if (!ctx) return TPC_EINVAL;
  if (enable && ctx->prof_ev.empty()) {
    ctx->prof_ev.resize(kProfRing);
    for (auto& set : ctx->prof_ev)
      for (auto& e : set) TPC_HIP(hipEventCreate(&e));
  }
  ctx->prof = enable != 0;
  ctx->prof_valid = false;
  ctx->prof_n = 0;
  return TPC_OK;
}

int tpc_get_profile(tpc_ctx* ctx, double* ms, uint64_t* counters) {
  if (!ctx) return TPC_EINVAL;
  if (!ctx->prof_valid || ctx->prof_slot < 0) return ctx->fail(TPC_ESTATE, "nothing profiled");
  SlotHost& h = ctx->slots[ctx->prof_slot];
  TPC_HIP(hipStreamSynchronize(ctx->stream));
  if (ms) {
    // mean over the profiled steps still in the ring
    const int64_t steps = std::min<int64_t>(ctx->prof_n, kProfRing);
    for (int i = 0; i < TPC_N_STAGES; ++i) {
      double sum = 0.0;
      for (int64_t k = 0; k < steps; ++k) {
        float t = 0.0f;
        TPC_HIP(hipEventElapsedTime(&t, ctx->prof_ev[(size_t)k][i], ctx->prof_ev[(size_t)k][i + 1]));
        sum += t;
      }
      ms[i] = steps > 0 ? sum / (double)steps : 0.0;
    }
  }
  if (counters) {
    unsigned long long st[8];
    TPC_HIP(hipMemcpy(st, h.d.stats, sizeof(st), hipMemcpyDeviceToHost));
    uint32_t sorted = 0, out[2] = {0, 0};
    TPC_HIP(hipMemcpy(&sorted, h.d.row_off + (size_t)h.d.n_sectors * kRows, 4, hipMemcpyDeviceToHost));
    TPC_HIP(hipMemcpy(out, h.d.out_count, sizeof(out), hipMemcpyDeviceToHost));
    for (int i = 0; i < 8; ++i) counters[i] = st[i];
    counters[4] = (uint64_t)h.n;
    counters[5] = sorted;
    counters[8] = out[0];
    counters[9] = out[1];
  }
  return TPC_OK;
}

int tpc_device_results(tpc_ctx* ctx, int slot, const tpc_track** tracks, const int32_t** hit_ids,
                       const uint32_t** event_track_off, const uint32_t** event_hit_off,
                       const uint32_t** totals) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (h.state == 3) {
    const int rc = finalize(ctx, h);
    if (rc) return rc;
  }
  if (h.state != 4) return ctx->fail(TPC_ESTATE, "slot not tracked");
  if (tracks) *tracks = h.d.out_tracks;
  if (hit_ids) *hit_ids = h.d.out_hits;
  if (event_track_off) *event_track_off = h.d.ev_track_off;
  if (event_hit_off) *event_hit_off = h.d.ev_hit_off;
  if (totals) *totals = h.d.out_count;
  return TPC_OK;
}

int tpc_get_tracks(tpc_ctx* ctx, int slot, int event, tpc_track* out, int64_t max_tracks,
                   int32_t* hit_ids, int64_t max_hits, int64_t* n_tracks, int64_t* n_hits) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (event < 0 || event >= std::max(1, h.n_events)) return ctx->fail(TPC_EINVAL, "event out of range");
  if (max_tracks < 0 || max_hits < 0) return ctx->fail(TPC_EINVAL, "negative buffer size");
  if ((max_tracks > 0 && !out) || (max_hits > 0 && !hit_ids))
    return ctx->fail(TPC_EINVAL, "null output buffer");
  if (h.state == 3) {
    const int rc = finalize(ctx, h);
    if (rc) return rc;
  }
  if (h.state != 4) return ctx->fail(TPC_ESTATE, "slot not tracked");
  hipStream_t st = ctx->stream;
  uint32_t err[4], toff[2], hoff[2];
  TPC_HIP(hipMemcpyAsync(err, h.d.err, sizeof(err), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(toff, h.d.ev_track_off + event, sizeof(toff), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(hoff, h.d.ev_hit_off + event, sizeof(hoff), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  if (err[0]) return ctx->fail(TPC_EINVAL, std::to_string(err[0]) + " invalid clusters (sector, row or coordinates)");
  if (err[1]) return ctx->fail(TPC_EINVAL, "a pad row holds more than 4096 clusters");
  if (err[2]) return ctx->fail(TPC_EDEVICE, "internal capacity exceeded");
  const int64_t nt = (int64_t)toff[1] - toff[0];
  const int64_t nh = (int64_t)hoff[1] - hoff[0];
  if (n_tracks) *n_tracks = nt;
  if (n_hits) *n_hits = nh;
  if (nt > max_tracks || nh > max_hits) return ctx->fail(TPC_EOVERFLOW, "output buffers too small");
  if (nt) TPC_HIP(hipMemcpyAsync(out, h.d.out_tracks + toff[0], nt * sizeof(tpc_track), hipMemcpyDeviceToHost, st));
  if (nh) TPC_HIP(hipMemcpyAsync(hit_ids, h.d.out_hits + hoff[0], nh * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  return TPC_OK;
}

int tpc_get_slot_tracks(tpc_ctx* ctx, int slot, tpc_track* out, int64_t max_tracks,
                        int32_t* hit_ids, int64_t max_hits, uint32_t* event_track_off,
                        uint32_t* event_hit_off, int64_t* n_tracks, int64_t* n_hits) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (max_tracks < 0 || max_hits < 0) return ctx->fail(TPC_EINVAL, "negative buffer size");
  if ((max_tracks > 0 && !out) || (max_hits > 0 && !hit_ids))
    return ctx->fail(TPC_EINVAL, "null output buffer");
  if (!event_track_off || !event_hit_off) return ctx->fail(TPC_EINVAL, "null offset array");
  if (h.state == 3) {
    const int rc = finalize(ctx, h);
    if (rc) return rc;
  }
  if (h.state != 4) return ctx->fail(TPC_ESTATE, "slot not tracked");
  const int ne = std::max(1, h.n_events);
  hipStream_t st = ctx->stream;
  uint32_t err[4];
  TPC_HIP(hipMemcpyAsync(err, h.d.err, sizeof(err), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(event_track_off, h.d.ev_track_off, (ne + 1) * sizeof(uint32_t),
                         hipMemcpyDeviceToHost, st));
  TPC_HIP(hipMemcpyAsync(event_hit_off, h.d.ev_hit_off, (ne + 1) * sizeof(uint32_t),
                         hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  if (err[0]) return ctx->fail(TPC_EINVAL, std::to_string(err[0]) + " invalid clusters (sector, row or coordinates)");
  if (err[1]) return ctx->fail(TPC_EINVAL, "a pad row holds more than 4096 clusters");
  if (err[2]) return ctx->fail(TPC_EDEVICE, "internal capacity exceeded");
  const uint32_t t0 = event_track_off[0], h0 = event_hit_off[0];
  for (int e = 0; e <= ne; ++e) {
    event_track_off[e] -= t0;
    event_hit_off[e] -= h0;
  }
  const int64_t nt = event_track_off[ne], nh = event_hit_off[ne];
  if (n_tracks) *n_tracks = nt;
  if (n_hits) *n_hits = nh;
  if (nt > max_tracks || nh > max_hits) return ctx->fail(TPC_EOVERFLOW, "output buffers too small");
  if (nt) TPC_HIP(hipMemcpyAsync(out, h.d.out_tracks + t0, nt * sizeof(tpc_track), hipMemcpyDeviceToHost, st));
  if (nh) TPC_HIP(hipMemcpyAsync(hit_ids, h.d.out_hits + h0, nh * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  return TPC_OK;
}

int tpc_get_links(tpc_ctx* ctx, int slot, int event, int32_t* up, int32_t* dn, int32_t* up_clean,
                  int32_t* dn_clean) {
  if (!ctx) return TPC_EINVAL;
  if (slot < 0 || slot >= ctx->p.max_slots) return ctx->fail(TPC_EINVAL, "slot out of range");
  SlotHost& h = ctx->slots[slot];
  if (h.state < 3) return ctx->fail(TPC_ESTATE, "slot not tracked");
  if (event < 0 || event >= h.n_events) return ctx->fail(TPC_EINVAL, "event out of range");
  if (h.state == 3) {                  // the scratch below is free once finalised
    const int rc = finalize(ctx, h);
    if (rc) return rc;
  }
  const int64_t ne = h.ev_off[event + 1] - h.ev_off[event];
  hipStream_t st = ctx->stream;
  // per-cluster buffers no longer needed after the canonical ordering
  int32_t* tmp[4] = {reinterpret_cast<int32_t*>(h.d.rank), reinterpret_cast<int32_t*>(h.d.scan_a),
                     h.d.tmap, reinterpret_cast<int32_t*>(h.d.weight)};
  for (int k = 0; k < 4; ++k) k_fill_i32<<<grid_stride_blocks(ne, 256), 256, 0, st>>>(tmp[k], ne, -1);
  k_links_out<<<grid_stride_blocks(ne, 256), 256, 0, st>>>(h.d, event, tmp[0], tmp[1], tmp[2], tmp[3]);
  TPC_LAUNCHED();
  int32_t* dst[4] = {up, dn, up_clean, dn_clean};
  for (int k = 0; k < 4; ++k)
    if (dst[k] && ne) TPC_HIP(hipMemcpyAsync(dst[k], tmp[k], ne * 4, hipMemcpyDeviceToHost, st));
  TPC_HIP(hipStreamSynchronize(st));
  return TPC_OK;
}

int tpc_kf_step_f32(tpc_ctx* ctx, float* state, const float* dx, const float* meas, float* result,
                    int64_t n) {
  if (!ctx) return TPC_EINVAL;
  if (n < 0 || (n > 0 && (!state || !dx || !meas || !result)))
    return ctx->fail(TPC_EINVAL, "bad arguments");
  if (n == 0) return TPC_OK;
  k_kf_step<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(ctx->k, state, dx, meas, result, n);
  TPC_LAUNCHED();
  return TPC_OK;
}

const char* tpc_last_error(const tpc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

int tpc_destroy(tpc_ctx* ctx) {
  if (!ctx) return TPC_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& set : ctx->prof_ev)
    for (hipEvent_t e : set)
      if (e) (void)hipEventDestroy(e);
  for (Lane& l : ctx->lanes) {
    if (l.st) {
      (void)hipStreamSynchronize(l.st);
      (void)hipStreamDestroy(l.st);
    }
    if (l.done) (void)hipEventDestroy(l.done);
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  for (SlotHost& h : ctx->slots) {
    if (h.graph) (void)hipGraphExecDestroy(h.graph);
    if (h.done) (void)hipEventDestroy(h.done);
  }
  delete ctx;
  return TPC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free tracking of one event: the workspace is a fixed array of
// device memory owned by the library (one per GPU, held until the process
// ends), for callers that cannot allocate device memory.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
}  // namespace

// In host code this name is only a stand-in for the device array: host code
// takes the array's device address from hipGetSymbolAddress (once per GPU)
// and passes that address, never this name.
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxStaticDevices = 64;
struct StaticDevice {
  uint8_t* ptr = nullptr;     // device address of `scratch` on this GPU
  tpc_ctx* ctx = nullptr;     // host-side context over it (no device memory of its own)
};
StaticDevice g_static[kMaxStaticDevices];
std::mutex g_static_mu;

__global__ void k_static_stage(int64_t* ev_off, int64_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ev_off[0] = 0;
    ev_off[1] = n;
  }
}

// Tracks and hit IDs of the slot's one event into the caller's arrays (at
// most max_tracks / max_hits of them) and the status words.
__global__ void k_static_out(Slot S, tpc_track* tracks, int64_t max_tracks, int32_t* hits,
                             int64_t max_hits, uint32_t* status) {
  constexpr int64_t kWords = (int64_t)(sizeof(tpc_track) / 4);
  const int64_t nt = S.out_count[0], nh = S.out_count[1];
  const int64_t words = (nt < max_tracks ? nt : max_tracks) * kWords;
  const int64_t nhc = nh < max_hits ? nh : max_hits;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(S.out_tracks);
  uint32_t* dst = reinterpret_cast<uint32_t*>(tracks);
  for (int64_t i = t0; i < words; i += stride) dst[i] = src[i];
  for (int64_t i = t0; i < nhc; i += stride) hits[i] = S.out_hits[i];
  if (t0 == 0) {
    uint32_t flags = 0u;
    if (S.err[0]) flags |= 1u;
    if (S.err[1]) flags |= 2u;
    if (S.err[2]) flags |= 4u;
    if (nt > max_tracks || nh > max_hits) flags |= 8u;
    status[0] = (uint32_t)nt;
    status[1] = (uint32_t)nh;
    status[2] = flags;
    status[3] = 0u;
  }
}

int static_fail(int code, const char* m) {
  g_init_error = m;
  return code;
}

}  // namespace

extern "C" int tpc_track_event_noalloc(const tpc_geometry* g, const tpc_params* p,
                                       const uint8_t* sector, const uint8_t* row, const float* y,
                                       const float* z, int64_t n, tpc_track* tracks,
                                       int64_t max_tracks, int32_t* hit_ids, int64_t max_hits,
                                       uint32_t* status, void* hip_stream) {
  g_init_error.clear();
  if (!g || !p || !status) return static_fail(TPC_EINVAL, "null argument");
  if (const char* bad = geometry_error(g)) return static_fail(TPC_EINVAL, bad);
  if (n < 0 || n > ((int64_t)1 << 24)) return static_fail(TPC_EINVAL, "cluster count must be 0..2^24");
  if (n > 0 && (!sector || !row || !y || !z)) return static_fail(TPC_EINVAL, "null cluster array");
  if (max_tracks < 0 || max_hits < 0) return static_fail(TPC_EINVAL, "negative buffer size");
  if ((max_tracks > 0 && !tracks) || (max_hits > 0 && !hit_ids))
    return static_fail(TPC_EINVAL, "null output buffer");
  tpc_params q = *p;
  q.max_slots = 1;
  q.max_events = 1;
  q.max_clusters = std::max<int64_t>(n, 1);
  if (!params_ok(&q)) return static_fail(TPC_EINVAL, "bad params");
  if (tpc_workspace_bytes(&q) > kStaticScratchBytes)
    return static_fail(TPC_ENOMEM, "event too large for the allocation-free entry (its 64 MiB "
                                   "workspace holds about 150,000 clusters)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxStaticDevices)
    return static_fail(TPC_EDEVICE, "no usable current device");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticDevice& sd = g_static[dev];
  if (!sd.ptr) {
    // set-up, once per GPU, with that GPU current: the array's device address
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return static_fail(TPC_EDEVICE, "hipGetSymbolAddress of the workspace array failed");
    }
    sd.ptr = static_cast<uint8_t*>(ptr);
    sd.ctx = new tpc_ctx();
    sd.ctx->slots.resize(1);
    sd.ctx->slots[0].ev_off.reserve(2);
  }
  tpc_ctx* ctx = sd.ctx;
  ctx->p = q;
  ctx->g = *g;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  ctx->ws = sd.ptr;
  ctx->ws_bytes = kStaticScratchBytes;
  fill_constants(ctx->k, g, &q);
  SlotHost& h = ctx->slots[0];
  Carver c{sd.ptr, 0, false};
  carve_slot(c, q, h.d, &h);
  carve_lanes(c, q, ctx->lanes);
  Slot& s = h.d;
  h.n = n;
  h.n_events = 1;
  h.merged = false;
  h.sec_n.clear();
  h.ev_off.resize(2);
  h.ev_off[0] = 0;
  h.ev_off[1] = n;
  s.n = n;
  s.n_events = 1;
  s.n_sectors = kSectorsPerEvent;
  s.sector = sector;
  s.row = row;
  s.y = y;
  s.z = z;
  hipStream_t st = ctx->stream;
  k_static_stage<<<1, 64, 0, st>>>(s.ev_off, n);
  h.state = 1;
  int rc = build_grid(ctx, h);
  if (rc == TPC_OK) rc = track_range(ctx, h, 0, s.n_sectors);
  if (rc == TPC_OK) rc = finalize(ctx, h);
  if (rc != TPC_OK) {
    g_init_error = ctx->err;
    return rc;
  }
  const int64_t work = std::max<int64_t>(max_tracks * (int64_t)(sizeof(tpc_track) / 4), max_hits);
  k_static_out<<<grid_stride_blocks(work, 256, 1024), 256, 0, st>>>(s, tracks, max_tracks, hit_ids,
                                                                    max_hits, status);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return static_fail(TPC_EDEVICE, hipGetErrorString(e));
  return TPC_OK;
}
