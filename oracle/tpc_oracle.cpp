// TEST INFRASTRUCTURE ONLY.  Plain, slow CPU oracle of the TPC sector tracker
// (Cellular-Automaton track finding + Kalman-filter track following, the two
// methods the paper's abstract names for its GPU tracker).  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark may load this library;
// the product path never calls it.  It shares no source with the HIP library.
//
// The paper gives the method by name only (Abstract; Section 2), so every step
// below is the written-out definition this project adopted for the names, in
// the order: grid (per-row hit lists) -> neighbours finder -> link cleaner ->
// start hits -> tracklet construction (Kalman filter outward, then inward) ->
// hit-ownership weights and tracklet selection -> inward refit -> canonical
// output order.  The oracle is templated on the arithmetic type: float is the
// decision-parity mode, double the physics mode; a separate replay recomputes
// every Kalman state in double along the decisions of a float run.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -shared -fPIC
// (no contraction: every float product and sum is rounded exactly as written).
//
// Parity pins: transport vs the exact helix, Jacobian vs finite differences,
// update vs the textbook dense Kalman update, straight-line and noiseless
// fits, pulls, brute-force helix-to-hit matching, exhaustive grid queries,
// efficiency / fake / clone rates against generator truth.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

extern "C" {

struct orc_geometry {
  int32_t n_sectors;
  int32_t n_rows;
  float row_x[160];
  float bz_tesla;
  float tan_half_angle;
  float z_max;
  float sigma_y0, sigma_y1, sigma_z0, sigma_z1;
};

struct orc_params {
  float nf_window;      // neighbours-finder window half-width (cm)
  float nf_mmax;        // max triplet deviation metric
  float chi2_max;       // Kalman gate
  float k_win;          // search window in units of sqrt(S)
  float w_max;          // search window cap (cm)
  float s_max;          // max |sin phi|
  float c_s0, c_t0, c_q0;  // prior variances of sin phi, tan lambda, q/pT
  float m_edge;         // sector-edge margin (cm)
  float m_z;            // membrane / drift-length margin (cm)
  int32_t n_gap;        // consecutive missed rows that end a phase
  int32_t n_min_tracklet;
  int32_t n_min_track;
  float x0_cm;          // radiation length of the gas for the scattering noise (0: none)
  float ms_mass;        // particle mass assumed by the scattering law (GeV)
  int32_t n_min_chain;  // hits of a cleaned chain that starts a tracklet (>= 3)
};

// One output track.  Values of a float run are stored exactly in double.
struct orc_track {
  int32_t sector;
  int32_t n_hits;
  int32_t row_in;
  int32_t row_out;
  int64_t hit_off;
  int32_t inner_id;     // cluster ID of the innermost hit (canonical order key)
  int32_t start_id;     // start hit of the tracklet the track came from
  double x_ref;         // x of the innermost hit's pad row
  double par[5];        // y, z, sin phi, tan lambda, q/pT at x_ref
  double cov[15];       // lower triangle, row-major over (y, z, s, T, Q)
  double chi2;
  int32_t ndf;
  int32_t tracklet;     // index into this sector's tracklet list (debug)
};

// Constants of the cross-sector merger.
struct orc_merge_params {
  float chi2_max;       // cut on the 5-parameter match chi2 of two segments
  int32_t row_gap;      // largest pad-row distance between the segments
  float step_max;       // longest transport step between frames (cm)
  int32_t passes;       // inward refit passes of a merged track
  float s_max;          // largest |sin phi| of the merger's transports (its
                        // hits are already chosen, so this is no search cut)
};

}  // extern "C"

namespace {

constexpr int kRows = 159;

// ---------------------------------------------------------------------------
// Kalman filter primitives.  State p = (y, z, s = sin phi, T = tan lambda,
// Q = q/pT) at x; covariance C packed as the lower triangle
// (yy, zy, zz, sy, sz, ss, Ty, Tz, Ts, TT, Qy, Qz, Qs, QT, QQ).
// ---------------------------------------------------------------------------

template <class T>
struct State {
  T p[5];
  T C[15];
};

template <class T> T tabs(T v) { return v < T(0) ? -v : v; }
template <class T> T tsqrt(T v) { return std::sqrt(v); }
// a*b + c rounded once (IEEE fused multiply-add): every sum of products of
// the Kalman filter below is written as a chain of these, the same chain as
// in the GPU code, so both round at exactly the same points
template <class T> T tfma(T a, T b, T c) { return std::fma(a, b, c); }

// Transport by dx along the helix with curvature b*Q (b = -c*Bz).  The
// circle is exact: sin phi is linear in x, y advances by dx times the tangent
// of the mid-angle, and z by T times the arc length, the arc length being
// the chord times asin(u)/u expanded to u^4 (u = half the chord over the
// radius).  Returns false if |sin phi| would exceed s_max.
template <class T>
bool predict(State<T>& st, T dx, T b, T smax, T kk = T(0), T m2 = T(0)) {
  T* p = st.p;
  T* C = st.C;
  const T s = p[2], tl = p[3], q = p[4];
  const T bq = b * q;
  const T s1 = tfma(bq, dx, s);
  if (!(tabs(s1) <= smax)) return false;
  const T c0 = tsqrt(tfma(-s, s, T(1)));
  const T c1 = tsqrt(tfma(-s1, s1, T(1)));
  const T N = s + s1;
  const T D = c0 + c1;
  // one division: the reciprocals of D, c0 and c1 are products with
  // 1/(c0 c1 D)
  const T c01 = c0 * c1;
  const T inv = T(1) / (c01 * D);
  const T iD = c01 * inv;
  const T ic0 = (c1 * D) * inv;
  const T ic1 = (c0 * D) * inv;
  const T t = N * iD;
  const T dl = tabs(dx) * tsqrt(tfma(t, t, T(1)));
  const T u = T(0.5) * bq * dl;
  const T u2 = u * u;
  T ds = dl * tfma(u2, tfma(u2, T(3) / T(40), T(1) / T(6)), T(1));
  if (dx < T(0)) ds = -ds;

  // Jacobian d(y1, z1, s1)/d(s, T, Q); the other entries are those of the
  // identity.  dz/dQ is the leading-order term T b s_m dx^2 / (2 c_m^3) with
  // s_m = N/2 and the mid-angle cosine c_m taken as D/2 (equal to leading
  // order), i.e. 2 T b N dx^2 / D^3.
  const T iD2 = iD * iD;
  const T sc0 = s * ic0;
  const T sc1 = s1 * ic1;
  const T jys = dx * tfma(N, sc0 + sc1, T(2) * D) * iD2;
  const T jyq = b * dx * dx * tfma(N, sc1, D) * iD2;
  const T jzs = tl * dx * N * (ic0 * ic1 * iD);
  const T jzt = ds;
  const T jzq = T(2) * tl * b * N * dx * dx * (iD2 * iD);
  const T jsq = b * dx;

  p[0] = tfma(dx, t, p[0]);
  p[1] = tfma(tl, ds, p[1]);
  p[2] = s1;

  // C <- J C J^T, first A = J C (rows y, z, s change), then A J^T.
  const T c00 = C[0], c10 = C[1], c11 = C[2], c20 = C[3], c21 = C[4], c22 = C[5];
  const T c30 = C[6], c31 = C[7], c32 = C[8], c33 = C[9];
  const T c40 = C[10], c41 = C[11], c42 = C[12], c43 = C[13], c44 = C[14];

  const T a00 = tfma(jyq, c40, tfma(jys, c20, c00));
  const T a02 = tfma(jyq, c42, tfma(jys, c22, c20));
  const T a04 = tfma(jyq, c44, tfma(jys, c42, c40));

  const T a10 = tfma(jzq, c40, tfma(jzt, c30, tfma(jzs, c20, c10)));
  const T a11 = tfma(jzq, c41, tfma(jzt, c31, tfma(jzs, c21, c11)));
  const T a12 = tfma(jzq, c42, tfma(jzt, c32, tfma(jzs, c22, c21)));
  const T a13 = tfma(jzq, c43, tfma(jzt, c33, tfma(jzs, c32, c31)));
  const T a14 = tfma(jzq, c44, tfma(jzt, c43, tfma(jzs, c42, c41)));

  const T a20 = tfma(jsq, c40, c20);
  const T a21 = tfma(jsq, c41, c21);
  const T a22 = tfma(jsq, c42, c22);
  const T a23 = tfma(jsq, c43, c32);
  const T a24 = tfma(jsq, c44, c42);

  C[0] = tfma(jyq, a04, tfma(jys, a02, a00));
  C[1] = tfma(jyq, a14, tfma(jys, a12, a10));
  C[2] = tfma(jzq, a14, tfma(jzt, a13, tfma(jzs, a12, a11)));
  C[3] = tfma(jyq, a24, tfma(jys, a22, a20));
  C[4] = tfma(jzq, a24, tfma(jzt, a23, tfma(jzs, a22, a21)));
  C[5] = tfma(jsq, a24, a22);
  C[6] = tfma(jyq, c43, tfma(jys, c32, c30));
  C[7] = tfma(jzq, c43, tfma(jzt, c33, tfma(jzs, c32, c31)));
  C[8] = tfma(jsq, c43, c32);
  // C[9] (TT) unchanged
  C[10] = tfma(jyq, c44, tfma(jys, c42, c40));
  C[11] = tfma(jzq, c44, tfma(jzt, c43, tfma(jzs, c42, c41)));
  C[12] = tfma(jsq, c44, c42);
  // C[13] (QT), C[14] (QQ) unchanged

  // Multiple scattering in the gas (kk = k^2/X0 > 0): plane-angle variance
  // theta0^2 = kk L / (beta p)^2 over the step's path L = |arc| sqrt(1+T^2),
  // with 1/(beta p)^2 = (p^2 + m^2)/p^4 = a + m^2 a^2, a = Q^2/(1+T^2)
  // (no division by Q, no logarithm).  The angles scatter at the end of the
  // step: var(phi) = theta0^2 (1+T^2), var(lambda) = theta0^2, and with
  // dQ = Q T dlambda, dT = (1+T^2) dlambda, ds = cos(phi) dphi.
  if (kk > T(0)) {
    const T t2 = tfma(tl, tl, T(1));
    const T L = tabs(ds) * tsqrt(t2);
    const T a = (q * q) / t2;
    const T th2 = kk * L * tfma(m2, a * a, a);
    C[5] = tfma(tfma(-s1, s1, T(1)), th2 * t2, C[5]);
    C[9] = tfma(th2, t2 * t2, C[9]);
    C[13] = tfma(th2, q * tl * t2, C[13]);
    C[14] = tfma(th2, q * q * (tl * tl), C[14]);
  }
  return true;
}

// Residual weight matrix W = (H C H^T + R)^-1 for a measurement of (y, z).
template <class T>
struct Gain2 {
  T w00, w01, w11, s00, s11;
};

template <class T>
Gain2<T> weights(const State<T>& st, T vy, T vz) {
  Gain2<T> g;
  const T s00 = st.C[0] + vy;
  const T s01 = st.C[1];
  const T s11 = st.C[2] + vz;
  const T det = tfma(s00, s11, -(s01 * s01));
  const T idet = T(1) / det;
  g.w00 = s11 * idet;
  g.w01 = -s01 * idet;
  g.w11 = s00 * idet;
  g.s00 = s00;
  g.s11 = s11;
  return g;
}

template <class T>
T chi2_of(const Gain2<T>& g, T ry, T rz) {
  return tfma(ry, tfma(g.w00, ry, g.w01 * rz), rz * tfma(g.w01, ry, g.w11 * rz));
}

// Kalman update with the measured (my, mz).  With `gated` the update is
// refused (state untouched) if chi2 > chi2_max, a diagonal element would
// not stay positive, or |sin phi| would reach s_max.
template <class T>
bool update(State<T>& st, T my, T mz, T vy, T vz, T chi2max, T smax, bool gated,
            T* chi2_out) {
  const Gain2<T> g = weights(st, vy, vz);
  const T ry = my - st.p[0];
  const T rz = mz - st.p[1];
  const T chi2 = chi2_of(g, ry, rz);
  if (chi2_out) *chi2_out = chi2;
  if (gated && !(chi2 <= chi2max)) return false;
  const T* C = st.C;
  const T col0[5] = {C[0], C[1], C[3], C[6], C[10]};  // C(i, y)
  const T col1[5] = {C[1], C[2], C[4], C[7], C[11]};  // C(i, z)
  T k0[5], k1[5];
  for (int i = 0; i < 5; ++i) {
    k0[i] = tfma(col0[i], g.w00, col1[i] * g.w01);
    k1[i] = tfma(col0[i], g.w01, col1[i] * g.w11);
  }
  State<T> nx;
  for (int i = 0; i < 5; ++i) nx.p[i] = tfma(k0[i], ry, tfma(k1[i], rz, st.p[i]));
  int idx = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j, ++idx)
      nx.C[idx] = tfma(-k0[i], col0[j], tfma(-k1[i], col1[j], C[idx]));
  if (gated) {
    if (!(nx.C[0] > T(0) && nx.C[2] > T(0) && nx.C[5] > T(0) && nx.C[9] > T(0) &&
          nx.C[14] > T(0) && tabs(nx.p[2]) < smax))
      return false;
  }
  st = nx;
  return true;
}

// ---------------------------------------------------------------------------
// Per-sector tracker
// ---------------------------------------------------------------------------

template <class T>
struct Ctx {
  const orc_geometry* g;
  const orc_params* P;
  T X[kRows];
  T b, smax, chi2max, kwin, wmax, tanh, medge, mz, zmax;
  T sy0, sy1, sz0, sz1, cs0, ct0, cq0, nfw, nfm;
  T sy1z, sz1z;         // sigma_1 / z_max of the error model
  T kk, m2;             // scattering law: k^2/X0 and mass^2 (0: no scattering)
};

template <class T>
void init_ctx(Ctx<T>& c, const orc_geometry* g, const orc_params* P) {
  c.g = g;
  c.P = P;
  for (int r = 0; r < kRows; ++r) c.X[r] = T(g->row_x[r]);
  // curvature per unit q/pT: b = -c Bz, c = 0.00299792458 GeV/(T cm)
  const double bd = -0.00299792458 * double(g->bz_tesla);
  c.b = T(bd);
  c.smax = T(P->s_max);
  c.chi2max = T(P->chi2_max);
  c.kwin = T(P->k_win);
  c.wmax = T(P->w_max);
  c.tanh = T(g->tan_half_angle);
  c.medge = T(P->m_edge);
  c.mz = T(P->m_z);
  c.zmax = T(g->z_max);
  c.sy0 = T(g->sigma_y0);
  c.sy1 = T(g->sigma_y1);
  c.sz0 = T(g->sigma_z0);
  c.sz1 = T(g->sigma_z1);
  c.sy1z = c.sy1 / c.zmax;
  c.sz1z = c.sz1 / c.zmax;
  c.cs0 = T(P->c_s0);
  c.ct0 = T(P->c_t0);
  c.cq0 = T(P->c_q0);
  c.nfw = T(P->nf_window);
  c.nfm = T(P->nf_mmax);
  // k = 13.6 MeV (1 + 0.038 ln(L_ref / X0)) at L_ref = 1 cm, so the
  // variance is linear in the path: theta0^2 = (k^2 / X0) L / (beta p)^2
  if (P->x0_cm > 0.0f) {
    const double x0 = double(P->x0_cm);
    const double k = 0.0136 * (1.0 + 0.038 * std::log(1.0 / x0));
    c.kk = T(k * k / x0);
    c.m2 = T(double(P->ms_mass) * double(P->ms_mass));
  } else {
    c.kk = T(0);
    c.m2 = T(0);
  }
}

// cluster errors sigma(z) = sigma_0 + sigma_1 |z| / z_max, with sigma_1 / z_max
// formed once
template <class T> T sig_y(const Ctx<T>& c, T z) { return c.sy0 + c.sy1z * tabs(z); }
template <class T> T sig_z(const Ctx<T>& c, T z) { return c.sz0 + c.sz1z * tabs(z); }

struct Tracklet {
  int32_t start_id = -1;
  int32_t n = 0;
  int32_t row_in = -1, row_out = -1;
  int32_t r0 = -1;
  bool valid = false;
  uint32_t weight = 0;
  int32_t uhit[kRows];   // outward-phase hits by row (cluster ID, -1 none)
  int32_t dhit[kRows];   // final (inward-phase) hits by row
  double inner_p[5];
  double inner_C[15];
};

struct SectorOut {
  std::vector<Tracklet> tracklets;
  std::vector<orc_track> tracks;       // hit_off relative to hits below
  std::vector<int32_t> hits;
  std::vector<int32_t> starts;
};


template <class R>
struct RefitOut {
  State<R> st;
  int rlast, n;
  R chi2;
};

// One inward pass from the outermost owned row `ro` down to `rmin`.
template <class R>
void refit_pass(const Ctx<R>& c, const float* Y, const float* Z, const int32_t* owned_by_row,
                int ro, int rmin, R s0, R tin, R qin, RefitOut<R>& o) {
  auto y = [&](int32_t id) { return R(Y[id]); };
  auto z = [&](int32_t id) { return R(Z[id]); };
  const int32_t ho = owned_by_row[ro];
  State<R> st;
  st.p[0] = y(ho);
  st.p[1] = z(ho);
  st.p[2] = s0;
  st.p[3] = tin;
  st.p[4] = qin;
  {
    const R sy = sig_y(c, z(ho)), sz = sig_z(c, z(ho));
    for (int i = 0; i < 15; ++i) st.C[i] = R(0);
    st.C[0] = sy * sy;
    st.C[2] = sz * sz;
    st.C[5] = c.cs0;
    st.C[9] = c.ct0;
    st.C[14] = c.cq0;
  }
  o.st = st;
  o.rlast = ro;
  o.n = 1;
  o.chi2 = R(0);
  for (int r = ro - 1; r >= rmin; --r) {
    if (!predict(st, c.X[r] - c.X[r + 1], c.b, c.smax, c.kk, c.m2)) break;
    const int32_t h = owned_by_row[r];
    if (h < 0) continue;
    const R sy = sig_y(c, st.p[1]), sz = sig_z(c, st.p[1]);
    R ch = R(0);
    update(st, y(h), z(h), sy * sy, sz * sz, c.chi2max, c.smax, false, &ch);
    o.chi2 = o.chi2 + ch;
    o.n += 1;
    o.st = st;
    o.rlast = r;
  }
}

// ---- O7: refit over the owned hits, inward, in `passes` passes (3) ---------
// Pass 1 seeds (s, T, Q) from the tracklet's inner state, with s carried to
// the outermost owned row along the circle (sin phi is linear in x) and the
// covariance reset; every owned hit updates the state (no gate); a failed
// transport ends the pass early.  Each later pass repeats the same inward
// fit seeded from the previous pass's result carried back to the outermost
// row the same way, so the transport Jacobians are evaluated along the
// fitted track rather than along the seed.  Output: the last pass's state at
// the innermost fitted hit.
// The refit takes no decision that changes which hits are tried, so it runs
// in double whatever the precision of the tracklet phases (a float covariance
// update loses too much precision when the wide prior collapses over a long
// track).
template <class R>
bool refit_track(const Ctx<R>& c, const float* Y, const float* Z, int sector,
                 const Tracklet& t, const int32_t* owned_by_row, orc_track& out,
                 std::vector<int32_t>& hit_ids, bool replay = false, int passes = 3) {
  int ro = -1, rmin = kRows;
  for (int r = 0; r < kRows; ++r)
    if (owned_by_row[r] >= 0) {
      ro = r;
      rmin = std::min(rmin, r);
    }
  if (ro < 0) return false;
  // In a replay the float run's decisions (range checks, where the fit
  // ended) are taken as given: the hit list is exactly the float track's.
  Ctx<R> cr = c;
  if (replay) cr.smax = R(0.999999);
  RefitOut<R> o;
  {
    const R sin_ = R(t.inner_p[2]), tin = R(t.inner_p[3]), qin = R(t.inner_p[4]);
    const R s0 = sin_ + (c.b * qin) * (c.X[ro] - c.X[t.row_in]);
    if (!(tabs(s0) <= cr.smax)) return false;
    refit_pass(cr, Y, Z, owned_by_row, ro, rmin, s0, tin, qin, o);
  }
  for (int pass = 1; pass < passes; ++pass) {
    const R sin_ = o.st.p[2], tin = o.st.p[3], qin = o.st.p[4];
    const R s0 = sin_ + (c.b * qin) * (c.X[ro] - c.X[o.rlast]);
    if (!(tabs(s0) <= cr.smax)) return false;
    refit_pass(cr, Y, Z, owned_by_row, ro, o.rlast, s0, tin, qin, o);
  }
  if (!replay && o.n < c.P->n_min_track) return false;
  hit_ids.clear();
  for (int r = o.rlast; r <= ro; ++r)
    if (owned_by_row[r] >= 0) hit_ids.push_back(owned_by_row[r]);
  out.sector = sector;
  out.n_hits = o.n;
  out.row_in = o.rlast;
  out.row_out = ro;
  out.hit_off = 0;
  out.inner_id = owned_by_row[o.rlast];
  out.start_id = t.start_id;
  out.x_ref = double(c.X[o.rlast]);
  for (int i = 0; i < 5; ++i) out.par[i] = double(o.st.p[i]);
  for (int i = 0; i < 15; ++i) out.cov[i] = double(o.st.C[i]);
  out.chi2 = double(o.chi2);
  out.ndf = 2 * o.n - 5;
  return true;
}

template <class T>
struct Sector {
  const Ctx<T>& c;
  const Ctx<double>* cd;  // arithmetic of the refit
  int sector;
  bool side_c;
  bool exhaustive;
  const float* Y;
  const float* Z;
  // rows[r]: cluster IDs of this sector in row r, sorted by (y, id)
  std::vector<int32_t> rows[kRows];
  std::vector<int32_t>* up;   // indexed by cluster ID
  std::vector<int32_t>* dn;
  std::vector<int32_t>* upc;
  std::vector<int32_t>* dnc;
  std::vector<int32_t>* rowof;
  std::vector<uint32_t>* wmap;  // weights, indexed by cluster ID (hits of this sector only)

  Sector(const Ctx<T>& cc) : c(cc) {}

  T y(int id) const { return T(Y[id]); }
  T z(int id) const { return T(Z[id]); }

  // Cluster IDs in row r inside the y interval [lo, hi] (a superset of any
  // exact window test; the caller applies the exact test).
  template <class F>
  void for_y_range(int r, T lo, T hi, F&& f) const {
    const std::vector<int32_t>& v = rows[r];
    if (exhaustive) {
      for (int32_t id : v) f(id);
      return;
    }
    auto it = std::lower_bound(v.begin(), v.end(), lo,
                               [&](int32_t id, T val) { return y(id) < val; });
    for (; it != v.end() && !(y(*it) > hi); ++it) f(*it);
  }

  // ---- O2: neighbours finder ------------------------------------------------
  void neighbours() {
    const T W = c.nfw;
    const T margin = T(1e-3);
    for (int r = 1; r + 1 < kRows; ++r) {
      const T rho_d = c.X[r - 1] / c.X[r];
      const T rho_u = c.X[r + 1] / c.X[r];
      const T f = (c.X[r] - c.X[r - 1]) / (c.X[r + 1] - c.X[r - 1]);
      for (int32_t h : rows[r]) {
        const T yh = y(h), zh = z(h);
        const T ypd = yh * rho_d, zpd = zh * rho_d;
        const T ypu = yh * rho_u, zpu = zh * rho_u;
        std::vector<int32_t> dc, uc;
        for_y_range(r - 1, ypd - W - margin, ypd + W + margin, [&](int32_t d) {
          if (tabs(y(d) - ypd) <= W && tabs(z(d) - zpd) <= W) dc.push_back(d);
        });
        for_y_range(r + 1, ypu - W - margin, ypu + W + margin, [&](int32_t u) {
          if (tabs(y(u) - ypu) <= W && tabs(z(u) - zpu) <= W) uc.push_back(u);
        });
        if (dc.empty() || uc.empty()) continue;
        const T sy = sig_y(c, zh), sz = sig_z(c, zh);
        const T wy = T(1) / (T(1.5) * (sy * sy));
        const T wz = T(1) / (T(1.5) * (sz * sz));
        bool have = false;
        T best = T(0);
        int32_t bd = -1, bu = -1;
        for (int32_t d : dc) {
          for (int32_t u : uc) {
            const T dy = y(d) + (y(u) - y(d)) * f - yh;
            const T dz = z(d) + (z(u) - z(d)) * f - zh;
            const T m = dy * dy * wy + dz * dz * wz;
            bool better = !have || m < best || (m == best && (d < bd || (d == bd && u < bu)));
            if (better) {
              have = true;
              best = m;
              bd = d;
              bu = u;
            }
          }
        }
        if (have && best <= c.nfm) {
          (*up)[h] = bu;
          (*dn)[h] = bd;
        }
      }
    }
  }

  // ---- O3: cleaner (reads only the pre-clean links) -------------------------
  void clean() {
    for (int r = 0; r < kRows; ++r)
      for (int32_t h : rows[r]) {
        const int32_t u = (*up)[h], d = (*dn)[h];
        (*upc)[h] = (u >= 0 && (*dn)[u] == h) ? u : -1;
        (*dnc)[h] = (d >= 0 && (*up)[d] == h) ? d : -1;
      }
  }

  // ---- O4: start hits: a cleaned chain of >= n_min_chain hits begins here ----
  // (no cleaned down link; following the cleaned up links reaches
  // n_min_chain hits in all)
  void starts(std::vector<int32_t>& out) const {
    for (int r = 0; r < kRows; ++r)
      for (int32_t h : rows[r]) {
        if ((*dnc)[h] >= 0 || (*upc)[h] < 0) continue;
        int n = 1;
        int32_t k = h;
        while (n < c.P->n_min_chain && (*upc)[k] >= 0) {
          k = (*upc)[k];
          ++n;
        }
        if (n >= c.P->n_min_chain) out.push_back(h);
      }
    std::sort(out.begin(), out.end());
  }

  // Stop rules after a predict to row r: left the sector sideways, crossed
  // the membrane, or left the drift volume.
  bool inside(const State<T>& st, int r) const {
    if (!(tabs(st.p[0]) <= c.X[r] * c.tanh + c.medge)) return false;
    if (!(tabs(st.p[1]) <= c.zmax + c.mz)) return false;
    if (side_c ? (st.p[1] > c.mz) : (st.p[1] < -c.mz)) return false;
    return true;
  }

  void prior(State<T>& st, T zv) const {
    const T sy = sig_y(c, zv), sz = sig_z(c, zv);
    for (int i = 0; i < 15; ++i) st.C[i] = T(0);
    st.C[0] = sy * sy;
    st.C[2] = sz * sz;
    st.C[5] = c.cs0;
    st.C[9] = c.ct0;
    st.C[14] = c.cq0;
  }

  // Best hit of row r for the predicted state: inside the window
  // |r_y| <= min(k sqrt(S_yy), w_max) (same for z), smallest chi2, ties to the
  // smaller cluster ID.  Returns -1 if the window is empty.
  int32_t search(const State<T>& st, int r, T vy, T vz) const {
    const Gain2<T> g = weights(st, vy, vz);
    T wy = c.kwin * tsqrt(g.s00);
    if (wy > c.wmax) wy = c.wmax;
    T wz = c.kwin * tsqrt(g.s11);
    if (wz > c.wmax) wz = c.wmax;
    const T yc = st.p[0], zc = st.p[1];
    int32_t best = -1;
    T bchi = T(0);
    for_y_range(r, yc - wy - T(1e-3), yc + wy + T(1e-3), [&](int32_t id) {
      const T ry = y(id) - yc, rz = z(id) - zc;
      if (!(tabs(ry) <= wy && tabs(rz) <= wz)) return;
      const T ch = chi2_of(g, ry, rz);
      if (best < 0 || ch < bchi || (ch == bchi && id < best)) {
        best = id;
        bchi = ch;
      }
    });
    return best;
  }

  bool try_hit(State<T>& st, int32_t id, T vy, T vz) const {
    return update(st, y(id), z(id), vy, vz, c.chi2max, c.smax, true, (T*)nullptr);
  }

  // ---- O5: tracklet from start hit h0 ---------------------------------------
  void tracklet(int32_t h0, Tracklet& t) const {
    for (int r = 0; r < kRows; ++r) t.uhit[r] = t.dhit[r] = -1;
    t.start_id = h0;
    const int r0 = (*rowof)[h0];
    t.r0 = r0;
    const int32_t h1 = (*upc)[h0];
    State<T> st;
    {
      const T dx = c.X[r0 + 1] - c.X[r0];
      const T dy = y(h1) - y(h0);
      const T dz = z(h1) - z(h0);
      const T L = tsqrt(dx * dx + dy * dy);
      st.p[0] = y(h0);
      st.p[1] = z(h0);
      st.p[2] = dy / L;
      st.p[3] = dz / L;
      st.p[4] = T(0);
      prior(st, z(h0));
    }
    t.uhit[r0] = h0;
    // Phase U: outward
    State<T> last = st;
    int rout = r0;
    int32_t cur = h0;
    bool chain = true;
    int miss = 0;
    for (int r = r0 + 1; r < kRows; ++r) {
      if (!predict(st, c.X[r] - c.X[r - 1], c.b, c.smax, c.kk, c.m2)) break;
      if (!inside(st, r)) break;
      const T sy = sig_y(c, st.p[1]), sz = sig_z(c, st.p[1]);
      const T vy = sy * sy, vz = sz * sz;
      int32_t got = -1;
      if (chain) {
        const int32_t nx = (*upc)[cur];
        if (nx >= 0 && try_hit(st, nx, vy, vz)) got = nx;
        else chain = false;
      }
      if (got < 0) {
        const int32_t bh = search(st, r, vy, vz);
        if (bh >= 0 && try_hit(st, bh, vy, vz)) got = bh;
      }
      if (got >= 0) {
        t.uhit[r] = got;
        cur = got;
        miss = 0;
        last = st;
        rout = r;
      } else if (++miss >= c.P->n_gap) {
        break;
      }
    }
    // Phase D: inward from the outermost hit with the covariance reset
    const int32_t hout = t.uhit[rout];
    st = last;
    st.p[0] = y(hout);
    st.p[1] = z(hout);
    prior(st, z(hout));
    t.dhit[rout] = hout;
    int n = 1;
    int rin = rout;
    last = st;
    miss = 0;
    for (int r = rout - 1; r >= 0; --r) {
      if (!predict(st, c.X[r] - c.X[r + 1], c.b, c.smax, c.kk, c.m2)) break;
      if (!inside(st, r)) break;
      const T sy = sig_y(c, st.p[1]), sz = sig_z(c, st.p[1]);
      const T vy = sy * sy, vz = sz * sz;
      int32_t got = -1;
      const int32_t uh = t.uhit[r];
      if (uh >= 0 && try_hit(st, uh, vy, vz)) got = uh;
      if (got < 0) {
        const int32_t bh = search(st, r, vy, vz);
        if (bh >= 0 && try_hit(st, bh, vy, vz)) got = bh;
      }
      if (got >= 0) {
        t.dhit[r] = got;
        ++n;
        miss = 0;
        last = st;
        rin = r;
      } else if (++miss >= c.P->n_gap) {
        break;
      }
    }
    t.n = n;
    t.row_in = rin;
    t.row_out = rout;
    t.valid = n >= c.P->n_min_tracklet;
    t.weight = (uint32_t(n) << 24) | (0xFFFFFFu - uint32_t(h0));
    for (int i = 0; i < 5; ++i) t.inner_p[i] = double(last.p[i]);
    for (int i = 0; i < 15; ++i) t.inner_C[i] = double(last.C[i]);
  }

  void run(SectorOut& so) {
    neighbours();
    clean();
    starts(so.starts);
    so.tracklets.resize(so.starts.size());
    for (size_t i = 0; i < so.starts.size(); ++i) tracklet(so.starts[i], so.tracklets[i]);
    // ---- O6: hit weights = max over valid tracklets; ownership -------------
    for (const Tracklet& t : so.tracklets) {
      if (!t.valid) continue;
      for (int r = 0; r < kRows; ++r)
        if (t.dhit[r] >= 0) (*wmap)[t.dhit[r]] = std::max((*wmap)[t.dhit[r]], t.weight);
    }
    std::vector<int32_t> owned(kRows), ids;
    for (size_t i = 0; i < so.tracklets.size(); ++i) {
      const Tracklet& t = so.tracklets[i];
      if (!t.valid) continue;
      int cnt = 0;
      for (int r = 0; r < kRows; ++r) {
        const int32_t h = t.dhit[r];
        owned[r] = (h >= 0 && (*wmap)[h] == t.weight) ? h : -1;
        cnt += owned[r] >= 0;
      }
      if (cnt < c.P->n_min_track) continue;
      orc_track tr;
      if (!refit_track(*cd, Y, Z, sector, t, owned.data(), tr, ids)) continue;
      tr.tracklet = int32_t(i);
      tr.hit_off = int64_t(so.hits.size());
      so.hits.insert(so.hits.end(), ids.begin(), ids.end());
      so.tracks.push_back(tr);
    }
  }
};

// ---------------------------------------------------------------------------
// Cross-sector merger.  A particle crossing the boundary between two
// neighbouring sectors of one side, or the central membrane between the
// two sectors of one azimuth, leaves one track segment in each; the
// per-sector tracker fits them separately.  The merger joins such segments
// and refits the joined hit list across the sector frames.  The paper names
// this step only as the continuation of the per-sector tracking; the
// definition below is this project's:
//  M1 every track's state at its outermost hit, from one outward Kalman pass
//     over its hits seeded with its fitted parameters at the innermost hit
//     and the prior covariance;
//  M2 a pair (A, B) of tracks of one event, B in a neighbouring sector of
//     A's side or in the sector across the membrane from A's (same
//     azimuth, same frame), with 0 < B.row_in - A.row_out <= row_gap, is
//     compatible if A's outer state, turned into B's frame (no turn across
//     the membrane) and transported to B's innermost row, matches B's
//     fitted state: chi2 = d^T (C_A + C_B)^-1 d
//     over the 5 parameters (Cholesky) <= chi2_max.  T and Q do not change
//     under rotation or transport, and d_i^2 / S_ii never exceeds the full
//     chi2, so pairs failing the cut on T or Q alone are skipped before any
//     transport;
//  M3 each A keeps its best B (smallest chi2, ties to the smaller track
//     index) and each B its best A; a pair is linked if each is the other's
//     best; links form chains inner -> outer;
//  M4 every chain of two or more segments is refitted inward over all its
//     hits (passes as in the per-sector refit: the first seeded with the
//     outermost segment's outer state, each later one with the previous
//     result carried out to the outermost hit), turning frames at the
//     boundaries; a chain whose transport fails (or whose outermost segment
//     has no outer state) is left unmerged.  Output at
//     the innermost hit, in the innermost segment's frame.
// The frame of sector k is turned by 2 atan(tan_half_angle) from that of
// sector k - 1; its cosine and sine are formed algebraically from the tangent.
// All transports of the merger stop only beyond its own s_max.
// ---------------------------------------------------------------------------

// The state at x in one frame, expressed in the frame turned by the angle
// with cosine ca and sine sa (the new x axis at azimuth +a): the point and
// direction are unchanged, x' = x ca + y sa, y' = -x sa + y ca,
// sin phi' = sin(phi - a).  The covariance is carried to the new x' along
// the track: J(y', y) = ca - sa tan phi', J(z', y) = -sa T / cos phi',
// J(s', y) = -b Q sa, J(s', s) = cos phi' / cos phi.  Returns false if
// |sin phi'| would exceed s_max.
template <class T>
bool rotate(State<T>& st, T& x, T ca, T sa, T b, T smax) {
  const T y = st.p[0], s = st.p[2], tl = st.p[3], q = st.p[4];
  const T c = tsqrt(T(1) - s * s);
  const T s1 = s * ca - c * sa;
  if (!(tabs(s1) <= smax)) return false;
  const T c1 = tsqrt(T(1) - s1 * s1);
  const T x1 = x * ca + y * sa;
  const T y1 = -x * sa + y * ca;
  T J[5][5] = {};
  for (int i = 0; i < 5; ++i) J[i][i] = T(1);
  J[0][0] = ca - sa * (s1 / c1);
  J[1][0] = -sa * tl / c1;
  J[2][0] = -(b * q) * sa;
  J[2][2] = c1 / c;
  T Cf[5][5];
  for (int i = 0, k = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j, ++k) Cf[i][j] = Cf[j][i] = st.C[k];
  T A[5][5];
  for (int i = 0; i < 5; ++i)
    for (int l = 0; l < 5; ++l) {
      T a = T(0);
      for (int k = 0; k < 5; ++k) a = a + J[i][k] * Cf[k][l];
      A[i][l] = a;
    }
  for (int i = 0, k = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j, ++k) {
      T v = T(0);
      for (int l = 0; l < 5; ++l) v = v + A[i][l] * J[j][l];
      st.C[k] = v;
    }
  st.p[0] = y1;
  st.p[2] = s1;
  x = x1;
  return true;
}

// Transport from x to xt in equal steps no longer than step_max (refused
// beyond 1000 cm: no path inside the chamber is that long).
template <class T>
bool transport_to(State<T>& st, T x, T xt, T b, T smax, T step_max, T kk = T(0), T m2 = T(0)) {
  const T d = xt - x;
  if (!(tabs(d) <= T(1000))) return false;
  const int n = std::max(1, int(std::ceil(tabs(d) / step_max)));
  const T dx = d / T(n);
  for (int i = 0; i < n; ++i)
    if (!predict(st, dx, b, smax, kk, m2)) return false;
  return true;
}

// chi2 = d^T S^-1 d for a symmetric positive definite S (lower triangle,
// packed like C), by Cholesky.  Returns false if S is not positive definite.
template <class T>
bool chi2_5(const T* S, const T* d, T& chi2) {
  T L[5][5] = {};
  for (int i = 0, k = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j, ++k) L[i][j] = S[k];
  for (int j = 0; j < 5; ++j) {
    T v = L[j][j];
    for (int k = 0; k < j; ++k) v = v - L[j][k] * L[j][k];
    if (!(v > T(0))) return false;
    const T ljj = tsqrt(v);
    L[j][j] = ljj;
    for (int i = j + 1; i < 5; ++i) {
      T w = L[i][j];
      for (int k = 0; k < j; ++k) w = w - L[i][k] * L[j][k];
      L[i][j] = w / ljj;
    }
  }
  T yv[5];
  T sum = T(0);
  for (int i = 0; i < 5; ++i) {
    T w = d[i];
    for (int k = 0; k < i; ++k) w = w - L[i][k] * yv[k];
    yv[i] = w / L[i][i];
    sum = sum + yv[i] * yv[i];
  }
  chi2 = sum;
  return true;
}

struct MergeIn {
  const orc_track* tracks;   // one event's tracks, canonical order
  int64_t n_tracks;
  const int32_t* hits;       // hit IDs, hit_off into this
  const uint8_t* row;        // pad row of each cluster ID
  const float* Y;
  const float* Z;
};

struct MergeOut {
  std::vector<orc_track> tracks;     // canonical order
  std::vector<int32_t> hits;
  std::vector<int32_t> n_segments;
  std::vector<int32_t> link_out;     // per input track: linked outer segment or -1
  std::vector<double> best_chi2;     // per input track: chi2 of its best outer partner
  std::vector<int32_t> best_out;     // per input track: best outer partner or -1
  std::vector<int32_t> merged_into;  // per input track: output track index
};

struct Merger {
  Ctx<double> c;
  orc_merge_params M;
  double ca, sa;          // rotation between neighbouring sectors
  const MergeIn& in;

  Merger(const orc_geometry* g, const orc_params* P, const orc_merge_params* m, const MergeIn& i)
      : M(*m), in(i) {
    init_ctx(c, g, P);
    c.smax = double(m->s_max);
    const double t = double(g->tan_half_angle);
    ca = (1.0 - t * t) / (1.0 + t * t);
    sa = (2.0 * t) / (1.0 + t * t);
  }

  void prior(State<double>& st, double zv) const {
    for (int i = 0; i < 15; ++i) st.C[i] = 0.0;
    const double sy = sig_y(c, zv), sz = sig_z(c, zv);
    st.C[0] = sy * sy;
    st.C[2] = sz * sz;
    st.C[5] = c.cs0;
    st.C[9] = c.ct0;
    st.C[14] = c.cq0;
  }

  // M1
  bool outer_state(const orc_track& t, State<double>& st) const {
    for (int i = 0; i < 5; ++i) st.p[i] = t.par[i];
    prior(st, st.p[1]);
    const int32_t* h = in.hits + t.hit_off;
    int k = 1;
    for (int r = t.row_in + 1; r <= t.row_out; ++r) {
      if (!predict(st, c.X[r] - c.X[r - 1], c.b, c.smax, c.kk, c.m2)) return false;
      if (k < t.n_hits && int(in.row[h[k]]) == r) {
        const double sy = sig_y(c, st.p[1]), sz = sig_z(c, st.p[1]);
        update(st, double(in.Y[h[k]]), double(in.Z[h[k]]), sy * sy, sz * sz, c.chi2max, c.smax,
               false, (double*)nullptr);
        ++k;
      }
    }
    return true;
  }

  // +1 if sector b follows a counter-clockwise on its side (frame turned by
  // +a), -1 if it precedes it, kMembrane if b is across the membrane from a
  // (same azimuth: the same frame), 0 otherwise.
  static constexpr int kMembrane = 2;
  static int neighbour(int a, int b) {
    const int ka = a % 18, kb = b % 18;
    if (a / 18 != b / 18) return ka == kb ? kMembrane : 0;
    if (kb == (ka + 1) % 18) return 1;
    if (ka == (kb + 1) % 18) return -1;
    return 0;
  }
  // the frame of sector b from that of sector a (neighbour(a, b) = dir != 0)
  bool turn(State<double>& st, double& x, int dir) const {
    if (dir == kMembrane) return true;
    return rotate(st, x, ca, double(dir) * sa, c.b, c.smax);
  }

  // M2: chi2 of the pair (outer state of A, track B), false if incompatible
  bool pair_chi2(const orc_track& A, const State<double>& outA, const orc_track& B,
                 double& chi2) const {
    const int dir = neighbour(A.sector, B.sector);
    if (dir == 0) return false;
    if (!(B.row_in > A.row_out && B.row_in - A.row_out <= M.row_gap)) return false;
    const double cut = double(M.chi2_max);
    const double dT = outA.p[3] - B.par[3], dQ = outA.p[4] - B.par[4];
    if (dT * dT > cut * (outA.C[9] + B.cov[9])) return false;
    if (dQ * dQ > cut * (outA.C[14] + B.cov[14])) return false;
    State<double> st = outA;
    double x = c.X[A.row_out];
    if (!turn(st, x, dir)) return false;
    if (!transport_to(st, x, c.X[B.row_in], c.b, c.smax, double(M.step_max), c.kk, c.m2)) return false;
    double d[5], S[15];
    for (int i = 0; i < 5; ++i) d[i] = st.p[i] - B.par[i];
    for (int i = 0; i < 15; ++i) S[i] = st.C[i] + B.cov[i];
    if (!chi2_5(S, d, chi2)) return false;
    return chi2 <= cut;
  }

  struct Seg {
    int sector;
    std::vector<int32_t> hits;   // ascending rows
  };

  // One inward pass over the chain (segments inner -> outer) seeded with
  // (s, T, Q) at the outermost hit.
  bool chain_pass(const std::vector<Seg>& segs, double s0, double t0, double q0,
                  State<double>& out, double& chi2, int& n) const {
    const Seg& last = segs.back();
    const int32_t ho = last.hits.back();
    State<double> st;
    st.p[0] = double(in.Y[ho]);
    st.p[1] = double(in.Z[ho]);
    st.p[2] = s0;
    st.p[3] = t0;
    st.p[4] = q0;
    prior(st, st.p[1]);
    chi2 = 0.0;
    n = 1;
    int cur_row = in.row[ho];
    for (int j = int(segs.size()) - 1; j >= 0; --j) {
      const Seg& sg = segs[j];
      int k = int(sg.hits.size()) - 1;
      if (j == int(segs.size()) - 1) {
        --k;                                  // the outermost hit seeded the pass
      } else {
        const int dir = neighbour(segs[j + 1].sector, sg.sector);   // outer -> inner frame
        double x = c.X[cur_row];
        if (!turn(st, x, dir)) return false;
        const int r = in.row[sg.hits[k]];
        if (!transport_to(st, x, c.X[r], c.b, c.smax, double(M.step_max), c.kk, c.m2)) return false;
        const double sy = sig_y(c, st.p[1]), sz = sig_z(c, st.p[1]);
        double ch = 0.0;
        update(st, double(in.Y[sg.hits[k]]), double(in.Z[sg.hits[k]]), sy * sy, sz * sz,
               c.chi2max, c.smax, false, &ch);
        chi2 += ch;
        ++n;
        cur_row = r;
        --k;
      }
      for (; k >= 0; --k) {
        const int32_t h = sg.hits[k];
        const int r = in.row[h];
        for (int rr = cur_row - 1; rr >= r; --rr)
          if (!predict(st, c.X[rr] - c.X[rr + 1], c.b, c.smax, c.kk, c.m2)) return false;
        const double sy = sig_y(c, st.p[1]), sz = sig_z(c, st.p[1]);
        double ch = 0.0;
        update(st, double(in.Y[h]), double(in.Z[h]), sy * sy, sz * sz, c.chi2max, c.smax, false,
               &ch);
        chi2 += ch;
        ++n;
        cur_row = r;
      }
    }
    out = st;
    return true;
  }

  // Carry the inner result of a pass out to the outermost hit (parameters
  // only matter: the next pass resets the covariance).
  bool carry_out(const std::vector<Seg>& segs, State<double> st, double& s0, double& t0,
                 double& q0) const {
    double x = c.X[in.row[segs[0].hits.front()]];
    for (size_t j = 0; j < segs.size(); ++j) {
      const double xo = c.X[in.row[segs[j].hits.back()]];
      if (!transport_to(st, x, xo, c.b, c.smax, double(M.step_max), c.kk, c.m2)) return false;
      x = xo;
      if (j + 1 < segs.size()) {
        if (!turn(st, x, neighbour(segs[j].sector, segs[j + 1].sector))) return false;
      }
    }
    s0 = st.p[2];
    t0 = st.p[3];
    q0 = st.p[4];
    return true;
  }

  void run(MergeOut& o) const {
    const int64_t n = in.n_tracks;
    std::vector<State<double>> outer(n);
    std::vector<char> ok(n, 0);
    for (int64_t i = 0; i < n; ++i) ok[i] = outer_state(in.tracks[i], outer[i]) ? 1 : 0;
    // M2 + M3: best partners both ways
    std::vector<int32_t> best_out(n, -1), best_in(n, -1);
    std::vector<double> chi_out(n, 0.0), chi_in(n, 0.0);
    std::vector<std::vector<int32_t>> by_sector(36);
    for (int64_t i = 0; i < n; ++i) by_sector[in.tracks[i].sector].push_back(int32_t(i));
    for (int64_t a = 0; a < n; ++a) {
      if (!ok[a]) continue;
      const int sa_ = in.tracks[a].sector;
      const int side = sa_ / 18, k = sa_ % 18;
      for (int sb : {side * 18 + (k + 1) % 18, side * 18 + (k + 17) % 18, (1 - side) * 18 + k}) {
        for (int32_t bi : by_sector[sb]) {
          double ch;
          if (!pair_chi2(in.tracks[a], outer[a], in.tracks[bi], ch)) continue;
          if (best_out[a] < 0 || ch < chi_out[a] || (ch == chi_out[a] && bi < best_out[a])) {
            best_out[a] = bi;
            chi_out[a] = ch;
          }
          if (best_in[bi] < 0 || ch < chi_in[bi] || (ch == chi_in[bi] && a < best_in[bi])) {
            best_in[bi] = int32_t(a);
            chi_in[bi] = ch;
          }
        }
      }
    }
    o.best_out = best_out;
    o.best_chi2 = chi_out;
    o.link_out.assign(n, -1);
    std::vector<int32_t> link_in(n, -1);
    for (int64_t a = 0; a < n; ++a) {
      const int32_t bi = best_out[a];
      if (bi >= 0 && best_in[bi] == a) {
        o.link_out[a] = bi;
        link_in[bi] = int32_t(a);
      }
    }
    // M4: chains from their innermost segment
    struct Out {
      orc_track t;
      std::vector<int32_t> hits;
      int32_t nseg;
      std::vector<int32_t> members;
    };
    std::vector<Out> outs;
    std::vector<char> used(n, 0);
    for (int64_t a = 0; a < n; ++a) {
      if (link_in[a] >= 0) continue;            // not a chain head
      std::vector<int32_t> chain{int32_t(a)};
      while (o.link_out[chain.back()] >= 0) chain.push_back(o.link_out[chain.back()]);
      bool merged = false;
      Out m;
      if (chain.size() > 1) {
        std::vector<Seg> segs;
        for (int32_t k : chain) {
          const orc_track& t = in.tracks[k];
          segs.push_back({t.sector, std::vector<int32_t>(in.hits + t.hit_off,
                                                         in.hits + t.hit_off + t.n_hits)});
        }
        const State<double>& so = outer[chain.back()];
        double s0 = so.p[2], t0 = so.p[3], q0 = so.p[4];
        State<double> res;
        double chi2 = 0.0;
        int nh = 0;
        bool good = ok[chain.back()] != 0;     // the seed must exist
        for (int pass = 0; pass < M.passes && good; ++pass) {
          if (pass > 0) good = carry_out(segs, res, s0, t0, q0);
          if (good) good = chain_pass(segs, s0, t0, q0, res, chi2, nh);
        }
        if (good) {
          const orc_track& t0r = in.tracks[chain.front()];
          const orc_track& tl = in.tracks[chain.back()];
          m.t = t0r;
          m.t.n_hits = nh;
          m.t.row_out = tl.row_out;
          for (int i = 0; i < 5; ++i) m.t.par[i] = res.p[i];
          for (int i = 0; i < 15; ++i) m.t.cov[i] = res.C[i];
          m.t.chi2 = chi2;
          m.t.ndf = 2 * nh - 5;
          for (const Seg& sg : segs) m.hits.insert(m.hits.end(), sg.hits.begin(), sg.hits.end());
          m.nseg = int32_t(chain.size());
          m.members = chain;
          outs.push_back(std::move(m));
          merged = true;
        }
      }
      if (!merged) {
        for (int32_t k : chain) {
          Out u;
          u.t = in.tracks[k];
          u.hits.assign(in.hits + u.t.hit_off, in.hits + u.t.hit_off + u.t.n_hits);
          u.nseg = 1;
          u.members = {k};
          outs.push_back(std::move(u));
        }
      }
    }
    std::sort(outs.begin(), outs.end(),
              [](const Out& x, const Out& y) { return x.t.inner_id < y.t.inner_id; });
    o.tracks.clear();
    o.hits.clear();
    o.n_segments.clear();
    o.merged_into.assign(n, -1);
    for (size_t i = 0; i < outs.size(); ++i) {
      Out& u = outs[i];
      u.t.hit_off = int64_t(o.hits.size());
      o.hits.insert(o.hits.end(), u.hits.begin(), u.hits.end());
      o.tracks.push_back(u.t);
      o.n_segments.push_back(u.nseg);
      for (int32_t k : u.members) o.merged_into[k] = int32_t(i);
    }
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------

struct OrcResult {
  int precision;
  std::vector<int32_t> up, dn, upc, dnc;
  std::vector<int32_t> starts;                   // all sectors, sector-major
  std::vector<std::vector<Tracklet>> tracklets;  // per sector
  std::vector<orc_track> tracks;                 // canonical order
  std::vector<int32_t> hits;
  std::vector<int32_t> rowof;
  orc_geometry g;
  orc_params P;
  std::vector<float> Y, Z;
};


// ---------------------------------------------------------------------------
// Replay: every Kalman state of a float run's track recomputed in double
// along that run's decisions: the seed pair, the rows where the outward and
// the inward phase updated and with which hit, and the refit's hit list.
// ---------------------------------------------------------------------------

static bool replay_one(const OrcResult& R, const Ctx<double>& c, const orc_track& ft,
                       orc_track& out) {
  const Tracklet& t = R.tracklets[ft.sector][ft.tracklet];
  auto y = [&](int32_t id) { return double(R.Y[id]); };
  auto z = [&](int32_t id) { return double(R.Z[id]); };
  auto var = [&](double zz, double& vy, double& vz) {
    const double sy = sig_y(c, zz), sz = sig_z(c, zz);
    vy = sy * sy;
    vz = sz * sz;
  };
  auto prior = [&](State<double>& st, double zv) {
    for (int i = 0; i < 15; ++i) st.C[i] = 0.0;
    double vy, vz;
    var(zv, vy, vz);
    st.C[0] = vy;
    st.C[2] = vz;
    st.C[5] = c.cs0;
    st.C[9] = c.ct0;
    st.C[14] = c.cq0;
  };
  const int r0 = t.r0;
  const int32_t h0 = t.start_id;
  const int32_t h1 = R.upc[h0];
  State<double> st;
  {
    const double dx = c.X[r0 + 1] - c.X[r0];
    const double dy = y(h1) - y(h0), dz = z(h1) - z(h0);
    const double L = std::sqrt(dx * dx + dy * dy);
    st.p[0] = y(h0);
    st.p[1] = z(h0);
    st.p[2] = dy / L;
    st.p[3] = dz / L;
    st.p[4] = 0.0;
    prior(st, z(h0));
  }
  bool ok = true;
  for (int r = r0 + 1; r <= t.row_out; ++r) {
    ok = ok && predict(st, c.X[r] - c.X[r - 1], c.b, 10.0, c.kk, c.m2);
    const int32_t h = t.uhit[r];
    if (h < 0) continue;
    double vy, vz;
    var(st.p[1], vy, vz);
    update(st, y(h), z(h), vy, vz, 0.0, 10.0, false, (double*)nullptr);
  }
  const int32_t hout = t.uhit[t.row_out];
  st.p[0] = y(hout);
  st.p[1] = z(hout);
  prior(st, z(hout));
  for (int r = t.row_out - 1; r >= t.row_in; --r) {
    ok = ok && predict(st, c.X[r] - c.X[r + 1], c.b, 10.0, c.kk, c.m2);
    const int32_t h = t.dhit[r];
    if (h < 0) continue;
    double vy, vz;
    var(st.p[1], vy, vz);
    update(st, y(h), z(h), vy, vz, 0.0, 10.0, false, (double*)nullptr);
  }
  // refit (double) along the float track's hit list from the replayed seed
  Tracklet tr = t;
  for (int i = 0; i < 5; ++i) tr.inner_p[i] = st.p[i];
  const int32_t* hits = R.hits.data() + ft.hit_off;
  std::vector<int32_t> byrow(kRows, -1), ids;
  for (int k = 0; k < ft.n_hits; ++k) byrow[R.rowof[hits[k]]] = hits[k];
  if (!refit_track(c, R.Y.data(), R.Z.data(), ft.sector, tr, byrow.data(), out, ids, true)) return false;
  out.hit_off = ft.hit_off;
  out.tracklet = ft.tracklet;
  ok = ok && out.n_hits == ft.n_hits;
  return ok;
}

template <class T>
static void run_all(OrcResult& R, int64_t n, const uint8_t* sec, const uint8_t* row,
                    const float* y, const float* z, int exhaustive, int nthreads) {
  Ctx<T> c;
  init_ctx(c, &R.g, &R.P);
  Ctx<double> cd;
  init_ctx(cd, &R.g, &R.P);
  const int ns = R.g.n_sectors;
  R.up.assign(n, -1);
  R.dn.assign(n, -1);
  R.upc.assign(n, -1);
  R.dnc.assign(n, -1);
  std::vector<int32_t>& rowof = R.rowof;
  rowof.assign(n, 0);
  std::vector<uint32_t> wmap(n, 0u);
  std::vector<std::vector<int32_t>> bysec(ns);
  for (int64_t i = 0; i < n; ++i) {
    rowof[i] = row[i];
    bysec[sec[i]].push_back(int32_t(i));
  }
  std::vector<SectorOut> outs(ns);
  std::atomic<int> next(0);
  auto worker = [&]() {
    for (;;) {
      const int s = next.fetch_add(1);
      if (s >= ns) break;
      Sector<T> S(c);
      S.sector = s;
      S.cd = &cd;
      S.side_c = s >= ns / 2;
      S.exhaustive = exhaustive != 0;
      S.Y = y;
      S.Z = z;
      S.up = &R.up;
      S.dn = &R.dn;
      S.upc = &R.upc;
      S.dnc = &R.dnc;
      S.rowof = &rowof;
      S.wmap = &wmap;
      for (int32_t id : bysec[s]) S.rows[row[id]].push_back(id);
      for (int r = 0; r < kRows; ++r)
        std::sort(S.rows[r].begin(), S.rows[r].end(), [&](int32_t a, int32_t b) {
          return y[a] < y[b] || (y[a] == y[b] && a < b);
        });
      S.run(outs[s]);
    }
  };
  const int nt = std::max(1, nthreads);
  if (nt == 1) {
    worker();
  } else {
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(worker);
    for (auto& t : th) t.join();
  }
  // gather and order tracks by the cluster ID of the innermost hit
  R.tracklets.resize(ns);
  std::vector<std::pair<int32_t, std::pair<int, int>>> order;
  for (int s = 0; s < ns; ++s) {
    R.starts.insert(R.starts.end(), outs[s].starts.begin(), outs[s].starts.end());
    for (size_t k = 0; k < outs[s].tracks.size(); ++k)
      order.push_back({outs[s].tracks[k].inner_id, {s, int(k)}});
  }
  std::sort(order.begin(), order.end());
  for (auto& o : order) {
    const SectorOut& so = outs[o.second.first];
    orc_track t = so.tracks[o.second.second];
    const int32_t* h = so.hits.data() + t.hit_off;
    t.hit_off = int64_t(R.hits.size());
    R.hits.insert(R.hits.end(), h, h + t.n_hits);
    R.tracks.push_back(t);
  }
  for (int s = 0; s < ns; ++s) R.tracklets[s] = std::move(outs[s].tracklets);
}

extern "C" {

void* orc_run(const orc_geometry* g, const orc_params* P, int precision, int64_t n,
              const uint8_t* sector, const uint8_t* row, const float* y, const float* z,
              int exhaustive, int nthreads) {
  OrcResult* R = new OrcResult();
  R->precision = precision;
  R->g = *g;
  R->P = *P;
  R->Y.assign(y, y + n);
  R->Z.assign(z, z + n);
  if (precision == 64)
    run_all<double>(*R, n, sector, row, y, z, exhaustive, nthreads);
  else
    run_all<float>(*R, n, sector, row, y, z, exhaustive, nthreads);
  return R;
}

void orc_free(void* h) { delete static_cast<OrcResult*>(h); }

int64_t orc_n_tracks(void* h) { return int64_t(static_cast<OrcResult*>(h)->tracks.size()); }
int64_t orc_n_track_hits(void* h) { return int64_t(static_cast<OrcResult*>(h)->hits.size()); }
int64_t orc_n_starts(void* h) { return int64_t(static_cast<OrcResult*>(h)->starts.size()); }

void orc_get_links(void* h, int32_t* up, int32_t* dn, int32_t* upc, int32_t* dnc) {
  OrcResult* R = static_cast<OrcResult*>(h);
  const size_t n = R->up.size();
  std::memcpy(up, R->up.data(), n * 4);
  std::memcpy(dn, R->dn.data(), n * 4);
  std::memcpy(upc, R->upc.data(), n * 4);
  std::memcpy(dnc, R->dnc.data(), n * 4);
}

void orc_get_starts(void* h, int32_t* out) {
  OrcResult* R = static_cast<OrcResult*>(h);
  std::memcpy(out, R->starts.data(), R->starts.size() * 4);
}

void orc_get_tracks(void* h, orc_track* out, int32_t* hit_ids) {
  OrcResult* R = static_cast<OrcResult*>(h);
  std::memcpy(out, R->tracks.data(), R->tracks.size() * sizeof(orc_track));
  std::memcpy(hit_ids, R->hits.data(), R->hits.size() * 4);
}

// Double-precision replay of every track of a float run (same order, same
// hit lists).  Returns the number of tracks whose replayed transport left the
// valid range (expected 0).
int64_t orc_replay_tracks(void* h, orc_track* out) {
  OrcResult* R = static_cast<OrcResult*>(h);
  Ctx<double> c;
  init_ctx(c, &R->g, &R->P);
  int64_t bad = 0;
  for (size_t k = 0; k < R->tracks.size(); ++k)
    bad += replay_one(*R, c, R->tracks[k], out[k]) ? 0 : 1;
  return bad;
}

// Tracklets of one sector: start IDs, n, row_in, row_out, valid, weight and
// the per-row hit arrays (outward phase and final).
int64_t orc_n_tracklets(void* h, int sector) {
  return int64_t(static_cast<OrcResult*>(h)->tracklets[sector].size());
}

void orc_get_tracklets(void* h, int sector, int32_t* info /* [n,6] */, uint32_t* weight,
                       int32_t* uhit /* [n,159] */, int32_t* dhit /* [n,159] */) {
  OrcResult* R = static_cast<OrcResult*>(h);
  const auto& v = R->tracklets[sector];
  for (size_t i = 0; i < v.size(); ++i) {
    info[6 * i + 0] = v[i].start_id;
    info[6 * i + 1] = v[i].n;
    info[6 * i + 2] = v[i].row_in;
    info[6 * i + 3] = v[i].row_out;
    info[6 * i + 4] = v[i].valid ? 1 : 0;
    info[6 * i + 5] = v[i].r0;
    weight[i] = v[i].weight;
    std::memcpy(uhit + 159 * i, v[i].uhit, 159 * 4);
    std::memcpy(dhit + 159 * i, v[i].dhit, 159 * 4);
  }
}

// Cross-sector merger of one event's tracks (canonical order, hit IDs
// into hit_ids; row / y / z indexed by cluster ID).
void* orc_merge(const orc_geometry* g, const orc_params* P, const orc_merge_params* M,
                const orc_track* tracks, int64_t n_tracks, const int32_t* hit_ids,
                const uint8_t* row, const float* y, const float* z) {
  MergeIn in{tracks, n_tracks, hit_ids, row, y, z};
  MergeOut* o = new MergeOut();
  Merger m(g, P, M, in);
  m.run(*o);
  return o;
}

void orc_merge_free(void* h) { delete static_cast<MergeOut*>(h); }
int64_t orc_merge_n_tracks(void* h) { return int64_t(static_cast<MergeOut*>(h)->tracks.size()); }
int64_t orc_merge_n_hits(void* h) { return int64_t(static_cast<MergeOut*>(h)->hits.size()); }

// Merged tracks (canonical order) and hit IDs; per input track, the linked
// outer segment, the best outer candidate, its chi2 and the output track
// it went into.
void orc_merge_get(void* h, orc_track* out, int32_t* hit_ids, int32_t* n_segments,
                   int32_t* link_out, int32_t* best_out, double* best_chi2,
                   int32_t* merged_into) {
  MergeOut* o = static_cast<MergeOut*>(h);
  std::memcpy(out, o->tracks.data(), o->tracks.size() * sizeof(orc_track));
  std::memcpy(hit_ids, o->hits.data(), o->hits.size() * 4);
  std::memcpy(n_segments, o->n_segments.data(), o->n_segments.size() * 4);
  const size_t n = o->link_out.size();
  std::memcpy(link_out, o->link_out.data(), n * 4);
  std::memcpy(best_out, o->best_out.data(), n * 4);
  std::memcpy(best_chi2, o->best_chi2.data(), n * 8);
  std::memcpy(merged_into, o->merged_into.data(), n * 4);
}

// Drift-velocity calibration, per track: the track's parameters at its
// innermost hit transported (double, equal steps of at most step_max, stop
// beyond |sin phi| = s_max) to x = 0 of its sector frame, i.e. to the beam
// axis for a track from the origin.  y0, z0 out; ok = 0 if the transport
// stopped.  A drift velocity off by a relative eps moves every cluster to
// z (1 + eps) - side eps z_max, so primary tracks then point to
// z0 = -side eps z_max: the two sides' z0 differ by 2 eps z_max.
void orc_calib_z0(const orc_geometry* g, const orc_track* tracks, int64_t n, double step_max,
                  double s_max, double* y0, double* z0, int32_t* ok) {
  const double b = -0.00299792458 * double(g->bz_tesla);
  for (int64_t i = 0; i < n; ++i) {
    State<double> st;
    for (int k = 0; k < 5; ++k) st.p[k] = tracks[i].par[k];
    for (int k = 0; k < 15; ++k) st.C[k] = 0.0;
    const bool good = transport_to(st, tracks[i].x_ref, 0.0, b, s_max, step_max);
    ok[i] = good ? 1 : 0;
    y0[i] = st.p[0];
    z0[i] = st.p[1];
  }
}

// Frame rotation of one double state (pins): x in/out; returns 0 if refused.
int orc_rotate_d(double* p, double* C, double* x, double ca, double sa, double b, double smax) {
  State<double> st;
  std::memcpy(st.p, p, 40);
  std::memcpy(st.C, C, 120);
  if (!rotate(st, *x, ca, sa, b, smax)) return 0;
  std::memcpy(p, st.p, 40);
  std::memcpy(C, st.C, 120);
  return 1;
}

// Cholesky chi2 of a 5-vector (pins): returns 0 if S is not positive definite.
int orc_chi2_5(const double* S, const double* d, double* chi2) {
  return chi2_5(S, d, *chi2) ? 1 : 0;
}

// Single steps, for the pins of the Kalman primitives.  p[5], C[15] in/out.
int orc_predict_f(float* p, float* C, float dx, float b, float smax) {
  State<float> st;
  std::memcpy(st.p, p, 20);
  std::memcpy(st.C, C, 60);
  if (!predict(st, dx, b, smax)) return 0;
  std::memcpy(p, st.p, 20);
  std::memcpy(C, st.C, 60);
  return 1;
}

int orc_predict_d(double* p, double* C, double dx, double b, double smax) {
  State<double> st;
  std::memcpy(st.p, p, 40);
  std::memcpy(st.C, C, 120);
  if (!predict(st, dx, b, smax)) return 0;
  std::memcpy(p, st.p, 40);
  std::memcpy(C, st.C, 120);
  return 1;
}

// One double transport with the scattering noise (kk = k^2/X0, m2 = mass^2).
int orc_predict_ms_d(double* p, double* C, double dx, double b, double smax, double kk, double m2) {
  State<double> st;
  std::memcpy(st.p, p, 40);
  std::memcpy(st.C, C, 120);
  if (!predict(st, dx, b, smax, kk, m2)) return 0;
  std::memcpy(p, st.p, 40);
  std::memcpy(C, st.C, 120);
  return 1;
}

int orc_update_f(float* p, float* C, float my, float mz, float vy, float vz, float chi2max,
                 float smax, int gated, float* chi2) {
  State<float> st;
  std::memcpy(st.p, p, 20);
  std::memcpy(st.C, C, 60);
  const bool ok = update(st, my, mz, vy, vz, chi2max, smax, gated != 0, chi2);
  std::memcpy(p, st.p, 20);
  std::memcpy(C, st.C, 60);
  return ok ? 1 : 0;
}

// n independent float steps, each a transport by dx[i] then a gated update
// with meas[i] = (y, z, var_y, var_z): state[i] = (p[5], C[15]) in/out,
// result[i] = (bits: transport ok | update accepted << 1, chi2 of the update
// or 0).  The same primitives as orc_predict_f / orc_update_f, looped here.
void orc_kf_steps_f(float* state, const float* dx, const float* meas, int32_t* bits,
                    float* chi2, int64_t n, float b, float smax, float chi2max) {
  for (int64_t i = 0; i < n; ++i) {
    State<float> st;
    std::memcpy(st.p, state + 20 * i, 20);
    std::memcpy(st.C, state + 20 * i + 5, 60);
    int32_t r = 0;
    float ch = 0.0f;
    if (predict(st, dx[i], b, smax)) {
      r = 1;
      const float* m = meas + 4 * i;
      if (update(st, m[0], m[1], m[2], m[3], chi2max, smax, true, &ch)) r |= 2;
    }
    std::memcpy(state + 20 * i, st.p, 20);
    std::memcpy(state + 20 * i + 5, st.C, 60);
    bits[i] = r;
    chi2[i] = ch;
  }
}

int orc_update_d(double* p, double* C, double my, double mz, double vy, double vz,
                 double chi2max, double smax, int gated, double* chi2) {
  State<double> st;
  std::memcpy(st.p, p, 40);
  std::memcpy(st.C, C, 120);
  const bool ok = update(st, my, mz, vy, vz, chi2max, smax, gated != 0, chi2);
  std::memcpy(p, st.p, 40);
  std::memcpy(C, st.C, 120);
  return ok ? 1 : 0;
}

}  // extern "C"
