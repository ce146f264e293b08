// Drift-velocity calibration from tracks, the kind of online calibration the
// paper's reconstruction feeds (Section 3: calibration runs on top of the
// online reconstruction, accumulates data over many events, fits from time
// to time, and its result is fed back into the cluster transformation).
//
// z of a cluster comes from its drift time to the readout plane of its side
// (A: sectors 0-17 at +z_max, C: 18-35 at -z_max).  With the drift velocity
// off by a relative eps the measured z is z (1 + eps) - side eps z_max, so
// tracks from the primary vertex, carried to the beam axis, point to
// z0 = -side eps z_max; the two sides' medians give
// eps = (z0_C - z0_A) / (2 z_max).
//   accumulate  per track of a slot: parameters at the innermost hit
//               transported (double, steps <= 2 cm) to x = 0 of its sector
//               frame; tracks with >= 30 hits and |y0| <= 2 cm add 1 to the
//               bin of z0 in their side's histogram (integer atomics: the
//               counts do not depend on the order);
//   fit         per side the median of the histogram, linear inside the
//               median bin, then eps (one block);
//   correct     z <- (z + side eps z_max) / (1 + eps) for every cluster.
#include "tpc_device.h"
#include "tpc_kernels.h"

namespace tpc {

constexpr int kCalNmin = 30;
constexpr double kCalY0 = 2.0;
constexpr double kCalStep = 2.0;
constexpr double kCalSmax = 0.999;

__global__ void __launch_bounds__(256) k_cal_accumulate(Slot S, DevConst K, uint32_t* hist,
                                                       int n_bins, double z_lo, double w) {
  const uint32_t ntk = S.out_count[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < ntk; a += stride) {
    const tpc_track& t = S.out_tracks[a];
    if (t.n_hits < kCalNmin) continue;
    Helix<double> st;              // parameters only: z0 needs no covariance
    st.y = t.par[0];
    st.z = t.par[1];
    st.s = t.par[2];
    st.t = t.par[3];
    st.q = t.par[4];
    if (!transport_to_x<false>(st, t.x_ref, 0.0, K.bd, kCalSmax, kCalStep)) continue;
    if (!(fabs(st.y) <= kCalY0)) continue;
    const double f = (st.z - z_lo) / w;
    if (!(f >= 0.0 && f < (double)n_bins)) continue;
    const int b = (int)floor(f);
    atomicAdd(&hist[(t.sector / 18) * n_bins + b], 1u);
  }
}

// one block: out[0] = median z0 of side A, out[1] = of side C (NaN if
// empty), out[2] = eps measured on the histogram's events, out[3] = the
// estimate to use from now on.  The events were tracked after a correction
// with eps_t; a drift error E corrected with eps_t leaves exactly the error
// r = (E - eps_t) / (1 + eps_t), so E = eps_t + r (1 + eps_t).
__global__ void __launch_bounds__(256) k_cal_fit(const uint32_t* hist, int n_bins, double z_lo,
                                                 double w, double z_max, double eps_t, double* out) {
  __shared__ unsigned long long part[256];
  __shared__ double med[2];
  for (int side = 0; side < 2; ++side) {
    const uint32_t* c = hist + side * n_bins;
    // each thread sums a contiguous stretch; an exclusive scan of the
    // stretch sums locates the stretch holding the median
    const int per = (n_bins + blockDim.x - 1) / blockDim.x;
    const int b0 = min(n_bins, (int)threadIdx.x * per), b1 = min(n_bins, b0 + per);
    unsigned long long sum = 0;
    for (int b = b0; b < b1; ++b) sum += c[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long run = 0;
      for (unsigned i = 0; i < blockDim.x; ++i) {
        const unsigned long long v = part[i];
        part[i] = run;
        run += v;
      }
      med[side] = run == 0 ? __builtin_nan("") : -1.0;
      part[0] = run;   // the total, kept in slot 0 (its prefix is 0)
    }
    __syncthreads();
    const unsigned long long total = part[0];
    if (total > 0) {
      const double half = (double)total / 2.0;
      unsigned long long cum = threadIdx.x == 0 ? 0ull : part[threadIdx.x];
      for (int b = b0; b < b1; ++b) {
        const unsigned long long nxt = cum + c[b];
        if ((double)cum < half && (double)nxt >= half)
          med[side] = z_lo + ((double)b + (half - (double)cum) / (double)c[b]) * w;
        cum = nxt;
      }
      // the first bin reaching half (the case cum == half at a bin start
      // belongs to the earlier bin, which is handled above)
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = med[0];
    out[1] = med[1];
    const double r = (med[1] - med[0]) / (2.0 * z_max);
    out[2] = r;
    out[3] = eps_t + r * (1.0 + eps_t);
  }
}

__global__ void k_cal_correct(const uint8_t* sector, float* z, int64_t n, double eps, double z_max) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double side = sector[i] < 18 ? 1.0 : -1.0;
    z[i] = (float)(((double)z[i] + side * eps * z_max) / (1.0 + eps));
  }
}

}  // namespace tpc
