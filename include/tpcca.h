/*
 * tpcca.h -- C ABI of the MI355X TPC sector tracker.
 *
 * The tracker is the hot path the paper puts at the centre of its online
 * reconstruction (Abstract; Section 2: tracking is the most compute-intense
 * reconstruction step; the GPU tracker is built on a Cellular Automaton and
 * the Kalman filter).  Clusters (pad row, y, z, charge) of the 36 sectors x
 * 159 pad rows of the TPC go in; track hit lists with fitted helix
 * parameters and covariances come out.  Each sector is tracked on its own
 * (a detector link sees one part of every event, Section 2).
 *
 * Steps, all in HIP kernels on one GPU: stage and validate clusters; pad-row
 * hit grid; neighbours finder (best up/down link per hit); link cleaner and
 * start hits; tracklet construction (float Kalman filter out- and inward);
 * hit ownership and tracklet selection; output refit (double Kalman filter)
 * and canonical ordering.
 *
 * Conventions
 *  - Return codes: TPC_OK (0) or a negative TPC_E* code; tpc_last_error()
 *    gives a message.  Arguments are checked on the host before any device
 *    work is enqueued, so a failed call has enqueued nothing.
 *  - A context owns no device memory: the caller passes one device
 *    workspace (e.g. a torch uint8 tensor's data pointer) of at least
 *    tpc_workspace_bytes() and a HIP stream; all work of the context is
 *    enqueued on that stream, in call order.  A context is not thread-safe.
 *  - Cluster ID = index of the cluster in the event's input arrays; IDs must
 *    be < 2^24 per event.
 *  - Slots: a context has params->max_slots slots.  A slot holds one event
 *    (tpc_load_clusters) or a batch of events tracked together
 *    (tpc_load_batch: events are concatenated, sector g of the slot is sector
 *    g % 36 of event g / 36).
 */
#ifndef TPCCA_H
#define TPCCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPC_N_SECTORS 36
#define TPC_N_ROWS 159

enum {
  TPC_OK = 0,
  TPC_EINVAL = -1,     /* bad argument or bad cluster data */
  TPC_ENOMEM = -2,     /* workspace too small for the requested capacity */
  TPC_EOVERFLOW = -3,  /* caller output buffer too small (required sizes returned) */
  TPC_EDEVICE = -4,    /* a HIP call failed */
  TPC_ESTATE = -5,     /* call out of order for the slot */
  TPC_EBUSY = -6       /* (serving) slot still in flight */
};

/* where the cluster arrays passed to tpc_load_* live */
enum { TPC_HOST = 1, TPC_DEVICE = 2 };

/* Detector description (inputs; the tracker has no built-in geometry). */
typedef struct tpc_geometry {
  int32_t n_sectors;        /* must be 36 */
  int32_t n_rows;           /* must be 159 */
  float row_x[160];         /* pad-row radius x_r (cm), 159 used, increasing */
  float bz_tesla;           /* solenoid field */
  float tan_half_angle;     /* tan of half the sector opening (20 deg sectors) */
  float z_max;              /* drift length (cm) */
  float sigma_y0, sigma_y1; /* cluster error sigma_y(z) = y0 + y1 |z| / z_max */
  float sigma_z0, sigma_z1; /* same for z */
} tpc_geometry;

/* Tracker constants and capacities.  tpc_params_default() fills the values
 * this implementation was tuned with. */
typedef struct tpc_params {
  float nf_window;          /* neighbours-finder window half width (cm) */
  float nf_mmax;            /* max triplet deviation metric */
  float chi2_max;           /* Kalman gate */
  float k_win;              /* search window, units of sqrt(residual variance) */
  float w_max;              /* search window cap (cm) */
  float s_max;              /* max |sin phi| */
  float c_s0, c_t0, c_q0;   /* prior variances of sin phi, tan lambda, q/pT */
  float m_edge;             /* sector edge margin (cm) */
  float m_z;                /* membrane / drift-length margin (cm) */
  int32_t n_gap;            /* consecutive rows without hit that end a phase */
  int32_t n_min_tracklet;   /* hits of a valid tracklet */
  int32_t n_min_track;      /* owned hits of an output track */
  float bin_target;         /* grid: clusters per bin aimed at (tuning only) */
  float bin_min_edge;       /* grid: smallest bin edge (cm) (tuning only) */
  int32_t max_slots;        /* slots of a context */
  int32_t max_events;       /* events per slot */
  int64_t max_clusters;     /* clusters per slot */
  float x0_cm;              /* radiation length of the gas for the multiple-scattering
                               noise of every transport (0: no scattering) */
  float ms_mass;            /* particle mass of the scattering law (GeV) */
  int32_t n_min_chain;      /* hits of a cleaned chain that starts a tracklet (3..159) */
  /* launch shape (tuning only: the tracks never depend on these) */
  int32_t tl_block;         /* tracklet kernel threads per block: 64, 128 or 256 */
  int32_t win_batch;        /* window hits read per memory round trip: 2, 4 or 8 */
  int32_t row_batch;        /* hit-list rows read per round trip by the selection: 4, 8 or 16 */
} tpc_params;

/* One output track.  par / cov are given at x_ref, the pad-row radius of
 * the innermost hit: (y, z, sin phi, tan lambda, q/pT [c/GeV]); cov is the
 * lower triangle (yy, zy, zz, sy, sz, ss, Ty, Tz, Ts, TT, Qy, Qz, Qs, QT, QQ). */
typedef struct tpc_track {
  int32_t event;            /* event index inside the slot */
  int32_t sector;           /* 0..35 */
  int32_t n_hits;
  int32_t row_in;           /* innermost pad row */
  int32_t row_out;          /* outermost pad row */
  int32_t ndf;              /* 2 n_hits - 5 */
  int64_t hit_off;          /* first entry in the event's hit-ID list */
  int32_t inner_id;         /* cluster ID of the innermost hit (order key) */
  int32_t start_id;         /* cluster ID of the tracklet's start hit */
  double x_ref;
  double par[5];
  double cov[15];
  double chi2;
} tpc_track;

typedef struct tpc_ctx tpc_ctx;

/* Fill *p with the default constants; max_slots = 1, max_events = 1,
 * max_clusters = 4M.  The paper names the method only (Abstract: a cellular
 * automaton and the Kalman filter); the constants are this implementation's
 * definition of its cuts.  Returns TPC_EINVAL if p is NULL. */
int tpc_params_default(tpc_params* p);

/* Device bytes a context with these capacities needs (0 if p is invalid).
 * The track regions are sized for n_min_track: each sector of n clusters
 * has room for n / n_min_track + 1 tracks, the most its hits allow. */
size_t tpc_workspace_bytes(const tpc_params* p);

/* Create a context: the tracker of the TPC, the detector the paper tracks
 * with (Section 2: TPC track reconstruction subscribes to the data of all
 * TPC links; each sector is one link's part of the event).  g, p: copied.
 * dev_workspace: device memory of ws_bytes >= tpc_workspace_bytes(p), owned
 * by the caller and used by the context until tpc_destroy.  hip_stream: a hipStream_t (NULL = default
 * stream).  Errors: TPC_EINVAL (geometry not 36 x 159 increasing rows,
 * bad params), TPC_ENOMEM (workspace too small). */
int tpc_init_geometry(tpc_ctx** out, const tpc_geometry* g, const tpc_params* p,
                      void* dev_workspace, size_t ws_bytes, void* hip_stream);

/* Stage one event into a slot (the input of TPC track reconstruction, the
 * clusters of the TPC cluster finder, Section 2): n clusters as
 * structure-of-arrays, sector[i] < 36, row[i] < 159, finite y[i], z[i]
 * (local sector frame, cm),
 * q[i] charge (carried, unused; may be NULL).  flags: TPC_DEVICE (arrays in
 * device memory, used in place: the caller keeps them alive and unchanged
 * until the slot's tracks are read) or TPC_HOST (copied asynchronously into
 * the slot; the caller keeps the arrays alive until the next synchronising
 * call).  Bad cluster values are detected on the device and reported by
 * tpc_get_tracks as TPC_EINVAL.  Errors: TPC_EINVAL (slot, n, pointers,
 * flags), TPC_ENOMEM (n > max_clusters). */
int tpc_load_clusters(tpc_ctx* ctx, int slot, const uint8_t* sector, const uint8_t* row,
                      const float* y, const float* z, const float* q, int64_t n, int flags);

/* Stage a batch of n_events events into one slot (Section 2: many events
 * are in the chain at once).  event_offsets (host,
 * n_events + 1 entries, non-decreasing, event_offsets[0] = 0) delimit the
 * events inside the concatenated arrays.  Otherwise as tpc_load_clusters. */
int tpc_load_batch(tpc_ctx* ctx, int slot, int n_events, const int64_t* event_offsets,
                   const uint8_t* sector, const uint8_t* row, const float* y, const float* z,
                   const float* q, int flags);

/* Track one sector of a staged slot (sector < 36 * events in the slot;
 * Abstract and Section 2: cellular-automaton track finding and Kalman-filter
 * fitting, sector by sector): the grid is built on the slot's first
 * tracking call, and the slot's per-sector cluster counts are then read
 * back once (the call waits for the grid), so each later launch is sized by
 * its own sector; the neighbours finder, cleaner, tracklets, selection and
 * refit run for this sector only, each as its own launch.  Errors:
 * TPC_EINVAL, TPC_ESTATE (slot not loaded, or already finalised),
 * TPC_EDEVICE. */
int tpc_track_sector(tpc_ctx* ctx, int slot, int sector);

/* Track every sector of every event in the slot (Abstract and Section 2:
 * the GPU tracker, cellular automaton then Kalman filter): each step is one
 * launch over all sectors of the slot, then the tracks are put in canonical
 * order (event, innermost cluster ID).  Asynchronous; results are read with
 * tpc_get_tracks.  Errors: TPC_EINVAL, TPC_ESTATE. */
int tpc_track_event(tpc_ctx* ctx, int slot);

/* Track n staged slots (each a single event or a batch of events), each by
 * one replay of its HIP graph (Section 2: many events flow through the chain
 * at once; Section 4.2: several kernels in flight).  A slot without a graph
 * for its current staging (same input pointers and event offsets) is
 * captured first, once, as by tpc_graph_capture; later calls with the same
 * staging only replay.  slots: host array of n distinct slot indices.
 * Asynchronous; every slot is tracked as after tpc_track_event.  Requires a
 * non-default stream.  Arguments are checked for all slots before anything
 * is enqueued.  Errors: TPC_EINVAL (bad list, a slot twice, default
 * stream), TPC_ESTATE (a slot not staged, or during capture), TPC_EDEVICE. */
int tpc_track_events(tpc_ctx* ctx, const int* slots, int n);

/* Serving entry (Section 2: events are pipelined through the chain; Section
 * 5.1: the loop must not stall): enqueue the tracking of a staged slot and
 * return at once.  The slot's HIP graph is replayed if it was captured for
 * the current staging, otherwise the one-launch-per-step sequence of
 * tpc_track_event runs.  Completion is tested with tpc_poll (never waits);
 * results are then read with tpc_get_tracks or tpc_device_results.
 * Errors: TPC_EINVAL, TPC_ESTATE (slot not staged, already tracked without
 * a matching graph, or during capture), TPC_EDEVICE. */
int tpc_submit(tpc_ctx* ctx, int slot);

/* Concurrent kernels (Section 4.2: several kernels in parallel give +15%,
 * more than +30% expected).  Track every sector of the slot with the
 * per-sector launch sequence of
 * tpc_track_sector, sector g on the library's own stream g mod n_streams
 * (1 <= n_streams <= 8; streams at default priority, created on first use),
 * after the grid is built on the context stream; the context stream waits
 * for all of them before the canonical ordering.  The paper's concurrent
 * kernels of independent sectors (Section 4.2), kept as an alternative to
 * the one-launch-per-step path: the tracks are identical to
 * tpc_track_event's.  Each stream has its own counters and scan space, so
 * sectors in flight together share no scratch.  Asynchronous.  Errors:
 * TPC_EINVAL, TPC_ESTATE (slot not staged or already tracked, or called
 * during graph capture), TPC_EDEVICE. */
int tpc_track_event_streams(tpc_ctx* ctx, int slot, int n_streams);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): track one
 * event as tpc_load_clusters(TPC_DEVICE) + tpc_track_event + tpc_get_tracks
 * would, with no context and no caller workspace.  The workspace is a fixed
 * 64 MiB array of device memory inside the library, one per GPU, held from
 * the first call on that GPU until the process ends; the event must fit in
 * it (about 185,000 clusters with the default params; TPC_ENOMEM beyond,
 * before anything is enqueued).  No device memory is allocated or freed and
 * no memset or copy node is enqueued: kernels only, on hip_stream
 * (asynchronous).  g, p: host; p's max_slots / max_events / max_clusters are
 * ignored (one event of n clusters).  sector, row, y, z: device arrays of n
 * clusters (as tpc_load_clusters).  Outputs, device memory owned by the
 * caller: tracks[max_tracks], hit_ids[max_hits] (the event's tracks in
 * canonical order and their hit IDs; at most max_tracks / max_hits written)
 * and status[4] = {tracks, hits, flags, 0} with flags bit 0 = invalid
 * clusters, bit 1 = a pad row over 4096 clusters, bit 2 = internal capacity
 * exceeded, bit 3 = tracks or hits beyond max_tracks / max_hits.  Calls on
 * one GPU share its array: calls on one stream are ordered, calls that
 * overlap on one GPU (other streams, or other threads) race and must not be
 * made.  Errors (tpc_last_error(NULL)): TPC_EINVAL, TPC_ENOMEM, TPC_EDEVICE. */
int tpc_track_event_noalloc(const tpc_geometry* g, const tpc_params* p, const uint8_t* sector,
                            const uint8_t* row, const float* y, const float* z, int64_t n,
                            tpc_track* tracks, int64_t max_tracks, int32_t* hit_ids,
                            int64_t max_hits, uint32_t* status, void* hip_stream);

/* Output of the tracker (Abstract: tracks of the TPC, fitted by the Kalman
 * filter).  Wait for the slot and copy the tracks of one event of it (event = 0 for
 * tpc_load_clusters) into caller host memory: out[max_tracks],
 * hit_ids[max_hits] (cluster IDs, each track's hits ascending by row).
 * *n_tracks, *n_hits receive the event's counts.  If sectors were tracked
 * one by one, finalises the slot first.  Errors: TPC_EOVERFLOW (buffers too
 * small; counts still returned, nothing copied), TPC_EINVAL (bad cluster
 * data or a pad row with more than 4096 clusters), TPC_ESTATE, TPC_EDEVICE. */
int tpc_get_tracks(tpc_ctx* ctx, int slot, int event, tpc_track* out, int64_t max_tracks,
                   int32_t* hit_ids, int64_t max_hits, int64_t* n_tracks, int64_t* n_hits);

/* The same output for every event of a slot in one copy (Section 2: the
 * event stream's results leave the tracker together; the serving loop reads
 * a continuous-batching slot this way, with a few synchronisations per slot
 * instead of per event).  out[max_tracks], hit_ids[max_hits]: the slot's
 * tracks and hit IDs, event after event, each event's block exactly what
 * tpc_get_tracks returns for it (hit_off relative to the event);
 * event_track_off, event_hit_off: host arrays of n_events + 1 entries (2 for
 * a slot staged with tpc_load_clusters) receiving the start of each event's
 * block and the totals, also when the buffers are too small.  *n_tracks,
 * *n_hits receive the totals.  Errors: as tpc_get_tracks, and TPC_EINVAL
 * for a NULL offset array. */
int tpc_get_slot_tracks(tpc_ctx* ctx, int slot, tpc_track* out, int64_t max_tracks,
                        int32_t* hit_ids, int64_t max_hits, uint32_t* event_track_off,
                        uint32_t* event_hit_off, int64_t* n_tracks, int64_t* n_hits);

/* Output of the tracker, as in tpc_get_tracks.  Device-resident results of
 * a tracked slot, without copies or
 * synchronisation: tracks of all events of the slot in canonical order,
 * hit IDs, per-event offsets (device arrays of n_events + 1 entries, into
 * the track array and the hit array) and the slot's [track, hit] totals
 * (device array of 2).  Pointers stay valid until the slot is loaded again. */
int tpc_device_results(tpc_ctx* ctx, int slot, const tpc_track** tracks, const int32_t** hit_ids,
                       const uint32_t** event_track_off, const uint32_t** event_hit_off,
                       const uint32_t** totals);

/* Cellular-automaton diagnostics (Abstract: track finding by a cellular
 * automaton).  The finding steps' links for one event of a tracked slot, copied
 * to host arrays of the event's cluster count: the neighbours finder's
 * up/down links and the cleaned links, as cluster IDs (-1 = none).  Any
 * pointer may be NULL.  Synchronises.  Errors: TPC_EINVAL, TPC_ESTATE. */
int tpc_get_links(tpc_ctx* ctx, int slot, int event, int32_t* up, int32_t* dn, int32_t* up_clean,
                  int32_t* dn_clean);

/* Kalman-filter primitives (Abstract: Kalman-filter track fitting).  Apply
 * one float transport + gated update to each of n states on the device (the
 * tracklet filter's primitives, for bit-level tests).  All
 * arrays are device memory: state[n][20] = (y, z, s, T, Q, C[15]) in/out,
 * dx[n], meas[n][4] = (y, z, var_y, var_z), result[n][2] = (int bits:
 * transport ok | update accepted << 1, chi2 as float).  Uses the context's
 * b, s_max, chi2_max.  Asynchronous on the context stream. */
int tpc_kf_step_f32(tpc_ctx* ctx, float* state, const float* dx, const float* meas,
                    float* result, int64_t n);

/* Constants of the cross-sector merger. */
typedef struct tpc_merge_params {
  float chi2_max;           /* cut on the 5-parameter match chi2 of two segments */
  int32_t row_gap;          /* largest pad-row distance between the segments */
  float step_max;           /* longest transport step between sector frames (cm, >= 0.1) */
  int32_t passes;           /* inward refit passes of a merged track (1..8) */
  float s_max;              /* largest |sin phi| of the merger's transports (< 1) */
} tpc_merge_params;

/* Defaults: chi2_max 30, row_gap 12, step_max 2 cm, passes 3, s_max 0.999. */
int tpc_merge_params_default(tpc_merge_params* m);

/* Join track segments across sector boundaries, for every event of a
 * tracked slot (Section 2: data of all links of an event are merged for the
 * global reconstruction; the step after the per-sector tracking: a particle crossing
 * from one sector into its neighbour on the same side, or across the central
 * membrane into the other side's sector of the same azimuth, leaves one
 * segment in each).  Per track, the state at its outermost hit (an outward
 * Kalman pass seeded with its fitted parameters); each pair (A, B), B in a
 * neighbouring sector or across the membrane with
 * 0 < B.row_in - A.row_out <= row_gap, is compared after turning A's outer
 * state into B's frame (neighbouring sectors are 2 atan(tan_half_angle)
 * apart; across the membrane the frame is the same) and transporting it to
 * B's innermost row: chi2 of the 5-parameter
 * difference with covariance C_A + C_B, kept if <= chi2_max; A and B are
 * linked when each is the other's smallest-chi2 partner (ties to the
 * smaller track index); each chain of linked segments is refitted inward
 * over all its hits in `passes` passes, turning frames at the boundaries,
 * and replaces its segments (a chain whose refit fails stays as segments).
 * The merged track keeps its innermost segment's sector, frame, inner hit
 * and canonical position.  Asynchronous on the context stream; read with
 * tpc_get_merged.  Errors: TPC_EINVAL (bad parameters), TPC_ESTATE (slot
 * not tracked, or during graph capture), TPC_EDEVICE. */
int tpc_merge(tpc_ctx* ctx, int slot, const tpc_merge_params* m);

/* Like tpc_get_tracks, for the merger's output of one event; n_segments
 * (may be NULL) receives the number of segments of each track.
 * Synchronises.  Errors: TPC_EINVAL, TPC_ESTATE (not merged since the last
 * staging), TPC_EOVERFLOW (buffers too small; counts filled in). */
int tpc_get_merged(tpc_ctx* ctx, int slot, int event, tpc_track* out, int64_t max_tracks,
                   int32_t* hit_ids, int64_t max_hits, int32_t* n_segments, int64_t* n_tracks,
                   int64_t* n_hits);

/* Merger diagnostics of one event, per track of tpc_get_tracks' list (host
 * arrays of that length, each may be NULL): the linked outer segment, the
 * best outer candidate (-1 none), its chi2, and the index of the
 * tpc_get_merged track the track went into.  Synchronises.  Errors:
 * TPC_EINVAL, TPC_ESTATE. */
int tpc_get_merge_links(tpc_ctx* ctx, int slot, int event, int32_t* link_out, int32_t* best_out,
                        double* best_chi2, int32_t* merged_into);

/* Drift-velocity calibration from tracks (paper, Section 3: online
 * calibration runs on the online reconstruction, accumulates data over many
 * events and fits from time to time; Section 5.3: its result is fed back
 * into the cluster transformation).  z of a cluster comes from its drift
 * time to its side's readout plane (sectors 0-17 at +z_max, 18-35 at
 * -z_max); a drift velocity off by the relative eps gives the measured
 * z' = z (1 + eps) - side eps z_max, so primary tracks carried to the beam
 * axis point to z0 = -side eps z_max.
 *
 * tpc_calib_accumulate: for every track of a tracked slot with >= 30 hits,
 * its parameters at the innermost hit are transported (double, steps of at
 * most 2 cm, |sin phi| <= 0.999) to x = 0 of its sector frame; if |y0| <= 2
 * cm, 1 is added to bin floor((z0 - z_lo) / w) (w = (z_hi - z_lo) / n_bins,
 * in range only) of hist[side][n_bins] (device memory, uint32, side 0 = A;
 * the caller zeroes it; integer atomics, so counts do not depend on order).
 * Asynchronous on the context stream (covered by tpc_poll); the context
 * stream does not wait for other streams, so writes of hist queued
 * elsewhere must be ordered before the call by the caller.  Errors:
 * TPC_EINVAL, TPC_ESTATE (slot not tracked).
 *
 * tpc_calib_fit (Section 3, item 4: a fit every n-th event, and Section
 * 5.1: run asynchronously): on the given stream (device hist and out), each
 * side's median of z0 (linear inside the median bin; NaN if the side is
 * empty), the drift error measured on the histogram's events
 * eps_r = (median_C - median_A) / (2 z_max), and the estimate to adopt:
 * the events were tracked after a correction with eps_tracked, which
 * leaves exactly the error eps_r = (E - eps_tracked) / (1 + eps_tracked)
 * of a true error E, so E = eps_tracked + eps_r (1 + eps_tracked):
 * out[4] = {median_A, median_C, eps_r, E} (NaN where a side is empty).
 * |eps_tracked| < 0.5.  One small kernel; meant to run beside the tracking
 * on a stream of its own.  Errors: TPC_EINVAL, TPC_EDEVICE.
 *
 * tpc_calib_correct_z (Section 5.3: the result is fed back into the cluster
 * transformation): z[i] <- (z[i] + side eps z_max) / (1 + eps) for n
 * device clusters (side from sector[i]), in place; |eps| < 0.5.
 * Asynchronous on the context stream (same ordering rule as above).
 * Errors: TPC_EINVAL. */
int tpc_calib_accumulate(tpc_ctx* ctx, int slot, uint32_t* hist, int n_bins, float z_lo,
                         float z_hi);
int tpc_calib_fit(const uint32_t* hist, int n_bins, float z_lo, float z_hi, float z_max,
                  double eps_tracked, double* out, void* hip_stream);
int tpc_calib_correct_z(tpc_ctx* ctx, const uint8_t* sector, float* z, int64_t n, double eps);

/* Batched launch (Section 2: events pipelined through the chain).  Record
 * into a HIP graph, without running it, the whole sequence
 * tpc_track_event would enqueue for the slot as currently staged (grid,
 * finding, fitting, ordering; kernels only, no memset or copy nodes).  The
 * graph is kept by the context, one per slot, and bakes in the slot's
 * staged shape: input pointers, cluster count and event offsets.
 * Requires a non-default stream.  Errors: TPC_EINVAL, TPC_ESTATE (slot not
 * staged), TPC_EDEVICE (capture failed). */
int tpc_graph_capture(tpc_ctx* ctx, int slot);

/* Batched launch, as tpc_graph_capture.  Launch the slot's graph on the
 * context stream (asynchronous); the slot is
 * then tracked as after tpc_track_event.  The slot must be staged with the
 * same shape as at capture (e.g. TPC_HOST copies of new clusters into the
 * slot's own buffers, or the same device arrays refilled in place).
 * Errors: TPC_EINVAL, TPC_ESTATE (no graph, or the staged shape changed). */
int tpc_graph_launch(tpc_ctx* ctx, int slot);

/* Serving completion test (Section 5.1: check at every event whether the
 * task has finished, never block).  TPC_OK if all work enqueued so far for
 * the slot (staging, tracking) has finished, TPC_EBUSY if not; never waits.
 * Errors: TPC_EINVAL. */
int tpc_poll(tpc_ctx* ctx, int slot);

/* Measurement (the paper reports tracking time per event, Section 4.2,
 * Table 1).  With profiling on, tpc_track_event records HIP events on the
 * context stream around its steps (no synchronisation; a ring of the last
 * 256 steps); tpc_set_profiling(ctx, 1) starts a new measurement.
 * tpc_get_profile waits for the stream and returns the milliseconds of each
 * step averaged over the steps tracked since profiling was switched on (the
 * last 256 if more) (ms[TPC_N_STAGES]: grid, neighbours, clean+starts,
 * tracklets, weights+selection, refit, output) and, for the last tracked
 * slot, its work counters
 * (counters[TPC_N_COUNTERS]: 0 tracklets, 1 tracklet row visits, 2 hits
 * inside the tracklet search windows, 3 tracks refitted, 4 clusters,
 * 5 sorted hits, 6 tracklet hits (final hit lists, all tracklets),
 * 7 gated Kalman updates tried by the tracklets, 8 output tracks,
 * 9 hits of the output tracks).  Either pointer may be NULL.  Errors:
 * TPC_EINVAL, TPC_ESTATE (nothing profiled yet), TPC_EDEVICE. */
#define TPC_N_STAGES 7
#define TPC_N_COUNTERS 10
int tpc_set_profiling(tpc_ctx* ctx, int enable);
int tpc_get_profile(tpc_ctx* ctx, double* ms, uint64_t* counters);

/* Message of the last failed call of ctx (or of the last failed
 * tpc_init_geometry when ctx is NULL). */
const char* tpc_last_error(const tpc_ctx* ctx);

/* Release the context (host memory only; the workspace stays the caller's).
 * Waits for the context's stream. */
int tpc_destroy(tpc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TPCCA_H */
