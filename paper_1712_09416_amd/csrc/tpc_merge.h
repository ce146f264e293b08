// Buffers and constants of the cross-sector merger (merge.hip), kept apart
// from the tracking structures of tpc_device.h.
#pragma once

#include "tpc_device.h"

namespace tpc {

// Buffers of the cross-sector merger, per slot (K = track capacity, S =
// sectors, E = events).  Track positions are the slot's canonical output
// positions.
// The compatible pairs are listed in segments, each with its own counter
// (a block lists into segment blockIdx % kPairSegs), so the counters'
// atomics are spread over many addresses instead of meeting at one.
constexpr int kPairSegs = 64;
constexpr int kPairPad = 16;        // counters 16 x 4 bytes apart

struct MergeSlot {
  uint32_t* in_off;         // [S*159+1] tracks per (event, sector, first row), then offsets
  uint32_t* in_cur;         // [S*159] scatter cursors
  int32_t* in_list;         // [K] track positions grouped by (event, sector, first row)
  uint32_t* out_off;        // [S*159+1] the same by last row
  uint32_t* out_cur;        // [S*159]
  int32_t* out_list;        // [K]
  double* op;               // [K][5] state at the outermost hit
  double* oc;               // [K][15]
  int32_t* ok;              // [K] outer state exists
  int32_t* best_out;        // [K] best outer partner, -1 none
  double* chi_out;          // [K]
  int32_t* best_in;         // [K] best inner partner, -1 none
  double* chi_in;           // [K]
  unsigned long long* in_key;   // [K] per B: bits of the smallest chi2 of a compatible A (~0: none)
  unsigned long long* out_key;  // [K] per A: the same over its compatible B's
  int32_t* pair_a;          // [P] compatible pairs listed by the first pair pass, in
  int32_t* pair_b;          //     kPairSegs segments of pair_cap entries
  unsigned long long* pair_key;  // [P] their chi2 bit patterns
  uint32_t* pair_n;         // [kPairSegs * kPairPad] pairs found per segment, one
                            //     counter per 64 bytes (may exceed pair_cap: then
                            //     not all listed)
  uint32_t pair_cap;        // entries per segment
  int32_t* link_out;        // [K] mutual best outer partner, -1 none
  int32_t* link_in;         // [K]
  int32_t* head_ok;         // [K] per chain head: chain of >= 2 segments refitted
  int32_t* nseg;            // [K] per chain head: segments
  int32_t* nfit;            // [K] per chain head: hits of the refitted chain
  double* par;              // [K][5] per chain head
  double* cov;              // [K][15]
  double* chi2;             // [K]
  uint32_t* emit;           // [K+1] 1 per output track, then its output position
  uint32_t* nh;             // [K+1] its hit count, then its first hit
  int32_t* into;            // [K] output track of each input track
  tpc_track* tracks;        // [K] merged output, canonical order
  int32_t* hits;            // [n]
  int32_t* out_nseg;        // [K]
  uint32_t* ev_track_off;   // [E+1]
  uint32_t* ev_hit_off;     // [E+1]
};

// Constants of one merge call.
struct MergeConst {
  double chi2_max;          // match cut
  double step_max;          // longest transport step between frames (cm)
  double smax;              // largest |sin phi| of the merger's transports
  double ca, sa;            // cosine and sine of the angle between neighbouring sectors
  int32_t row_gap;          // largest pad-row distance between segments
  int32_t passes;           // refit passes of a merged chain
};

}  // namespace tpc
