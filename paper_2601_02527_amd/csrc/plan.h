// Host-side event plan: everything about a batch of series that does not
// depend on the hyperparameters, built once per dataset.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gpssm {

constexpr int WAVE = 64;        // lanes per wavefront; chunks per segment and per work wave
constexpr int MAX_TERMS = 4;
constexpr int MAX_SLOTS = 4;

// step-length distribution kept per series for the launch-order cost model:
// the fraction of the series' steps with dt <= 2^(DT_KMIN + k), k < DT_NE
constexpr int DT_KMIN = -30;
constexpr int DT_NE = 48;

struct PlanOptions {
  int32_t chunk_min = 24;          // shortest chunk the planner makes (events)
  int32_t chunk_target = 0;        // target chunk length; 0 = derive from the batch size
  int64_t target_chunks = 131072;  // chunks wanted over the batch when deriving
  int32_t single_chunk = 0;        // 1: one chunk per series (no time splitting)
  int32_t threads = 0;             // host threads for planning; 0 = hardware concurrency
};

struct HostPlan {
  int64_t n_series = 0, n_meas = 0;
  int32_t max_slots = 0;  // largest overlap depth over the batch
  int64_t n_events = 0;   // real events
  int64_t n_ev_pad = 0;   // events in the interleaved layout (with padding)
  int32_t n_chunks = 0, n_seg = 0, n_wv = 0, max_chunk_len = 0;
  int32_t n_grp = 0, max_series_nseg = 0, max_series_ngrp = 0;

  // interleaved events: work wave w, step k, lane l at wv_ev0[w] + k*WAVE + l
  std::vector<double> dt, t, y, r, invd;
  std::vector<uint32_t> info;
  std::vector<int64_t> meas;  // global measurement index at end/instantaneous events, else -1

  // scan segments: runs of up to WAVE consecutive chunks of one series, whose
  // summaries the time-parallel scan composes across the lanes of a wavefront
  std::vector<int32_t> seg_chunk0, seg_nch;
  // groups of up to WAVE consecutive segments of one series: a second scan
  // level over the segment totals when a series has more than WAVE segments
  std::vector<int32_t> grp_seg0, grp_nseg, series_grp0, series_ngrp;
  // work waves of the per-chunk kernels: up to WAVE chunks of one series taken
  // in order of length, so that the lanes of a wavefront run similar lengths;
  // wv_chunk holds WAVE entries per wave (chunk of each lane, -1 if idle)
  std::vector<int32_t> wv_series, wv_nch, wv_len, wv_chunk;
  std::vector<int64_t> wv_ev0;
  std::vector<int32_t> chunk_len, chunk_series, chunk_wv, chunk_lane;
  std::vector<uint8_t> chunk_first;
  std::vector<double> chunk_t0, chunk_t1;  // time of the first / last event of each chunk
  std::vector<int32_t> series_chunk0, series_nch, series_slots, series_seg0, series_nseg, series_wv0, series_nwv;
  std::vector<int64_t> series_nev;
  std::vector<float> series_dt_cdf;  // n_series * DT_NE, see DT_KMIN
};

// Builds the plan from host copies of the inputs.  Returns 0 or a negative
// error code (see gp_ssm.h) with a message in err.
int build_plan(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end, const double* y,
               const double* yerr, const PlanOptions& opt, HostPlan& plan, std::string& err);

}  // namespace gpssm
