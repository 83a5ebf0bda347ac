// Host-side event plan (see plan.h).
//
// Per series:
//  * validation (finite inputs, t_end >= t_start, start times non-decreasing,
//    yerr >= 0);
//  * instrument slots: exposures in start order take the lowest slot whose
//    previous exposure ended at or before their start, so no slot
//    self-overlaps and the number of slots equals the overlap depth (any
//    valid labelling gives the same result, Sec. 3.2.3);
//  * events: each exposure with t_end > t_start gives a start and an end event
//    (Sec. 3.2, K = 2N states), a zero-length exposure one instantaneous
//    event; events are ordered by time, ends before instantaneous before
//    starts at equal times;
//  * chunks: the event sequence is cut after events where no exposure is open
//    ("quiet" points), so that a chunk's boundary state is the SHO state
//    alone; the cuts are the quiet points nearest to an even grid of the
//    target length, which keeps the chunks of a segment of similar length.
// Over the batch, runs of up to 64 consecutive chunks of one series form a
// scan segment (the lanes of one wavefront in the scan kernels).  The
// per-chunk kernels instead take a series' chunks longest first, 64 to a work
// wave (one chunk per lane), and events are stored interleaved by work wave so
// a wavefront reads 64 consecutive values per step.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

namespace gpssm {

namespace {

enum : uint32_t { K_END = 0u, K_INSTANT = 1u, K_START = 2u, K_PAD = 3u };

struct Ev {
  double t;
  uint32_t kind;
  int32_t slot;
  int64_t n;  // global measurement index
};

struct SeriesWork {
  int rc = 0;
  std::string err;
  int32_t slots = 0;
  std::vector<Ev> ev;
  std::vector<uint32_t> open_before;
  std::vector<int64_t> cuts;  // chunk end positions (exclusive)
  float dt_cdf[DT_NE] = {};   // see HostPlan::series_dt_cdf
};

int plan_series(int64_t b, int64_t lo, int64_t hi, const double* ts, const double* te, const double* yerr, int64_t Lb,
                int32_t chunk_min, bool single, SeriesWork& w) {
  const int64_t n = hi - lo;
  for (int64_t i = lo; i < hi; ++i) {
    if (!std::isfinite(ts[i]) || !std::isfinite(te[i]) || !std::isfinite(yerr[i])) {
      w.err = "non-finite input in series " + std::to_string(b);
      return -2;
    }
    if (te[i] < ts[i]) {
      w.err = "t_end < t_start at measurement " + std::to_string(i);
      return -2;
    }
    if (yerr[i] < 0) {
      w.err = "negative yerr at measurement " + std::to_string(i);
      return -2;
    }
    if (i > lo && ts[i] < ts[i - 1]) {
      w.err = "t_start not sorted in series " + std::to_string(b);
      return -2;
    }
  }
  // slots
  double last_end[MAX_SLOTS];
  int32_t used = 0;
  std::vector<int32_t> slot(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    const double s = ts[lo + i], e = te[lo + i];
    if (!(e > s)) continue;
    int32_t k = -1;
    for (int32_t j = 0; j < used; ++j)
      if (last_end[j] <= s) {
        k = j;
        break;
      }
    if (k < 0) {
      if (used == MAX_SLOTS) {
        w.err = "more than " + std::to_string(MAX_SLOTS) + " overlapping exposures in series " + std::to_string(b);
        return -4;
      }
      k = used++;
    }
    last_end[k] = e;
    slot[i] = k;
  }
  w.slots = used;
  // events
  w.ev.clear();
  w.ev.reserve(2 * n);
  for (int64_t i = 0; i < n; ++i) {
    if (slot[i] >= 0) {
      w.ev.push_back({ts[lo + i], K_START, slot[i], lo + i});
      w.ev.push_back({te[lo + i], K_END, slot[i], lo + i});
    } else {
      w.ev.push_back({ts[lo + i], K_INSTANT, -1, lo + i});
    }
  }
  std::sort(w.ev.begin(), w.ev.end(), [](const Ev& a, const Ev& c) {
    if (a.t != c.t) return a.t < c.t;
    if (a.kind != c.kind) return a.kind < c.kind;
    return a.n < c.n;
  });
  // open sets and the quiet points (cut positions after which no exposure
  // is open)
  const int64_t ne = (int64_t)w.ev.size();
  w.open_before.resize(ne);
  w.cuts.clear();
  std::vector<int64_t> quiet;
  uint32_t open = 0;
  for (int64_t k = 0; k < ne; ++k) {
    w.open_before[k] = open;
    const Ev& e = w.ev[k];
    if (e.kind == K_START) open |= (1u << e.slot);
    if (e.kind == K_END) open &= ~(1u << e.slot);
    if (open == 0 && k + 1 < ne) quiet.push_back(k + 1);
  }
  // chunks: ne / L of them (L the target length, at least chunk_min), each cut
  // at the quiet point nearest to its place on an even grid, so that chunk
  // lengths stay close to the mean even where quiet points are sparse (the
  // lanes of a wavefront all run as long as its longest chunk)
  const int64_t L = std::max<int64_t>(Lb, chunk_min);
  const int64_t nc = single ? 1 : std::max<int64_t>(1, ne / L);
  // the smallest longest chunk with which nc chunks cover the series: cutting
  // at the farthest admissible quiet point needs the fewest chunks for a
  // given longest chunk; no chunk below is made longer than that
  auto chunks_needed = [&](int64_t lmax) {
    int64_t at = 0, n = 1;
    while (ne - at > lmax) {
      auto it = std::upper_bound(quiet.begin(), quiet.end(), at + lmax);
      if (it == quiet.begin() || *(it - 1) - at < std::min<int64_t>(chunk_min, lmax)) return ne + 1;
      at = *(it - 1);
      ++n;
    }
    return n;
  };
  int64_t lmax = ne;
  if (nc > 1) {
    int64_t lo = (ne + nc - 1) / nc, hi = ne;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (chunks_needed(mid) <= nc)
        hi = mid;
      else
        lo = mid + 1;
    }
    lmax = lo;
  }
  int64_t prev = 0;
  for (int64_t i = 1; i < nc && ne - prev > lmax; ++i) {
    const double target = (double)ne * (double)i / (double)nc;
    // first quiet point at or after the target, and the one before it
    auto it = std::lower_bound(quiet.begin(), quiet.end(), (int64_t)std::ceil(target));
    int64_t best = -1;
    double dbest = 0.0;
    for (int cand = 0; cand < 2; ++cand) {
      auto jt = (cand == 0) ? it : it - 1;
      if (cand == 1 && it == quiet.begin()) continue;
      if (jt == quiet.end()) continue;
      const int64_t q = *jt;
      if (q - prev < chunk_min || ne - q < chunk_min) continue;
      const double d = std::fabs((double)q - target);
      if (best < 0 || d < dbest) {
        best = q;
        dbest = d;
      }
    }
    if (best < 0) {
      // nearest admissible quiet point after the previous cut
      auto kt = std::lower_bound(quiet.begin(), quiet.end(), prev + chunk_min);
      if (kt == quiet.end() || ne - *kt < chunk_min) break;
      best = *kt;
    }
    if (best - prev > lmax) {
      // too long: the farthest quiet point within the bound instead
      auto kt = std::upper_bound(quiet.begin(), quiet.end(), prev + lmax);
      if (kt != quiet.begin() && *(kt - 1) > prev) best = *(kt - 1);
    }
    if (best <= prev) continue;
    w.cuts.push_back(best);
    prev = best;
  }
  // whatever the grid left longer than the bound
  while (ne - prev > lmax) {
    auto kt = std::upper_bound(quiet.begin(), quiet.end(), prev + lmax);
    if (kt == quiet.begin() || *(kt - 1) <= prev) break;
    prev = *(kt - 1);
    w.cuts.push_back(prev);
  }
  // a series without measurements has no chunk (its log-likelihood is 0)
  if (ne > 0) w.cuts.push_back(ne);
  // step-length histogram in powers of two, then its cumulative fractions
  int64_t cnt[DT_NE] = {};
  for (int64_t k = 1; k < ne; ++k) {
    const double d = w.ev[k].t - w.ev[k - 1].t;
    int bin = 0;
    if (d > 0.0) {
      int ex;
      std::frexp(d, &ex);  // d in [2^(ex-1), 2^ex)
      bin = std::min(DT_NE - 1, std::max(0, ex - DT_KMIN));
    }
    ++cnt[bin];
  }
  int64_t acc = 0;
  for (int k = 0; k < DT_NE; ++k) {
    acc += cnt[k];
    w.dt_cdf[k] = ne > 1 ? (float)((double)acc / (double)(ne - 1)) : 1.0f;
  }
  return 0;
}

}  // namespace

int build_plan(int64_t n_series, const int64_t* offsets, const double* t_start, const double* t_end, const double* y,
               const double* yerr, const PlanOptions& opt, HostPlan& P, std::string& err) {
  if (n_series < 1) {
    err = "n_series < 1";
    return -1;
  }
  if (offsets[0] != 0) {
    err = "offsets[0] != 0";
    return -1;
  }
  for (int64_t b = 0; b < n_series; ++b)
    if (offsets[b + 1] < offsets[b]) {
      err = "offsets not ascending at series " + std::to_string(b);
      return -1;
    }
  const int64_t N = offsets[n_series];
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(y[i])) {
      err = "non-finite y at measurement " + std::to_string(i);
      return -2;
    }
  // total event estimate for the target chunk length
  int64_t total_ev = 0;
  for (int64_t i = 0; i < N; ++i) total_ev += (t_end[i] > t_start[i]) ? 2 : 1;
  int64_t Lglob = opt.chunk_target > 0 ? opt.chunk_target
                                       : std::max<int64_t>(opt.chunk_min, (total_ev + opt.target_chunks - 1) /
                                                                            std::max<int64_t>(1, opt.target_chunks));

  std::vector<SeriesWork> work(n_series);
  unsigned nth = opt.threads > 0 ? (unsigned)opt.threads : std::max(1u, std::thread::hardware_concurrency());
  nth = (unsigned)std::min<int64_t>(nth, n_series);
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      const int64_t b = next.fetch_add(1);
      if (b >= n_series) break;
      const int64_t lo = offsets[b], hi = offsets[b + 1];
      int64_t eb = 0;
      for (int64_t i = lo; i < hi; ++i) eb += (t_end[i] > t_start[i]) ? 2 : 1;
      const int64_t Lb = std::min<int64_t>(Lglob, std::max<int64_t>(opt.chunk_min, (eb + WAVE - 1) / WAVE));
      work[b].rc = plan_series(b, lo, hi, t_start, t_end, yerr, Lb, opt.chunk_min, opt.single_chunk != 0, work[b]);
    }
  };
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nth; ++i) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  for (int64_t b = 0; b < n_series; ++b)
    if (work[b].rc) {
      err = work[b].err;
      return work[b].rc;
    }

  // chunk and segment tables
  P = HostPlan();
  P.n_series = n_series;
  P.n_meas = N;
  P.series_chunk0.resize(n_series);
  P.series_nch.resize(n_series);
  P.series_slots.resize(n_series);
  P.series_seg0.resize(n_series);
  P.series_nseg.resize(n_series);
  P.series_wv0.resize(n_series);
  P.series_nwv.resize(n_series);
  P.series_grp0.resize(n_series);
  P.series_ngrp.resize(n_series);
  P.series_nev.resize(n_series);
  std::vector<int64_t> chunk_evstart;  // (series-local start of each chunk)
  for (int64_t b = 0; b < n_series; ++b) {
    SeriesWork& w = work[b];
    P.max_slots = std::max(P.max_slots, w.slots);
    P.series_slots[b] = w.slots;
    P.series_nev[b] = (int64_t)w.ev.size();
    P.series_dt_cdf.insert(P.series_dt_cdf.end(), w.dt_cdf, w.dt_cdf + DT_NE);
    P.n_events += (int64_t)w.ev.size();
    P.series_chunk0[b] = P.n_chunks;
    int64_t prev = 0;
    const int32_t c_first = P.n_chunks;
    for (size_t q = 0; q < w.cuts.size(); ++q) {
      const int64_t len = w.cuts[q] - prev;
      P.chunk_len.push_back((int32_t)len);
      P.chunk_series.push_back((int32_t)b);
      P.chunk_first.push_back(q == 0 ? 1 : 0);
      P.chunk_t0.push_back(w.ev[prev].t);
      P.chunk_t1.push_back(w.ev[w.cuts[q] - 1].t);
      chunk_evstart.push_back(prev);
      P.max_chunk_len = std::max<int32_t>(P.max_chunk_len, (int32_t)len);
      prev = w.cuts[q];
      ++P.n_chunks;
    }
    P.series_nch[b] = P.n_chunks - c_first;
    P.series_seg0[b] = P.n_seg;
    // scan segments of up to WAVE consecutive chunks
    for (int32_t c = c_first; c < P.n_chunks; c += WAVE) {
      P.seg_chunk0.push_back(c);
      P.seg_nch.push_back(std::min<int32_t>(WAVE, P.n_chunks - c));
      ++P.n_seg;
    }
    P.series_nseg[b] = P.n_seg - P.series_seg0[b];
    P.max_series_nseg = std::max(P.max_series_nseg, P.series_nseg[b]);
    // groups of segments for the second scan level
    P.series_grp0[b] = P.n_grp;
    for (int32_t q = 0; q < P.series_nseg[b]; q += WAVE) {
      P.grp_seg0.push_back(P.series_seg0[b] + q);
      P.grp_nseg.push_back(std::min<int32_t>(WAVE, P.series_nseg[b] - q));
      ++P.n_grp;
    }
    P.series_ngrp[b] = P.n_grp - P.series_grp0[b];
    P.max_series_ngrp = std::max(P.max_series_ngrp, P.series_ngrp[b]);
    // work waves: the series' chunks longest first, WAVE to a wave
    std::vector<int32_t> order(P.n_chunks - c_first);
    for (size_t q = 0; q < order.size(); ++q) order[q] = c_first + (int32_t)q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t z) { return P.chunk_len[x] > P.chunk_len[z]; });
    P.series_wv0[b] = P.n_wv;
    P.chunk_wv.resize(P.n_chunks);
    P.chunk_lane.resize(P.n_chunks);
    for (size_t q0 = 0; q0 < order.size(); q0 += WAVE) {
      const int32_t nch = (int32_t)std::min<size_t>(WAVE, order.size() - q0);
      P.wv_series.push_back((int32_t)b);
      P.wv_nch.push_back(nch);
      P.wv_len.push_back(P.chunk_len[order[q0]]);
      P.wv_ev0.push_back(P.n_ev_pad);
      for (int32_t l = 0; l < WAVE; ++l) {
        const int32_t c = l < nch ? order[q0 + l] : -1;
        P.wv_chunk.push_back(c);
        if (c >= 0) {
          P.chunk_wv[c] = P.n_wv;
          P.chunk_lane[c] = l;
        }
      }
      P.n_ev_pad += (int64_t)P.chunk_len[order[q0]] * WAVE;
      ++P.n_wv;
    }
    P.series_nwv[b] = P.n_wv - P.series_wv0[b];
  }
  // a layout that pads the events many times over (one chunk per series puts
  // one lane of a work wave to use) is refused before its arrays are made
  if (P.n_ev_pad > 16 * P.n_events + (int64_t(1) << 24)) {
    err = "the event layout would hold " + std::to_string(P.n_ev_pad) + " padded events for " +
          std::to_string(P.n_events) + " events (one chunk per series uses one lane of 64; split the series in time)";
    return -7;
  }
  // interleaved event arrays
  P.dt.assign(P.n_ev_pad, 0.0);
  P.t.assign(P.n_ev_pad, 0.0);
  P.y.assign(P.n_ev_pad, 0.0);
  P.r.assign(P.n_ev_pad, 1.0);
  P.invd.assign(P.n_ev_pad, 0.0);
  P.info.assign(P.n_ev_pad, K_PAD);
  P.meas.assign(P.n_ev_pad, -1);
  std::atomic<int32_t> nextwv(0);
  auto filler = [&]() {
    for (;;) {
      const int32_t v = nextwv.fetch_add(1);
      if (v >= P.n_wv) break;
      const int32_t b = P.wv_series[v];
      const SeriesWork& w = work[b];
      for (int32_t l = 0; l < P.wv_nch[v]; ++l) {
        const int32_t c = P.wv_chunk[(int64_t)v * WAVE + l];
        const int64_t e0 = chunk_evstart[c];
        for (int32_t k = 0; k < P.chunk_len[c]; ++k) {
          const int64_t q = e0 + k;
          const Ev& e = w.ev[q];
          const int64_t at = P.wv_ev0[v] + (int64_t)k * WAVE + l;
          P.t[at] = e.t;
          P.dt[at] = (q == 0) ? 0.0 : e.t - w.ev[q - 1].t;
          uint32_t info = e.kind | (e.slot >= 0 ? ((uint32_t)e.slot << 2) : 0u) | (w.open_before[q] << 8);
          P.info[at] = info;
          if (e.kind == K_END || e.kind == K_INSTANT) {
            P.y[at] = y[e.n];
            P.r[at] = yerr[e.n] * yerr[e.n];
            P.meas[at] = e.n;
            if (e.kind == K_END) P.invd[at] = 1.0 / (t_end[e.n] - t_start[e.n]);
          } else {
            P.r[at] = 1.0;
          }
        }
        // pad the tail of the chunk at its end time
        const double tend = P.chunk_t1[c];
        for (int32_t k = P.chunk_len[c]; k < P.wv_len[v]; ++k) P.t[P.wv_ev0[v] + (int64_t)k * WAVE + l] = tend;
      }
    }
  };
  pool.clear();
  for (unsigned i = 1; i < nth; ++i) pool.emplace_back(filler);
  filler();
  for (auto& th : pool) th.join();
  return 0;
}

}  // namespace gpssm
