// Test driver for the host-side planner: reads a batch from binary files,
// builds the plan and prints its tables as "name value value ..." lines.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_2601_02527_amd/csrc/plan.h"

using namespace gpssm;

static std::vector<char> slurp(const std::string& f) {
  FILE* p = std::fopen(f.c_str(), "rb");
  if (!p) std::exit(3);
  std::fseek(p, 0, SEEK_END);
  const long n = std::ftell(p);
  std::fseek(p, 0, SEEK_SET);
  std::vector<char> b(n);
  if (n && std::fread(b.data(), 1, n, p) != (size_t)n) std::exit(3);
  std::fclose(p);
  return b;
}

template <class T>
static void put(const char* name, const std::vector<T>& v) {
  std::printf("%s", name);
  for (const T& x : v) std::printf(" %.17g", (double)x);
  std::printf("\n");
}

int main(int argc, char** argv) {
  if (argc < 6) return 2;
  const std::string d = argv[1];
  PlanOptions opt;
  opt.chunk_min = std::atoi(argv[2]);
  opt.chunk_target = std::atoi(argv[3]);
  opt.single_chunk = std::atoi(argv[4]);
  opt.target_chunks = std::atoll(argv[5]);
  const auto o = slurp(d + "/offs.bin"), a = slurp(d + "/ts.bin"), e = slurp(d + "/te.bin"), y = slurp(d + "/y.bin"),
             r = slurp(d + "/yerr.bin");
  HostPlan P;
  std::string err;
  const int rc = build_plan((int64_t)(o.size() / 8 - 1), (const int64_t*)o.data(), (const double*)a.data(),
                            (const double*)e.data(), (const double*)y.data(), (const double*)r.data(), opt, P, err);
  std::printf("rc %d\n", rc);
  if (rc) return 0;
  std::printf("scalars %lld %lld %d %d %d %d\n", (long long)P.n_events, (long long)P.n_ev_pad, P.n_chunks, P.n_seg,
              P.n_wv, P.max_slots);
  put("t", P.t);
  put("info", P.info);
  put("meas", P.meas);
  put("seg_chunk0", P.seg_chunk0);
  put("seg_nch", P.seg_nch);
  put("wv_series", P.wv_series);
  put("wv_nch", P.wv_nch);
  put("wv_len", P.wv_len);
  put("wv_chunk", P.wv_chunk);
  put("wv_ev0", P.wv_ev0);
  put("chunk_len", P.chunk_len);
  put("chunk_series", P.chunk_series);
  put("chunk_wv", P.chunk_wv);
  put("chunk_lane", P.chunk_lane);
  put("chunk_first", P.chunk_first);
  put("series_chunk0", P.series_chunk0);
  put("series_nch", P.series_nch);
  put("series_seg0", P.series_seg0);
  put("series_nseg", P.series_nseg);
  put("series_wv0", P.series_wv0);
  put("series_nwv", P.series_nwv);
  put("series_slots", P.series_slots);
  put("grp_seg0", P.grp_seg0);
  put("grp_nseg", P.grp_nseg);
  put("series_grp0", P.series_grp0);
  put("series_ngrp", P.series_ngrp);
  return 0;
}
