// Interface of the time-parallel combination of chunk summaries (scan.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace gpssm {

// doubles of a composed summary (A, b, C, eta, J) for N SHO states
GPD constexpr int elem_fields(int N) { return N * N + N + N * (N + 1) / 2 + N + N * (N + 1) / 2; }

// workspace, all field-major ([field][chunk] or [field][segment])
struct ScanWork {
  const double* summ;  // chunk summaries (elem_fields + 1 per chunk)
  double* pre;         // inclusive prefix compositions within each segment
  double* suf;         // inclusive suffix compositions within each segment
  double* segtot;      // segment totals
  double* segstate;    // filtered SHO state at each segment start (N + N(N+1)/2)
  double* segfut;      // future information after each segment (J packed, then eta)
  double* bstate;      // filtered state at each chunk start
  double* badj;        // adjoint of the state at each chunk end
  double* bsmooth;     // smoother adjoint pair (lambda, Lambda) at each chunk end (may be null)
  double* segll;       // log-likelihood of each segment
  int32_t* segok;      // 1 when every combination of the segment succeeded
  // second scan level (null p2: one level), over groups of segments
  const DevPlan* p2;   // the plan seen by the second level (groups as segments, segments as chunks)
  double *pre2, *suf2, *grptot, *grpstate, *grpfut;
};

// loglik and status of the call are read from args (device memory)
void run_scan(int M, hipStream_t st, const DevPlan& p, const DevParams& pr, const ScanWork& w, const CallArgs* args,
              int back);

}  // namespace gpssm
