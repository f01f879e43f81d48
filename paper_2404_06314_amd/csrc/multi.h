// Uneven-batch runtime: one persistent sweep kernel per direction over many
// circuits (one sample each), launched as a hipGraph.
#pragma once

#include <string>
#include <vector>

#include "kernels.h"

namespace qtm {

struct MultiItemIn {
  const CircuitDesc *desc;
  int kt, klo;
  // offsets of the item in the packed caller arrays (elements) and in the
  // packed complex64 state (amplitudes)
  int64_t in_off, w_off, out_off, st_off;
};

struct MultiRuntime;

// Host planning only (no device work).  nullptr and `err` on failure.
MultiRuntime *multi_runtime_create(const std::vector<MultiItemIn> &items, std::string &err);
void multi_runtime_destroy(MultiRuntime *m);
// The first call on a device uploads the tables and builds the graphs.  With
// a timer, the kernels are launched one by one and the persistent kernel is
// bracketed by tm->before / tm->after (kind 0 forward, 1 backward).
hipError_t multi_runtime_forward(MultiRuntime *m, const double *x, const double *w, double *out,
                                 void *state, hipStream_t s, SweepTimer *tm);
hipError_t multi_runtime_backward(MultiRuntime *m, const double *x, const double *w, const double *G,
                                  void *state, double *gw, double *gx, hipStream_t s, SweepTimer *tm);
// The HIP call behind the last error of this runtime.
const char *multi_runtime_where(const MultiRuntime *m);
// Number of work units of a pass (-1 before the first call).
int multi_runtime_units(const MultiRuntime *m, int pass);

}  // namespace qtm
