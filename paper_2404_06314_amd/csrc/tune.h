// Autotuner interface between the C-ABI layer and autotune.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "qtm.h"

namespace qtm {

struct TuneInfo {
  int n = 0, n_inputs = 0, n_weights = 0, n_obs = 0;
  std::string signature;  // hash of the gate list, observables and sizes
};

// Search tile size, contiguous low qubits and generic / specialised sweep
// kernels for (batch, precision); install the fastest candidate that
// reproduces the complex128 per-gate reference.  report: JSON summary.
int autotune(qtm_circuit_t c, const TuneInfo &info, int32_t batch, int32_t precision, hipStream_t stream,
             bool use_cache, std::string &report);

}  // namespace qtm
