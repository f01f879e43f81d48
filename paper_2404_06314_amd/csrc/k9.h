// Shared-weight dense-block forward (see k9.hip).
#pragma once

#include <string>
#include <vector>

#include "circuit.h"
#include "kernels.h"

namespace qtm {

// Slots of a layered circuit: layer l, qubit q: RX reads inputs[rx[l n + q]],
// RY and RZ read weights[ry[...]], weights[rz[...]]; the entangler is the open
// CZ chain.
struct K9Layout {
  int n = 0, L = 0;
  std::vector<int32_t> rx, ry, rz;
};
// Device copies of the slot tables.
struct K9Dev {
  int n = 0, L = 0;
  const int32_t *rx = nullptr, *ry = nullptr, *rz = nullptr;
};

// Does the circuit have that form (n a multiple of 4, at least 12)?
bool k9_detect(const CircuitDesc &d, K9Layout &out, std::string &why);
// Workspace: matrix-core operand tables (floats), RX cosines and sines
// ([B][L][n] float2), observable partial rows per sample.
size_t k9_tab_floats(const K9Layout &k);
int k9_part_rows(const K9Layout &k);

// The forward pass: |0...0>, then per layer and block of 4 qubits the
// per-sample RX on the VALU and the shared dense block on the matrix cores,
// the CZ gates between blocks as signs; the last pass reads the observables
// and the norm; expvals normalised.  complex64 states.
hipError_t k9_forward(const K9Dev &k, const DevCircuit &d, int B, const double *x, const double *w, void *state,
                      float *tab, float2 *rxcs, double *part, double *out, hipStream_t s, SweepTimer *tm);

}  // namespace qtm
