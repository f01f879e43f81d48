// Runtime-specialised sweep kernels.
//
// The compiled sweep kernels interpret the encoded program: per op they read
// its code, register bit, matrix slot and sign tables, and the register bit
// of a gate is a run-time value, so every op goes through a switch whose
// branches must leave the 16 amplitudes in the same registers.  For a fixed
// circuit all of that is known when the plan is made.  This module turns
// each sweep of a plan into HIP source with those values as literals (the
// same device helpers, instantiated for the op's register bit), compiles it
// with hiprtc and loads it as a module: straight-line code per stage, no op
// dispatch, and the compiler is free to keep amplitudes in whatever
// registers the matrix-core instructions leave them in.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "circuit.h"

namespace qtm {

struct JitSpec {
  int n = 0;          // qubits
  int kt = 0;         // tile qubits
  bool dbl = false;   // complex128 (else complex64)
  int M = 0;          // observables
  int n_blocks = 0;   // fused blocks (matrix table stride per sample)
  bool seed_add = false;  // backward: lam holds a bra term to add in the first sweep
  std::vector<uint64_t> masks;
  const HostPlan *hp = nullptr;
};

// HIP source of forward / backward sweep `sweep` (argument FwdArgs / BwdArgs
// as for the compiled kernels).  Its kernel is named by jit_kernel_name:
// qtm_jit_fwd / qtm_jit_bwd with the tile configuration appended
// (`_t<kt>l<klo>`, plus `_c128` for complex128), so that profiles tell
// configurations apart.
std::string jit_source(const JitSpec &sp, int dir, int sweep);
std::string jit_kernel_name(const JitSpec &sp, int dir);

// Static LDS bytes of that kernel.
size_t jit_lds_bytes(const JitSpec &sp, int dir, int sweep);

struct JitKernel {
  std::vector<char> code;  // code object
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int vgprs = -1, scratch = -1;
};

struct JitSweeps {
  std::vector<JitKernel> k[2];  // [dir][sweep]
  std::string name[2];          // kernel name per direction
  int device = -1;
  bool loaded = false;
  ~JitSweeps();
};

// Compile every sweep of both directions (host only, no device needed).
// Returns "" or the compiler's message.
std::string jit_compile(const JitSpec &sp, JitSweeps &out);
// Load the code objects on the current device (once).
hipError_t jit_load(JitSweeps &js);

}  // namespace qtm
