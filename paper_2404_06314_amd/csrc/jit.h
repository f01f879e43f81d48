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
// registers the matrix-core instructions leave them in.  Knowing the plan
// also lets each sweep skip the tiles and amplitudes that are still 0
// (SweepLive below).
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
  int nwg_full = 0;   // row stride of the per-workgroup partial buffers
  int renorm = 0;     // periodic renormalisation every `renorm` sweeps (0 = off; see FwdArgs / BwdArgs)
  std::vector<uint64_t> masks;
  const HostPlan *hp = nullptr;
};

// HIP source of forward / backward sweep `sweep` (argument FwdArgs / BwdArgs
// as for the compiled kernels).  Its kernel is named by jit_kernel_name:
// qtm_jit_fwd / qtm_jit_bwd with the tile configuration appended
// (`_t<kt>l<klo>`, plus `_c128` for complex128), so that profiles tell
// configurations apart.
// share = false: the backward keeps separate LDS tiles for psi and lambda
// (the fallback for kernels that the shared form makes spill).
std::string jit_source(const JitSpec &sp, int dir, int sweep, bool share = true);
std::string jit_kernel_name(const JitSpec &sp, int dir);

// Work of a specialised sweep restricted to the amplitudes that can be
// nonzero (Program::excited): with D_in / D_out the qubits not excited before
// / after forward sweep s, the state is 0 wherever a bit of D_out is set
// throughout the sweep, and the backward needs psi and lambda only where no
// bit of D_out is set (each gate keeps the bits of D_out, so that part of
// lambda evolves on its own, and every gradient term pairs it with psi).
struct SweepLive {
  uint64_t skip = 0;     // tile-outer qubits: tiles with one of them set are not run
  uint64_t zin = 0;      // amplitudes with one of these bits set load as 0 (not read)
  uint64_t nostore = 0;  // amplitudes with one of these bits set are not stored
  uint64_t din = 0;      // D_in of the forward sweep
  int64_t tiles = 0;     // tiles run per sample
  int nwg = 0;           // workgroups launched per sample
};
SweepLive sweep_live(const JitSpec &sp, int dir, int sweep);

// Static LDS bytes of that kernel.
size_t jit_lds_bytes(const JitSpec &sp, int dir, int sweep, bool share = true);

struct JitKernel {
  std::vector<char> code;  // code object
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int vgprs = -1, scratch = -1;
};

struct JitSweeps {
  std::vector<JitKernel> k[2];  // [dir][sweep]
  std::vector<int> nwg[2];      // workgroups per sample of each launch
  std::vector<int32_t> gs_rows;  // per gradient slot: partial rows its sweep writes
  int32_t *gs_rows_dev = nullptr;
  bool direct_obs = false;      // the last forward sweep writes <Z_m> itself
  bool direct_grad = false;     // the backward writes the per-rotation gradients itself
  bool direct_prep = false;     // the forward prepares the gate matrices itself
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
