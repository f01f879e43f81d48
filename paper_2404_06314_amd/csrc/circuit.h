// Host-side circuit representation, validation and the fused-sweep planner.
//
// A circuit is the gate list of the paper's ansatz (Eq. (7)): rotations whose
// angle is read from an input slot (data encoding) or a weight slot
// (trainable), and CNOT / CZ entanglers.  The planner turns it into a
// program for the fused GPU path:
//
//   1. fusion: consecutive single-qubit rotations on one wire (no two-qubit
//      gate on that wire in between) become one 2x2 "block";
//   2. a dependency DAG over blocks, CNOTs and CZs that knows which pairs
//      commute (diagonal ops with each other, CNOTs sharing only a control or
//      only a target, diagonal ops on a CNOT's control);
//   3. sweeps: each sweep fixes a set T of `kt` tile qubits (always holding the
//      `klo` lowest qubits, so a tile row is contiguous in memory) and runs
//      every op whose target lies in T, as long as new ops become ready;
//   4. stages: inside a sweep, groups of ops whose targets lie in 4 tile
//      bits ("register bits"); between stages the tile is exchanged through
//      LDS so that the next stage's 4 bits are held in registers.
//
// CZ gates are diagonal: they need no qubit of the tile and are applied as a
// sign computed from the amplitude's global index.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "layout.h"

namespace qtm {

enum GateType : int32_t {
  G_RX = 0, G_RY = 1, G_RZ = 2, G_CNOT = 3, G_CZ = 4,
  // fixed one-qubit gates
  G_H = 5, G_X = 6, G_Y = 7, G_Z = 8, G_S = 9, G_SDG = 10, G_T = 11, G_TDG = 12, G_SX = 13,
  // controlled rotations: q0 control, q1 target
  G_CRX = 14, G_CRY = 15, G_CRZ = 16
};
enum GateSrc : int32_t { S_NONE = 0, S_INPUT = 1, S_WEIGHT = 2, S_SCALED = 3 };

struct Gate {
  int32_t type, q0, q1, src, index;
};

inline bool is_rotation(int t) { return t == G_RX || t == G_RY || t == G_RZ; }
inline bool is_fixed(int t) { return t >= G_H && t <= G_SX; }
inline bool is_crot(int t) { return t >= G_CRX && t <= G_CRZ; }
inline bool is_param(int t) { return is_rotation(t) || is_crot(t); }
// diagonal in the computational basis (commutes with CZ and CNOT controls)
inline bool is_diag1(int t) { return t == G_RZ || t == G_Z || t == G_S || t == G_SDG || t == G_T || t == G_TDG; }

// Fused-op kinds (host) and device op codes.
enum FKind : int32_t { FK_BLOCK = 0, FK_CNOT = 1, FK_CZ = 2 };

struct FOp {
  int32_t kind = FK_BLOCK;
  int32_t q0 = 0, q1 = 0;      // block: q0 = qubit; CNOT: q0 ctl, q1 tgt; CZ: pair
  std::vector<int32_t> gates;  // gate indices (block: in application order)
  bool diagonal = false;       // CZ, or a block of RZ only
  bool has_param = false;
  int32_t block = -1;          // block id (FK_BLOCK)
  int32_t gslot = -1;          // global gradient slot of a parameterised block
  int32_t target() const { return kind == FK_BLOCK ? q0 : (kind == FK_CNOT ? q1 : -1); }
};

// One stage: 4 register bits (tile-local positions) and its ops (indices into
// Plan::ops, in execution order).  CZs of one stage are merged into a single
// diagonal op.
struct Stage {
  int32_t regpos[kRegBits];
  std::vector<int32_t> ops;
};

struct Sweep {
  std::vector<int32_t> tile;  // global qubit of tile-local bit k (tile[k] = k for k < klo)
  std::vector<Stage> stages;
  std::vector<int32_t> gslots;  // parameterised blocks of this sweep (global slot ids)
};

struct Plan {
  int32_t n = 0, kt = 0, klo = 0;
  std::vector<FOp> ops;
  std::vector<Sweep> sweeps;
  int32_t n_blocks = 0;
  int32_t n_gslots = 0;
  std::vector<int32_t> block_op;  // block id -> op index
};

struct CircuitDesc {
  int32_t n = 0, n_inputs = 0, n_weights = 0;
  std::vector<Gate> gates;
  // Observables as Pauli strings (X-part, Z-part; Y sets both bits).  masks
  // is what the sweeps and the diagonal kernels evaluate: the Z-part of a
  // Z string, and 0 (the identity) for a string with X or Y factors, whose
  // value and bra term the off-diagonal Pauli kernels supply.
  std::vector<uint64_t> masks;
  std::vector<uint64_t> pauli_x, pauli_z;
  bool has_crot() const {
    for (const Gate &g : gates)
      if (is_crot(g.type)) return true;
    return false;
  }
  bool has_offdiag() const {
    for (uint64_t x : pauli_x)
      if (x) return true;
    return false;
  }
  // parameter occurrences (rotations) in gate order
  std::vector<int32_t> occ_gate;  // occurrence -> gate index
  std::vector<int32_t> gate_occ;  // gate -> occurrence or -1
};

// Parameter slot -> rotation occurrences (CSR, construction order).  A
// weight-scaled input (S_SCALED) occurs in both lists; its entry carries the
// slot of the other factor of the angle: in the weight list the input index
// (d angle / d weight = inputs[b][fac]), in the input list the weight index
// (d angle / d input = weights[fac]); -1 where the derivative is 1.
struct ParamCsr {
  std::vector<int32_t> w_ptr, w_list, w_fac, x_ptr, x_list, x_fac;
};
ParamCsr param_csr(const CircuitDesc &c);

// Returns 0 or a QTM_ERR_* code with a message.
int validate_and_build(int32_t n, const Gate *gates, int32_t n_gates, int32_t n_inputs,
                       int32_t n_weights, const uint64_t *zmasks, const uint64_t *xmasks,
                       int32_t n_obs, CircuitDesc &out, std::string &err);

// Plan the fused path for tile size kt (<= n) with klo contiguous low qubits.
// zero_skip > 0: plan for kernels that skip all-zero tiles (the sweeps'
// tiles are chosen by an estimated cost that counts only the tiles that
// run, with zero_skip the HBM traffic of a full-state sweep pair in units of
// one fused block applied to the whole state); 0: each sweep takes the tile
// that runs the most ops.
Plan make_plan(const CircuitDesc &c, int32_t kt, int32_t klo, int32_t zero_skip = 0);

// Check the plan's invariants (each gate scheduled once, dependency order,
// stage/tile membership).  Returns "" when valid.
std::string check_plan(const CircuitDesc &c, const Plan &p);

// JSON description of a plan (diagnostics and tests).
std::string plan_json(const CircuitDesc &c, const Plan &p);

struct Program {
  std::vector<int32_t> code;
  std::vector<int32_t> thr;  // per-stage per-thread global offsets
  std::vector<int32_t> sweep_off_fwd;  // forward order
  std::vector<int32_t> sweep_off_bwd;  // backward order (stages and ops reversed)
  int32_t max_gslots_per_sweep = 0;
  // Per forward sweep: the qubits excited by its end, i.e. the target of a
  // non-diagonal block or of a CNOT in it or an earlier sweep.  The state
  // starts at |0...0>, and diagonal gates and CNOT controls never move
  // weight onto a set bit of a qubit not yet excited, so at every point of
  // sweep s the amplitudes with such a bit set are exactly 0.
  std::vector<uint64_t> excited;
};

Program encode_program(const CircuitDesc &c, const Plan &p);

// Everything the fused kernels read for one (circuit, kt, klo), in host
// memory: the program, the block records of the matrix prep, the
// occurrence -> gradient slot map and the two sign tables.
struct HostPlan {
  int32_t kt = 0, klo = 0, n_blocks = 0, n_gslots = 0, max_gslots = 0, n_sweeps = 0;
  int32_t zero_skip = 0;  // > 0: planned for kernels that skip all-zero tiles (make_plan)
  Program prog;
  std::vector<int32_t> blk;        // per block: [q, ng, (type, src, idx, widx, occ) x ng]
  std::vector<int32_t> blk_off;    // block -> offset in blk
  std::vector<int32_t> occ_gslot;  // occurrence -> gradient slot
  std::vector<float> obs_sgn;      // [(M+1)][16] signs of the last forward stage
  std::vector<double> seed_sgn;    // [M][16] signs of the first backward load layout
};

// Plan, check and encode.  Returns "" or the planner's error.
std::string build_host_plan(const CircuitDesc &c, int32_t kt, int32_t klo, HostPlan &out,
                            int32_t zero_skip = 0);

}  // namespace qtm
