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

// Functions used by both the planner (host) and the kernels (device).
#ifdef __HIP__
#define QTM_HOST_DEVICE __host__ __device__
#else
#define QTM_HOST_DEVICE
#endif

namespace qtm {

enum GateType : int32_t { G_RX = 0, G_RY = 1, G_RZ = 2, G_CNOT = 3, G_CZ = 4 };
enum GateSrc : int32_t { S_NONE = 0, S_INPUT = 1, S_WEIGHT = 2 };

struct Gate {
  int32_t type, q0, q1, src, index;
};

inline bool is_rotation(int t) { return t == G_RX || t == G_RY || t == G_RZ; }

// Register bits per stage: each thread holds 2^kRegBits amplitudes of a tile.
constexpr int kRegBits = 4;
constexpr int kRegs = 1 << kRegBits;
constexpr int kMaxTileQubits = 12;
constexpr int kMinTileQubits = kRegBits;
// At most this many fused blocks per sweep: their matrices are staged in LDS
// and their gradient accumulators live in registers.
constexpr int kMaxSweepBlocks = 96;

// Fused-op kinds (host) and device op codes.
enum FKind : int32_t { FK_BLOCK = 0, FK_CNOT = 1, FK_CZ = 2 };
enum OpCode : int32_t { OP_U1 = 1, OP_CNOT = 2, OP_DIAG = 3 };

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
  std::vector<uint64_t> masks;
  // parameter occurrences (rotations) in gate order
  std::vector<int32_t> occ_gate;  // occurrence -> gate index
  std::vector<int32_t> gate_occ;  // gate -> occurrence or -1
};

// Returns 0 or a QTM_ERR_* code with a message.
int validate_and_build(int32_t n, const Gate *gates, int32_t n_gates, int32_t n_inputs,
                       int32_t n_weights, const uint64_t *masks, int32_t n_obs,
                       CircuitDesc &out, std::string &err);

// Plan the fused path for tile size kt (<= n) with klo contiguous low qubits.
Plan make_plan(const CircuitDesc &c, int32_t kt, int32_t klo);

// Check the plan's invariants (each gate scheduled once, dependency order,
// stage/tile membership).  Returns "" when valid.
std::string check_plan(const CircuitDesc &c, const Plan &p);

// JSON description of a plan (diagnostics and tests).
std::string plan_json(const CircuitDesc &c, const Plan &p);

// --- device program -------------------------------------------------------
//
// Flat int32 program read by the fused kernels (uniform, scalar loads).
//
// sweep header at sweep_off[s]:
//   [0] n_stages  [1] n_outer  [2] n_gslots (this sweep)  [3] n_mats (matrices used)
//   [4 .. 4+30)        outer global positions (n_outer used)
//   [34 .. 34+12)      tile global positions (kt used)
//   [46 .. 46+16)      load layout: global offset of register j
//   [62 .. 62+16)      load layout: LDS (swizzled) offset of register j
//   [78 .. 78+12)      load layout: global position of thread bit i
//   [90 .. 90+n_st)    stage offsets
//   then n_gslots global slot ids, then n_mats global block ids (the
//   sweep-local matrix slots, staged in LDS by the kernels)
// stage at stage_off:
//   [0] n_ops  [1] flags (bit 0: some diag op has a per-thread part, whose
//       sign is applied once at the end of the stage)  [2] offset of this
//       stage's per-thread table in Program::thr  [3] reserved
//   [4 .. 20)   LDS (swizzled) offset of register j
//   [20 .. 36)  global offset of register j
//   [36 .. 40)  tile-local positions of the 4 register bits, ascending
//   [40 ..)     ops, 4 int32 each: {code, a, b, c}
//     OP_U1:   a = register bit, b = sweep-local matrix slot, c = sweep-local gslot or -1
//     OP_CNOT: a = target register bit, b = 0 (control is register bit c) or
//              1 (control is global qubit c)
//     OP_DIAG: a = offset of a diag record (below), b, c unused
//   diag record for a set of CZ pairs with sign (-1)^Q(x), Q(x) = sum over
//   pairs of x_a x_b: for x = G | W_j (G the thread's bits, W_j register j's
//   bits) Q(x) = Q(G) + sum_b j_b parity(G & C_b) + Q(W_j) (mod 2).
//     [0] n_groups, then (d, mask) pairs with Q(G) = parity of
//         sum_g popcount(G & (G >> d_g) & mask_g);
//     then C_0..C_3 (per register bit, 0 = no term), then a 16-bit mask of
//     Q(W_j) over j.
// Program::thr: for stage s and thread t, the global bits of the thread's
// register-0 amplitude (without the tile base).
constexpr int kSwOuter = 4, kSwTile = 34, kSwLoadG = 46, kSwLoadL = 62, kSwLoadTb = 78,
              kSwStages = 90;
constexpr int kStFlags = 1, kStThr = 2, kStLds = 4, kStGlob = 20, kStRegPos = 36, kStOps = 40;

// Swizzle of a tile-local index into its LDS slot: XOR of the low 5 bits with
// two higher 5-bit fields.  It is GF(2)-linear, so swz(a ^ b) = swz(a) ^ swz(b).
QTM_HOST_DEVICE inline uint32_t lds_swizzle(uint32_t i) { return i ^ ((i >> 5) & 31u) ^ ((i >> 10) & 31u); }

struct Program {
  std::vector<int32_t> code;
  std::vector<int32_t> thr;  // per-stage per-thread global offsets
  std::vector<int32_t> sweep_off_fwd;  // forward order
  std::vector<int32_t> sweep_off_bwd;  // backward order (stages and ops reversed)
  int32_t max_gslots_per_sweep = 0;
};

Program encode_program(const CircuitDesc &c, const Plan &p);

// Everything the fused kernels read for one (circuit, kt, klo), in host
// memory: the program, the block records of the matrix prep, the
// occurrence -> gradient slot map and the two sign tables.
struct HostPlan {
  int32_t kt = 0, klo = 0, n_blocks = 0, n_gslots = 0, max_gslots = 0, n_sweeps = 0;
  Program prog;
  std::vector<int32_t> blk;        // per block: [q, ng, (type, src, idx, occ) x ng]
  std::vector<int32_t> blk_off;    // block -> offset in blk
  std::vector<int32_t> occ_gslot;  // occurrence -> gradient slot
  std::vector<float> obs_sgn;      // [(M+1)][16] signs of the last forward stage
  std::vector<double> seed_sgn;    // [M][16] signs of the first backward load layout
};

// Plan, check and encode.  Returns "" or the planner's error.
std::string build_host_plan(const CircuitDesc &c, int32_t kt, int32_t klo, HostPlan &out);

}  // namespace qtm
