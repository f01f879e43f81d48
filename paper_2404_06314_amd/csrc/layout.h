// Tile, stage and program-layout constants shared by the planner (host), the
// compiled kernels and the runtime-specialised sweep kernels (which are
// compiled from source at run time, so this header has no host-only
// dependencies).
#pragma once

#ifndef __HIPCC_RTC__
#include <stdint.h>
#else
// runtime compilation: the fixed-width integer types live in hiprtc's namespace
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
typedef unsigned long uintptr_t;
#endif

// Functions used by both the planner (host) and the kernels (device).
#ifdef __HIP__
#define QTM_HOST_DEVICE __host__ __device__
#else
#define QTM_HOST_DEVICE
#endif

namespace qtm {

// Register bits per stage: each thread holds 2^kRegBits amplitudes of a tile.
constexpr int kRegBits = 4;
constexpr int kRegs = 1 << kRegBits;
constexpr int kMaxTileQubits = 12;
constexpr int kMinTileQubits = kRegBits;
// At most this many fused blocks per sweep: their matrices and gradient
// accumulators are staged in LDS.
constexpr int kMaxSweepBlocks = 96;

enum OpCode : int32_t { OP_U1 = 1, OP_CNOT = 2, OP_DIAG = 3, OP_U1_LAST = 4, OP_U1_FIRST = 5 };

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
//     OP_U1_LAST (backward only): as OP_U1 for a block that is the first op
//              on its qubit in forward order, i.e. the last one the
//              backward meets on that qubit: its transition-matrix sums are
//              taken, its un-apply is skipped.  Every later op of the
//              backward acts on other qubits and commutes with it, so
//              keeping the block applied on both psi and lambda changes no
//              later <lambda|P|psi>, and nothing reads the final states.
//              The specialised backward sweeps un-apply it anyway in every
//              sweep but the last one they run: the next sweep takes the
//              qubit's |1> half as 0 (not excited yet), which holds only
//              once the block is undone.
//     OP_U1_FIRST (forward only): as OP_U1 for a block that is the first op
//              on its qubit: every amplitude with that qubit's bit set is
//              still 0, so only the matrix columns of the |0> inputs are
//              needed.
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

}  // namespace qtm
