// Device building blocks of the fused sweeps, shared by the batched kernels
// (one circuit, B samples) and the persistent uneven-batch kernels (many
// circuits, one sample each): the FP64 matrix prep of a fused block, the
// register-level gate ops, and the argument blocks the sweep bodies
// (sweep_fwd.inc, sweep_bwd.inc) read.
#pragma once

#include "device_common.h"
#include "layout.h"

namespace qtm {

// ---------------------------------------------------------------------------
// matrix prep: U = G_last ... G_first per (sample, block), FP64, stored in R;
// for each rotation j of the block, P'_j = A_j P_j A_j^dag with A_j the
// block's rotations after j, stored as (px, py, pz): P'_j = px X + py Y + pz Z.

struct CD {
  double x, y;
};
__device__ __forceinline__ CD cd_mul(CD a, CD b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ CD cd_add(CD a, CD b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ CD cd_conj(CD a) { return {a.x, -a.y}; }
struct MD {
  CD m[2][2];
};
__device__ __forceinline__ MD md_mul(const MD &a, const MD &b) {
  MD r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = cd_add(cd_mul(a.m[i][0], b.m[0][j]), cd_mul(a.m[i][1], b.m[1][j]));
  return r;
}
__device__ __forceinline__ MD md_adj(const MD &a) {
  MD r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = cd_conj(a.m[j][i]);
  return r;
}
__device__ __forceinline__ MD md_rot(int type, double t) {
  double s, c;
  sincos(0.5 * t, &s, &c);
  MD r;
  if (type == 0) {
    r.m[0][0] = {c, 0}; r.m[0][1] = {0, -s}; r.m[1][0] = {0, -s}; r.m[1][1] = {c, 0};
  } else if (type == 1) {
    r.m[0][0] = {c, 0}; r.m[0][1] = {-s, 0}; r.m[1][0] = {s, 0}; r.m[1][1] = {c, 0};
  } else {
    r.m[0][0] = {c, -s}; r.m[0][1] = {0, 0}; r.m[1][0] = {0, 0}; r.m[1][1] = {c, s};
  }
  return r;
}
__device__ __forceinline__ MD md_fixed(int type) {
  double re[4], im[4];
  fixed_gate(type, re, im);
  MD r;
  for (int k = 0; k < 4; ++k) r.m[k >> 1][k & 1] = {re[k], im[k]};
  return r;
}
// Matrix of gate record entry e: a rotation (types 0-2) at angle t, or a
// fixed gate (types 5-13).
__device__ __forceinline__ MD md_gate(int type, double t) { return type <= 2 ? md_rot(type, t) : md_fixed(type); }
__device__ __forceinline__ MD md_pauli(int type) {
  MD r;
  r.m[0][0] = r.m[0][1] = r.m[1][0] = r.m[1][1] = {0, 0};
  if (type == 0) { r.m[0][1] = {1, 0}; r.m[1][0] = {1, 0}; }
  else if (type == 1) { r.m[0][1] = {0, -1}; r.m[1][0] = {0, 1}; }
  else { r.m[0][0] = {1, 0}; r.m[1][1] = {-1, 0}; }
  return r;
}

// One fused block of one sample: U = G_last ... G_first into *mat and, if
// coef is set, the (px, py, pz) of every rotation j at coef[3 * occ_j].
// blk record: [q, ng, (type, src, idx, widx, occ) x ng]; x is the sample's
// input row.  The angle is x[idx] (src 1), w[idx] (src 2) or the scaled
// input w[widx] * x[idx] (src 3, Eq. (7)); fixed gates have src 0 and
// occ -1.
constexpr int kBlkGate = 5;
template <typename R>
__device__ __forceinline__ void prep_block(const int32_t *__restrict__ r, const double *__restrict__ x,
                                           const double *__restrict__ w, M2<R> *__restrict__ mat,
                                           double *__restrict__ coef) {
  const int ng = r[1];
  auto ang = [&](int g) {
    const int32_t *e = r + 2 + kBlkGate * g;
    if (e[1] == 0) return 0.0;
    if (e[1] == 3) return w[e[3]] * x[e[2]];
    return e[1] == 1 ? x[e[2]] : w[e[2]];
  };
  // From the last gate back to the first: when rotation g's coefficients
  // are taken, A is the product of the gates after it, and at the end A is
  // the block's unitary (one sine and cosine per gate).
  MD A;
  A.m[0][0] = {1, 0}; A.m[0][1] = {0, 0}; A.m[1][0] = {0, 0}; A.m[1][1] = {1, 0};
  for (int g = ng - 1; g >= 0; --g) {
    const int32_t *e = r + 2 + kBlkGate * g;
    if (coef && e[4] >= 0) {
      MD P = md_mul(md_mul(A, md_pauli(e[0])), md_adj(A));
      double *cf = coef + (int64_t)e[4] * 3;
      cf[0] = P.m[1][0].x;
      cf[1] = P.m[1][0].y;
      cf[2] = P.m[0][0].x;
    }
    A = md_mul(A, md_gate(e[0], ang(g)));
  }
  M2<R> o;
  o.a = {(R)A.m[0][0].x, (R)A.m[0][0].y};
  o.b = {(R)A.m[0][1].x, (R)A.m[0][1].y};
  o.c = {(R)A.m[1][0].x, (R)A.m[1][0].y};
  o.d = {(R)A.m[1][1].x, (R)A.m[1][1].y};
  *mat = o;
}

// ---------------------------------------------------------------------------
// register-level ops

template <typename R, int P>
__device__ __forceinline__ void u1_bit(Cx<R> (&v)[kRegs], const M2<R> &m) {
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if (!(j & (1 << P))) apply_m2(m, v[j], v[j | (1 << P)]);
}
template <typename R, int P>
__device__ __forceinline__ void u1_bit_adj(Cx<R> (&v)[kRegs], const M2<R> &m) {
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if (!(j & (1 << P))) apply_m2_adj(m, v[j], v[j | (1 << P)]);
}
template <typename R>
__device__ __forceinline__ void u1(Cx<R> (&v)[kRegs], int p, const M2<R> &m) {
  switch (p) {
    case 0: u1_bit<R, 0>(v, m); break;
    case 1: u1_bit<R, 1>(v, m); break;
    case 2: u1_bit<R, 2>(v, m); break;
    default: u1_bit<R, 3>(v, m); break;
  }
}
template <typename R>
__device__ __forceinline__ void u1_adj(Cx<R> (&v)[kRegs], int p, const M2<R> &m) {
  switch (p) {
    case 0: u1_bit_adj<R, 0>(v, m); break;
    case 1: u1_bit_adj<R, 1>(v, m); break;
    case 2: u1_bit_adj<R, 2>(v, m); break;
    default: u1_bit_adj<R, 3>(v, m); break;
  }
}

// Transition-matrix components of one pair (v0, v1) / (l0, l1), one fused
// multiply-add per product:
//   tx += Im(v0 conj l1 + v1 conj l0), ty += Re(v0 conj l1 - v1 conj l0),
//   tz += Im(v0 conj l0 - v1 conj l1).
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename R>
__device__ __forceinline__ void tpair(const Cx<R> &p0, const Cx<R> &p1, const Cx<R> &l0, const Cx<R> &l1,
                                      R &tx, R &ty, R &tz) {
  tx = fmadd(p0.y, l1.x, tx);
  tx = fmadd(-p0.x, l1.y, tx);
  tx = fmadd(p1.y, l0.x, tx);
  tx = fmadd(-p1.x, l0.y, tx);
  ty = fmadd(p0.x, l1.x, ty);
  ty = fmadd(p0.y, l1.y, ty);
  ty = fmadd(-p1.x, l0.x, ty);
  ty = fmadd(-p1.y, l0.y, ty);
  tz = fmadd(p0.y, l0.x, tz);
  tz = fmadd(-p0.x, l0.y, tz);
  tz = fmadd(-p1.y, l1.x, tz);
  tz = fmadd(p1.x, l1.y, tz);
}

// --- complex64 gates on the matrix cores -----------------------------------
//
// A 2x2 complex gate [[a, b], [c, d]] acting on one pair (v0, v1) is the 4x4
// real matrix M on (re0, im0, re1, im1):
//   row 0: ( a.x, -a.y,  b.x, -b.y)    row 1: ( a.y,  a.x,  b.y,  b.x)
//   row 2: ( c.x, -c.y,  d.x, -d.y)    row 3: ( c.y,  c.x,  d.y,  d.x)
// v_mfma_f32_4x4x1_16b_f32 computes, for every 4-lane block, the outer product
// D[i][j] += A(lane 4b + i) * B(lane 4b + j) with D[i] held in register i of
// lane 4b + j.  With A = column k of M in "row = lane & 3" order and B = the
// k-th component of each lane's own pair, four instructions (k = 0..3) give
// every lane M times its pair: each lane's 8 pairs are 8 independent
// matrix-vector products, with no data moved between lanes.
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct MCols {
  float k0, k1, k2, k3;
};

__device__ __forceinline__ MCols mfma_cols(Cx<float> a, Cx<float> b, Cx<float> c, Cx<float> d,
                                           int row) {
  const Cx<float> p = row < 2 ? a : c;
  const Cx<float> q = row < 2 ? b : d;
  const bool odd = row & 1;
  return {odd ? p.y : p.x, odd ? p.x : -p.y, odd ? q.y : q.x, odd ? q.x : -q.y};
}

// A operand columns of a gate (adjoint = false) or of its conjugate transpose.
__device__ __forceinline__ MCols mfma_cols_m(const M2<float> &m, int row, bool adjoint) {
  return adjoint ? mfma_cols(Cx<float>{m.a.x, -m.a.y}, Cx<float>{m.c.x, -m.c.y},
                             Cx<float>{m.b.x, -m.b.y}, Cx<float>{m.d.x, -m.d.y}, row)
                 : mfma_cols(m.a, m.b, m.c, m.d, row);
}

// Entry (row, k) of the 4x4 real form of a gate (or of its conjugate
// transpose) given as the 8 floats a.x a.y b.x b.y c.x c.y d.x d.y.
__device__ __forceinline__ float mfma_entry(const float *e, int row, int k, bool adjoint) {
  Cx<float> a{e[0], e[1]}, b{e[2], e[3]}, c{e[4], e[5]}, d{e[6], e[7]};
  if (adjoint) {
    const Cx<float> t = b;
    a = Cx<float>{a.x, -a.y};
    b = Cx<float>{c.x, -c.y};
    c = Cx<float>{t.x, -t.y};
    d = Cx<float>{d.x, -d.y};
  }
  const MCols m = mfma_cols(a, b, c, d, row);
  return k == 0 ? m.k0 : k == 1 ? m.k1 : k == 2 ? m.k2 : m.k3;
}

// A operand columns of slot `slot` from a table of expanded gates
// ([slot][row][k] floats); arow = 4 * (lane & 3).
__device__ __forceinline__ MCols lds_cols(const float *tab, int slot, int arow) {
  const floatx4 x = *reinterpret_cast<const floatx4 *>(tab + slot * 16 + arow);
  return MCols{x[0], x[1], x[2], x[3]};
}

template <int P>
__device__ __forceinline__ constexpr int pair_lo(int p) {
  return ((p >> P) << (P + 1)) | (p & ((1 << P) - 1));
}

// Sign flips of A operand values (bit 31 of m), e.g. rows 2-3 of the
// expanded gate, which negates the |1> half of every output pair.
__device__ __forceinline__ MCols mcols_xor(const MCols &a, uint32_t m) {
  auto f = [m](float x) { return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x) ^ m); };
  return MCols{f(a.k0), f(a.k1), f(a.k2), f(a.k3)};
}

// Gate on register bit P of NS register tiles with the matrix cores; pair p
// (registers pair_lo<P>(p) and that | 2^P) uses A1 if bit p of SEL is set,
// else A0 (A1 carries the sign of a diagonal op folded into the output).
// LOW0: the inputs of the |1> half are known to be 0 (the gate is the first
// on its qubit), so only the two accumulation steps of the |0> half run.
template <int P, int NS, int SEL, bool LOW0 = false>
__device__ __forceinline__ void u1_mfma_bit_sel(Cx<float> (*const *vs)[kRegs], const MCols &A0,
                                                const MCols &A1) {
  constexpr int NP = kRegs / 2, CH = 4;  // 4 independent accumulation chains at a time
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int c0 = 0; c0 < NP; c0 += CH) {
      Cx<float>(&v)[kRegs] = *vs[s];
      floatx4 acc[CH];
#pragma unroll
      for (int p = 0; p < CH; ++p)
        acc[p] = __builtin_amdgcn_mfma_f32_4x4x1f32(((SEL >> (c0 + p)) & 1) ? A1.k0 : A0.k0,
                                                    v[pair_lo<P>(c0 + p)].x, zero, 0, 0, 0);
#pragma unroll
      for (int p = 0; p < CH; ++p)
        acc[p] = __builtin_amdgcn_mfma_f32_4x4x1f32(((SEL >> (c0 + p)) & 1) ? A1.k1 : A0.k1,
                                                    v[pair_lo<P>(c0 + p)].y, acc[p], 0, 0, 0);
      if constexpr (!LOW0) {
#pragma unroll
        for (int p = 0; p < CH; ++p)
          acc[p] = __builtin_amdgcn_mfma_f32_4x4x1f32(((SEL >> (c0 + p)) & 1) ? A1.k2 : A0.k2,
                                                      v[pair_lo<P>(c0 + p) | (1 << P)].x, acc[p], 0, 0, 0);
#pragma unroll
        for (int p = 0; p < CH; ++p)
          acc[p] = __builtin_amdgcn_mfma_f32_4x4x1f32(((SEL >> (c0 + p)) & 1) ? A1.k3 : A0.k3,
                                                      v[pair_lo<P>(c0 + p) | (1 << P)].y, acc[p], 0, 0, 0);
      }
#pragma unroll
      for (int p = 0; p < CH; ++p) {
        v[pair_lo<P>(c0 + p)] = Cx<float>{acc[p][0], acc[p][1]};
        v[pair_lo<P>(c0 + p) | (1 << P)] = Cx<float>{acc[p][2], acc[p][3]};
      }
    }
}

template <int P, int NS>
__device__ __forceinline__ void u1_mfma_bit(Cx<float> (*const *vs)[kRegs], const MCols &A) {
  u1_mfma_bit_sel<P, NS, 0>(vs, A, A);
}

// Apply m (adjoint = false) or m^dag (adjoint = true) to register bit p of
// NS register tiles.
template <int NS>
__device__ __forceinline__ void u1_mfma(Cx<float> (*const *vs)[kRegs], int p, const M2<float> &m,
                                        bool adjoint, int row) {
  const MCols A = adjoint ? mfma_cols(Cx<float>{m.a.x, -m.a.y}, Cx<float>{m.c.x, -m.c.y},
                                      Cx<float>{m.b.x, -m.b.y}, Cx<float>{m.d.x, -m.d.y}, row)
                          : mfma_cols(m.a, m.b, m.c, m.d, row);
  switch (p) {
    case 0: u1_mfma_bit<0, NS>(vs, A); break;
    case 1: u1_mfma_bit<1, NS>(vs, A); break;
    case 2: u1_mfma_bit<2, NS>(vs, A); break;
    default: u1_mfma_bit<3, NS>(vs, A); break;
  }
}

// Backward block on register bit P: transition-matrix components of the
// states after the block, then the adjoint applied to psi and lambda.  The
// FMAs and the matrix-core instructions are kept in separate groups: on
// gfx950 a wave's VALU and MFMA work does not overlap, and issuing the two
// interleaved costs ~30% more than issuing them one group after the other
// (measured: 8 MFMA + 12 FMA per step take 150 cycles interleaved, 114
// grouped, 78 + 37 alone).
template <int P, int SEL>
__device__ __forceinline__ void bwd_u1_mfma_bit_sel(Cx<float> (&v)[kRegs], Cx<float> (&l)[kRegs],
                                                    const MCols &A0, const MCols &A1, float &tx,
                                                    float &ty, float &tz) {
  tx = ty = tz = 0.f;
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if (!(j & (1 << P))) {
      const Cx<float> p0 = v[j], p1 = v[j | (1 << P)], l0 = l[j], l1 = l[j | (1 << P)];
      tpair(p0, p1, l0, l1, tx, ty, tz);
    }
  __builtin_amdgcn_sched_barrier(0);
  Cx<float>(*const vs[2])[kRegs] = {&v, &l};
  u1_mfma_bit_sel<P, 2, SEL>(vs, A0, A1);
  __builtin_amdgcn_sched_barrier(0);
}
template <int P>
__device__ __forceinline__ void bwd_u1_mfma_bit(Cx<float> (&v)[kRegs], Cx<float> (&l)[kRegs],
                                                const MCols &A, float &tx, float &ty, float &tz) {
  bwd_u1_mfma_bit_sel<P, 0>(v, l, A, A, tx, ty, tz);
}

__device__ __forceinline__ void bwd_u1_mfma(Cx<float> (&v)[kRegs], Cx<float> (&l)[kRegs], int p,
                                            const M2<float> &m, int row, float &tx, float &ty,
                                            float &tz) {
  const MCols A = mfma_cols(Cx<float>{m.a.x, -m.a.y}, Cx<float>{m.c.x, -m.c.y},
                            Cx<float>{m.b.x, -m.b.y}, Cx<float>{m.d.x, -m.d.y}, row);
  switch (p) {
    case 0: bwd_u1_mfma_bit<0>(v, l, A, tx, ty, tz); break;
    case 1: bwd_u1_mfma_bit<1>(v, l, A, tx, ty, tz); break;
    case 2: bwd_u1_mfma_bit<2>(v, l, A, tx, ty, tz); break;
    default: bwd_u1_mfma_bit<3>(v, l, A, tx, ty, tz); break;
  }
}

// CNOT with target register bit P and control register bit C
template <typename R, int P, int C>
__device__ __forceinline__ void cnot_rr(Cx<R> (&v)[kRegs]) {
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if (!(j & (1 << P)) && (j & (1 << C))) {
      Cx<R> t = v[j];
      v[j] = v[j | (1 << P)];
      v[j | (1 << P)] = t;
    }
}
template <typename R, int P>
__device__ __forceinline__ void cnot_r(Cx<R> (&v)[kRegs], int c) {
  switch (c) {
    case 0: if (P != 0) cnot_rr<R, P, 0>(v); break;
    case 1: if (P != 1) cnot_rr<R, P, 1>(v); break;
    case 2: if (P != 2) cnot_rr<R, P, 2>(v); break;
    default: if (P != 3) cnot_rr<R, P, 3>(v); break;
  }
}
// CNOT with target register bit P, control fixed for the thread (on / off)
template <typename R, int P>
__device__ __forceinline__ void cnot_t(Cx<R> (&v)[kRegs], bool on) {
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if (!(j & (1 << P))) {
      Cx<R> a = v[j], b = v[j | (1 << P)];
      v[j] = on ? b : a;
      v[j | (1 << P)] = on ? a : b;
    }
}
template <typename R>
__device__ __forceinline__ void cnot_op(Cx<R> (&v)[kRegs], int p, int kind, int c, uint32_t gt) {
  if (kind == 0) {
    switch (p) {
      case 0: cnot_r<R, 0>(v, c); break;
      case 1: cnot_r<R, 1>(v, c); break;
      case 2: cnot_r<R, 2>(v, c); break;
      default: cnot_r<R, 3>(v, c); break;
    }
  } else {
    const bool on = (gt >> c) & 1u;
    switch (p) {
      case 0: cnot_t<R, 0>(v, on); break;
      case 1: cnot_t<R, 1>(v, on); break;
      case 2: cnot_t<R, 2>(v, on); break;
      default: cnot_t<R, 3>(v, on); break;
    }
  }
}

// Sign flips: xor of the IEEE sign bit with `sgn` (0 or 0x80000000).
__device__ __forceinline__ float flip(float x, uint32_t sgn) {
  return __uint_as_float(__float_as_uint(x) ^ sgn);
}
__device__ __forceinline__ double flip(double x, uint32_t sgn) {
  return __longlong_as_double(__double_as_longlong(x) ^ ((unsigned long long)sgn << 32));
}

// Tile-local index of a thread's register-0 amplitude in a stage: the thread
// id with a zero bit inserted at each of the 4 register positions.
__device__ __forceinline__ uint32_t stage_local_index(uint32_t t, cptr<int32_t> S) {
  uint32_t x = t;
#pragma unroll
  for (int r = 0; r < kRegBits; ++r) {
    const uint32_t low = (1u << S[kStRegPos + r]) - 1u;
    x = ((x & ~low) << 1) | (x & low);
  }
  return x;
}

// The same with the register positions as template arguments (ascending).
template <int R0, int R1, int R2, int R3>
__device__ __forceinline__ uint32_t stage_local_index_c(uint32_t t) {
  uint32_t x = t;
  x = ((x & ~((1u << R0) - 1u)) << 1) | (x & ((1u << R0) - 1u));
  x = ((x & ~((1u << R1) - 1u)) << 1) | (x & ((1u << R1) - 1u));
  x = ((x & ~((1u << R2) - 1u)) << 1) | (x & ((1u << R2) - 1u));
  x = ((x & ~((1u << R3) - 1u)) << 1) | (x & ((1u << R3) - 1u));
  return x;
}

// Diagonal op (a run of CZ gates): sign (-1)^Q(x) with x = gt | W_j.  The
// per-thread part Q(gt) is the same for all 16 registers, so it commutes with
// every op of the stage: it is accumulated in `tsg` and applied once when the
// stage ends.  The part linear in the register bits flips the registers with
// bit b set when parity(gt & C_b) = 1; the part depending only on j is a
// uniform mask.
template <typename R, int NS>
__device__ __forceinline__ void diag_apply(Cx<R> (*const *vs)[kRegs], cptr<int32_t> rec,
                                           uint32_t gt, uint32_t &tsg) {
  const int ng = rec[0];
  for (int g = 0; g < ng; ++g)
    tsg += __popc(gt & (gt >> rec[1 + 2 * g]) & (uint32_t)rec[2 + 2 * g]);
  const cptr<int32_t> L = rec + 1 + 2 * ng;
#pragma unroll
  for (int b = 0; b < kRegBits; ++b) {
    const uint32_t Cb = (uint32_t)L[b];
    if (Cb) {
      const uint32_t sgn = (__popc(gt & Cb) & 1u) << 31;
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int j = 0; j < kRegs; ++j)
          if (j & (1 << b)) {
            Cx<R> &z = (*vs[s])[j];
            z = Cx<R>{flip(z.x, sgn), flip(z.y, sgn)};
          }
    }
  }
  const uint32_t qm = (uint32_t)L[kRegBits];
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if ((qm >> j) & 1u)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        Cx<R> &z = (*vs[s])[j];
        z = Cx<R>{-z.x, -z.y};
      }
}

template <typename R, int NS>
__device__ __forceinline__ void apply_thread_sign(Cx<R> (*const *vs)[kRegs], uint32_t tsg) {
  const uint32_t sgn = (tsg & 1u) << 31;
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
      Cx<R> &z = (*vs[s])[j];
      z = Cx<R>{flip(z.x, sgn), flip(z.y, sgn)};
    }
}

// Transition-matrix components for register bit P over the thread's pairs:
// tx = Im Tr(X T), ty = Im Tr(Y T), tz = Im Tr(Z T), T[a][b] = sum psi_b conj(lam_a).
template <typename R, int P>
__device__ __forceinline__ void tcomp_bit(const Cx<R> (&v)[kRegs], const Cx<R> (&l)[kRegs],
                                          R &tx, R &ty, R &tz) {
#pragma unroll
  for (int j = 0; j < kRegs; ++j)
    if (!(j & (1 << P))) {
      const Cx<R> p0 = v[j], p1 = v[j | (1 << P)], l0 = l[j], l1 = l[j | (1 << P)];
      tpair(p0, p1, l0, l1, tx, ty, tz);
    }
}
template <typename R>
__device__ __forceinline__ void tcomp(const Cx<R> (&v)[kRegs], const Cx<R> (&l)[kRegs], int p,
                                      R &tx, R &ty, R &tz) {
  switch (p) {
    case 0: tcomp_bit<R, 0>(v, l, tx, ty, tz); break;
    case 1: tcomp_bit<R, 1>(v, l, tx, ty, tz); break;
    case 2: tcomp_bit<R, 2>(v, l, tx, ty, tz); break;
    default: tcomp_bit<R, 3>(v, l, tx, ty, tz); break;
  }
}

// Streaming (non-temporal) access to one complex64 amplitude of the state
// arrays, which are read and written once per sweep.
__device__ __forceinline__ Cx<float> ld_nt(const Cx<float> *p) {
  const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
  return __builtin_bit_cast(Cx<float>, u);
}
__device__ __forceinline__ void st_nt(Cx<float> *p, Cx<float> v) {
  __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), reinterpret_cast<unsigned long long *>(p));
}

// Arguments of one forward sweep (one circuit, samples along blockIdx.y).
struct FwdArgs {
  const int32_t *prog;
  const int32_t *thr;
  int sweep_off;
  int n;
  void *state;
  const void *mats;
  int n_blocks;
  int ntiles;
  int first, last, store;
  const uint64_t *masks;
  int M;
  const float *obs_sgn;  // [(M+1)][16]
  double *part_obs;      // [B][gridDim.x][M+1]
  double *out;           // [B][M] <Z_m>, written directly by a specialised last
                         // sweep when one tile holds a whole sample
  // periodic renormalisation (NULL: off for this sweep): the previous
  // sweep's end-norm partials [B][rn_prev_n], whose sum rescales this
  // sweep's loads to norm 1; this sweep's own partials [B][gridDim.x]
  const double *rn_prev = nullptr;
  int rn_prev_n = 0;
  double *rn_out = nullptr;
  // specialised first forward sweep with one workgroup per sample and a
  // thread per fused block: the kernel prepares its sample's gate matrices
  // itself (as k_fused_prep does) and writes them to mats_out, and the
  // derivative coefficients to coef[B][n_occ][3] when coef is not NULL
  const int32_t *blk = nullptr, *blk_off = nullptr;
  const double *x = nullptr, *w = nullptr;
  int n_in = 0, n_occ = 0;
  void *mats_out = nullptr;
  double *coef = nullptr;
};


// Arguments of one backward sweep.
struct BwdArgs {
  const int32_t *prog;
  const int32_t *thr;
  int sweep_off;
  int n;
  void *psi;
  void *lam;
  const void *mats;
  int n_blocks;
  int ntiles;
  int first, store;
  const uint64_t *masks;
  int M;
  const double *G;         // [B][M]
  const double *seed_sgn;  // [M][16]
  int seed_add;            // first sweep: lam holds a bra term to add to D psi
  double *part_grad;       // [B][n_gslots][gridDim.x][3]
  int n_gslots;
  double *part_norm;       // [B][gridDim.x]
  // periodic renormalisation (rn_rec NULL: off): per sweep i, sample b and
  // workgroup the partial norms of psi at load, psi at the end, lambda at
  // load and lambda at the end, [S][B][rn_rows][4]; sweep rn_i rescales psi
  // and lambda at load when rn_i is a positive multiple of rn_period, by the
  // square roots of the products of their load / end ratios over the
  // rn_period sweeps before it (each sweep's drift undone)
  double *rn_rec = nullptr;
  int rn_i = 0, rn_period = 0, rn_rows = 0;
  // first sweep: psi is read from here instead of from psi (NULL: from psi);
  // the sweep still writes psi (one state buffer read, another written)
  const void *psi_in = nullptr;
  // specialised backward of a one-sweep plan over single-tile samples: the
  // per-rotation gradients gocc[B][n_occ] from the derivative coefficients
  // coef[B][n_occ][3] (see k_fused_grad_slot)
  const double *coef = nullptr;
  double *gocc = nullptr;
  int n_occ = 0;
};

// Sum over a workgroup of NT threads (a power of two) in FP64, in a fixed
// order (wave sums, then the waves in order); every thread gets it.  sh: NW
// doubles of LDS.  Contains barriers: every thread of the workgroup calls it.
template <int NT>
__device__ __forceinline__ double wg_sum_d(double v, double *sh) {
  constexpr int NW = (NT + 63) / 64, WS = NT < 64 ? NT : 64;
  v = wave_sum_w<WS>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < NW; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// Load / end norm ratios of psi and lambda in backward sweep j (see
// BwdArgs), its norms summed over the `rows` workgroup partials of sample b,
// multiplied into rp and rl.  sh: NW doubles of LDS; every thread calls it.
template <int NT>
__device__ __forceinline__ void rn_bwd_ratio(const double *__restrict__ rec, int j, int rows, int row_stride,
                                             int B, int b, double *sh, double &rp, double &rl) {
  const double *r = rec + ((int64_t)j * B + b) * row_stride * 4;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < rows; k += NT)
    for (int c = 0; c < 4; ++c) q[c] += r[4 * k + c];
  for (int c = 0; c < 4; ++c) q[c] = wg_sum_d<NT>(q[c], sh);
  // (a state that is exactly 0, e.g. lambda for G = 0, keeps its scale)
  rp *= q[1] > 0.0 ? q[0] / q[1] : 1.0;
  rl *= q[3] > 0.0 ? q[2] / q[3] : 1.0;
}

// Scales of a backward sweep that renormalises (see BwdArgs): psi and
// lambda each by sqrt(prod over the previous `period` sweeps of load / end
// norm), the norms summed over `rows` workgroup partials of sample b.
// Every thread gets them; sh: NW doubles of LDS.
template <int NT>
__device__ __forceinline__ void rn_bwd_scales(const double *__restrict__ rec, int i, int period, int rows,
                                              int B, int b, double *sh, double &sp, double &sl) {
  double rp = 1.0, rl = 1.0;
  for (int j = i - period; j < i; ++j) rn_bwd_ratio<NT>(rec, j, rows, rows, B, b, sh, rp, rl);
  sp = sqrt(rp);
  sl = sqrt(rl);
}

}  // namespace qtm
