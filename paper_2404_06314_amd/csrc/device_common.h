// Device helpers shared by the HIP kernels of libqtm.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif
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

namespace qtm {

// Read-only tables that all lanes of a wave read at the same address (sweep
// program, gate matrices, sign tables) are addressed through the constant
// address space, so the compiler issues scalar loads instead of vector loads
// that would wait behind the kernel's own state traffic.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)(uintptr_t)p;
}

template <typename A, typename B>
struct same_type {
  static constexpr bool value = false;
};
template <typename A>
struct same_type<A, A> {
  static constexpr bool value = true;
};

template <typename R>
struct Cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) {
  return {a.x + b.x, a.y + b.y};
}

// 2x2 complex matrix, row-major: m00, m01, m10, m11.
template <typename R>
struct M2 {
  Cx<R> a, b, c, d;
};

template <typename R>
__device__ __forceinline__ M2<R> load_m2(cptr<M2<R>> p) {
  const cptr<R> f = reinterpret_cast<cptr<R>>(p);
  return M2<R>{{f[0], f[1]}, {f[2], f[3]}, {f[4], f[5]}, {f[6], f[7]}};
}

// out0 = a v0 + b v1 ; out1 = c v0 + d v1
template <typename R>
__device__ __forceinline__ void apply_m2(const M2<R> &m, Cx<R> &v0, Cx<R> &v1) {
  Cx<R> o0, o1;
  o0.x = m.a.x * v0.x - m.a.y * v0.y + m.b.x * v1.x - m.b.y * v1.y;
  o0.y = m.a.x * v0.y + m.a.y * v0.x + m.b.x * v1.y + m.b.y * v1.x;
  o1.x = m.c.x * v0.x - m.c.y * v0.y + m.d.x * v1.x - m.d.y * v1.y;
  o1.y = m.c.x * v0.y + m.c.y * v0.x + m.d.x * v1.y + m.d.y * v1.x;
  v0 = o0;
  v1 = o1;
}

// Conjugate transpose applied: out0 = conj(a) v0 + conj(c) v1 ; out1 = conj(b) v0 + conj(d) v1
template <typename R>
__device__ __forceinline__ void apply_m2_adj(const M2<R> &m, Cx<R> &v0, Cx<R> &v1) {
  Cx<R> o0, o1;
  o0.x = m.a.x * v0.x + m.a.y * v0.y + m.c.x * v1.x + m.c.y * v1.y;
  o0.y = m.a.x * v0.y - m.a.y * v0.x + m.c.x * v1.y - m.c.y * v1.x;
  o1.x = m.b.x * v0.x + m.b.y * v0.y + m.d.x * v1.x + m.d.y * v1.y;
  o1.y = m.b.x * v0.y - m.b.y * v0.x + m.d.x * v1.y - m.d.y * v1.x;
  v0 = o0;
  v1 = o1;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a workgroup whose size is a multiple of 64 (every thread gets the
// same value; fixed order, so results are reproducible bit for bit).  sh
// holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r += sh[w];
  return r;
}

// Sum over the first W lanes of a wave (W = power of two <= 64); every lane
// of those W must be active.
template <int W, typename T>
__device__ __forceinline__ T wave_sum_w(T v) {
#pragma unroll
  for (int o = W / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// One DPP reduction step: x + x[lane permuted by CTRL] (rows outside ROW_MASK add 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  int o = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, 0xf, false);
  return x + __builtin_bit_cast(float, o);
}

// Sum of a float over each row of 16 lanes with DPP (every lane of the row
// ends up holding its row's sum).  Every lane must be active.
__device__ __forceinline__ float dpp_sum_row(float v) {
  v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  return v;
}

// Sum of a float over all 64 lanes with DPP row operations (no LDS traffic);
// the total ends up in lane 63.  Every lane must be active.
__device__ __forceinline__ float dpp_sum_to_lane63(float v) {
  v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror: every lane of a row holds the row sum
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// A double from another lane of the same row of 16, by a DPP pattern that
// is valid for every lane (quad_perm, row_ror, row_mirror): both 32-bit
// halves move with the same pattern.
template <int CTRL>
__device__ __forceinline__ double dpp_perm_d(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// FP64 sum of a per-thread value over the 64 lanes of a wave (every lane
// gets it): DPP steps within rows of 16, lane shuffles across rows.
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_perm_d<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_perm_d<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_perm_d<0x124>(v);  // row_ror:4
  v += dpp_perm_d<0x128>(v);  // row_ror:8
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Exchange of 64-bit values between halves (32) or rows (16) of a wave with
// the gfx950 lane swaps, applied to both 32-bit words: swap32 trades lanes
// 32-63 of x for lanes 0-31 of y; swap16 trades the odd rows (16 lanes) of x
// for the even rows of y.
__device__ __forceinline__ void swap32_d(double &x, double &y) {
  const unsigned long long ux = __builtin_bit_cast(unsigned long long, x);
  const unsigned long long uy = __builtin_bit_cast(unsigned long long, y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ux, (unsigned)uy, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ux >> 32), (unsigned)(uy >> 32), false, false);
  x = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
  y = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void swap16_d(double &x, double &y) {
  const unsigned long long ux = __builtin_bit_cast(unsigned long long, x);
  const unsigned long long uy = __builtin_bit_cast(unsigned long long, y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ux, (unsigned)uy, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ux >> 32), (unsigned)(uy >> 32), false, false);
  x = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
  y = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}

// FP64 sums of four per-thread values a, b, c, d over the 64 lanes of a
// wave.  The two swap steps transpose while they reduce (each lane adds
// pairs of halves, then of rows, of different values), so one row reduction
// finishes all four: on return every lane of row 0 (lanes 0-15) holds the
// sum of a, row 1 the sum of c, row 2 the sum of b, row 3 the sum of d.
__device__ __forceinline__ double wave_sum4_d(double a, double b, double c, double d) {
  // rows of 16 lanes written [r0, r1, r2, r3]; A0 = a(r0) + a(r2), A1 =
  // a(r1) + a(r3), likewise B, C, D
  swap32_d(a, b);                 // a: [a(r0), a(r1), b(r0), b(r1)], b: [a(r2), a(r3), b(r2), b(r3)]
  swap32_d(c, d);                 // c: [c(r0), c(r1), d(r0), d(r1)], d: [c(r2), c(r3), d(r2), d(r3)]
  double ab = a + b, cd = c + d;  // ab: [A0, A1, B0, B1], cd: [C0, C1, D0, D1]
  swap16_d(ab, cd);               // ab: [A0, C0, B0, D0], cd: [A1, C1, B1, D1]
  double r = ab + cd;             // [a, c, b, d] summed over the rows, per lane of a row
  r += dpp_perm_d<0xb1>(r);       // quad_perm [1,0,3,2]
  r += dpp_perm_d<0x4e>(r);       // quad_perm [2,3,0,1]
  r += dpp_perm_d<0x124>(r);      // row_ror:4
  r += dpp_perm_d<0x128>(r);      // row_ror:8
  return r;
}
// Which of wave_sum4_d's values (0 = a, 1 = b, 2 = c, 3 = d) the lanes of
// row (lane >> 4) hold.
__device__ __forceinline__ int wave_sum4_comp(unsigned lane) {
  const unsigned row = lane >> 4;
  return row == 0u ? 0 : row == 1u ? 2 : row == 2u ? 1 : 3;
}
// Three values: rows 0-2 hold the sums of a, c, b (row 3: zero).
__device__ __forceinline__ double wave_sum3_d(double a, double b, double c) {
  return wave_sum4_d(a, b, c, 0.0);
}
__device__ __forceinline__ int wave_sum3_comp(unsigned lane) { return wave_sum4_comp(lane); }

__device__ __forceinline__ int parity_u64(uint64_t v) { return __popcll(v) & 1; }

// Matrix of a fixed one-qubit gate (type 5 H, 6 X, 7 Y, 8 Z, 9 S, 10 S^dag,
// 11 T, 12 T^dag, 13 SX), row-major re[4] / im[4] in FP64.
__device__ __forceinline__ void fixed_gate(int type, double (&re)[4], double (&im)[4]) {
  const double r = 0.70710678118654752440;  // 1 / sqrt 2
  for (int k = 0; k < 4; ++k) re[k] = im[k] = 0.0;
  re[0] = re[3] = 1.0;
  switch (type) {
    case 5: re[0] = re[1] = re[2] = r; re[3] = -r; break;
    case 6: re[0] = re[3] = 0.0; re[1] = re[2] = 1.0; break;
    case 7: re[0] = re[3] = 0.0; im[1] = -1.0; im[2] = 1.0; break;
    case 8: re[3] = -1.0; break;
    case 9: re[3] = 0.0; im[3] = 1.0; break;
    case 10: re[3] = 0.0; im[3] = -1.0; break;
    case 11: re[3] = r; im[3] = r; break;
    case 12: re[3] = r; im[3] = -r; break;
    default:  // SX
      re[0] = re[1] = re[2] = re[3] = 0.5;
      im[0] = im[3] = 0.5;
      im[1] = im[2] = -0.5;
  }
}
__device__ __forceinline__ int parity_u32(uint32_t v) { return __popc(v) & 1; }

}  // namespace qtm
