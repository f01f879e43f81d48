// Plain per-gate path: one launch per gate over all (sample, pair) indices.
//
// This is the unfused form of the method (Sec. II-A: evolve once, read all
// observables; reverse gradient by un-applying gates on the ket and the
// combined bra).  It runs in complex64 or complex128 and serves as the plain
// per-sample GPU form shown beside the fused path, and as the path for
// circuits too small for a register tile.
#include "kernels.h"


namespace qtm {

constexpr int kThreads = 256;

// (cos(t/2), sin(t/2)) in FP64 for every (sample, rotation occurrence); the
// angle is an input, a weight, or a weight-scaled input (Eq. (7)).
__global__ void k_half_angles(int B, int n_occ, const int32_t *__restrict__ occ_src,
                              const int32_t *__restrict__ occ_idx, const int32_t *__restrict__ occ_widx,
                              const double *__restrict__ x, int n_in, const double *__restrict__ w,
                              double2 *__restrict__ cs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * n_occ) return;
  int b = (int)(i / n_occ), k = (int)(i % n_occ);
  const int src = occ_src[k];
  double t = src == 2 ? w[occ_idx[k]] : x[(int64_t)b * n_in + occ_idx[k]];
  if (src == 3) t = w[occ_widx[k]] * t;
  double s, c;
  sincos(0.5 * t, &s, &c);
  cs[i] = make_double2(c, s);
}

template <typename R>
__device__ __forceinline__ M2<R> rot_m2(int type, double2 csd, bool adjoint) {
  R c = (R)csd.x, s = (R)(adjoint ? -csd.y : csd.y);
  M2<R> m;
  if (type == 0) {  // RX
    m.a = {c, 0};
    m.b = {0, -s};
    m.c = {0, -s};
    m.d = {c, 0};
  } else if (type == 1) {  // RY
    m.a = {c, 0};
    m.b = {-s, 0};
    m.c = {s, 0};
    m.d = {c, 0};
  } else {  // RZ
    m.a = {c, -s};
    m.b = {0, 0};
    m.c = {0, 0};
    m.d = {c, s};
  }
  return m;
}

template <typename R>
__global__ void k_plain_init(Cx<R> *__restrict__ st, int64_t total, int64_t dim) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  st[i] = Cx<R>{(i % dim) == 0 ? (R)1 : (R)0, (R)0};
}

template <typename R>
__device__ __forceinline__ M2<R> fixed_m2(int type, bool adjoint) {
  double re[4], im[4];
  fixed_gate(type, re, im);
  M2<R> m;
  if (adjoint) {
    m.a = {(R)re[0], (R)-im[0]};
    m.b = {(R)re[2], (R)-im[2]};
    m.c = {(R)re[1], (R)-im[1]};
    m.d = {(R)re[3], (R)-im[3]};
  } else {
    m.a = {(R)re[0], (R)im[0]};
    m.b = {(R)re[1], (R)im[1]};
    m.c = {(R)re[2], (R)im[2]};
    m.d = {(R)re[3], (R)im[3]};
  }
  return m;
}

// One-qubit gate on q for every (sample, pair): a rotation (type 0-2, angle
// of occurrence occ) or a fixed gate (type 5-13); with ctl >= 0 only on the
// pairs whose bit ctl is 1 (a controlled rotation).
template <typename R>
__global__ void k_plain_1q(Cx<R> *__restrict__ a, Cx<R> *__restrict__ a2, int B, int n, int q,
                           int type, int occ, const double2 *__restrict__ cs, int n_occ,
                           int adjoint, int ctl) {
  const int64_t half = (int64_t)1 << (n - 1);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * half) return;
  int b = (int)(i / half);
  int64_t p = i % half;
  int64_t lo = p & (((int64_t)1 << q) - 1);
  int64_t x0 = ((p >> q) << (q + 1)) | lo, x1 = x0 | ((int64_t)1 << q);
  if (ctl >= 0 && !((x0 >> ctl) & 1)) return;
  M2<R> m = type <= 2 ? rot_m2<R>(type, cs[(int64_t)b * n_occ + occ], adjoint != 0)
                      : fixed_m2<R>(type, adjoint != 0);
  int64_t base = (int64_t)b << n;
  Cx<R> v0 = a[base + x0], v1 = a[base + x1];
  apply_m2(m, v0, v1);
  a[base + x0] = v0;
  a[base + x1] = v1;
  if (a2) {
    v0 = a2[base + x0];
    v1 = a2[base + x1];
    apply_m2(m, v0, v1);
    a2[base + x0] = v0;
    a2[base + x1] = v1;
  }
}

template <typename R>
__global__ void k_plain_cnot(Cx<R> *__restrict__ a, Cx<R> *__restrict__ a2, int B, int n, int ctl,
                             int tgt) {
  const int64_t half = (int64_t)1 << (n - 1);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * half) return;
  int b = (int)(i / half);
  int64_t p = i % half;
  int64_t lo = p & (((int64_t)1 << tgt) - 1);
  int64_t x0 = ((p >> tgt) << (tgt + 1)) | lo, x1 = x0 | ((int64_t)1 << tgt);
  if (!((x0 >> ctl) & 1)) return;
  int64_t base = (int64_t)b << n;
  Cx<R> t = a[base + x0];
  a[base + x0] = a[base + x1];
  a[base + x1] = t;
  if (a2) {
    t = a2[base + x0];
    a2[base + x0] = a2[base + x1];
    a2[base + x1] = t;
  }
}

template <typename R>
__global__ void k_plain_cz(Cx<R> *__restrict__ a, Cx<R> *__restrict__ a2, int B, int n, int q0,
                           int q1) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dim = (int64_t)1 << n;
  if (i >= (int64_t)B * dim) return;
  int64_t x = i & (dim - 1);
  if (((x >> q0) & 1) && ((x >> q1) & 1)) {
    a[i] = Cx<R>{-a[i].x, -a[i].y};
    if (a2) a2[i] = Cx<R>{-a2[i].x, -a2[i].y};
  }
}

// Expectation values: per (sample, block) FP64 partial sums of
// (-1)^popcount(x & S_m) |psi_x|^2 for m < M, and the norm at m = M.
template <typename R>
__global__ void __launch_bounds__(kThreads)
    k_plain_expval(const Cx<R> *__restrict__ st, int n, const uint64_t *__restrict__ masks, int M,
                   double *__restrict__ part, int nblk) {
  __shared__ double red[kThreads / 64];
  const int b = blockIdx.y;
  const int64_t dim = (int64_t)1 << n;
  const Cx<R> *s = st + (int64_t)b * dim;
  for (int m = 0; m <= M; ++m) {
    const uint64_t mask = m < M ? masks[m] : 0;
    double acc = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < dim;
         x += (int64_t)nblk * kThreads) {
      double p = (double)s[x].x * s[x].x + (double)s[x].y * s[x].y;
      acc += parity_u64((uint64_t)x & mask) ? -p : p;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int wv = 0; wv < kThreads / 64; ++wv) t += red[wv];
      part[((int64_t)b * nblk + blockIdx.x) * (M + 1) + m] = t;
    }
    __syncthreads();
  }
}

// <Z_m> of sample b: sum over the partial rows of column m, divided by the
// sum of column M (the norm).  One workgroup per (m, b), fixed-order sums.
__global__ void __launch_bounds__(256) k_obs_final(const double *__restrict__ part, int nblk, int M,
                                                   double *__restrict__ out, int normalise) {
  __shared__ double sh[4];
  const int m = blockIdx.x, b = blockIdx.y;
  const double *p = part + (int64_t)b * nblk * (M + 1);
  double acc = 0.0, nrm = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    acc += p[(int64_t)k * (M + 1) + m];
    nrm += p[(int64_t)k * (M + 1) + M];
  }
  acc = block_sum(acc, sh);
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) out[(int64_t)b * M + m] = normalise ? acc / nrm : acc;
}

// lambda = D psi with D(x) = sum_m G[b][m] (-1)^popcount(x & S_m), D in FP64.
template <typename R>
__global__ void k_plain_seed(const Cx<R> *__restrict__ psi, Cx<R> *__restrict__ lam, int B, int n,
                             const uint64_t *__restrict__ masks, int M,
                             const double *__restrict__ G) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dim = (int64_t)1 << n;
  if (i >= (int64_t)B * dim) return;
  int b = (int)(i >> n);
  uint64_t x = (uint64_t)(i & (dim - 1));
  double d = 0.0;
  for (int m = 0; m < M; ++m) {
    double g = G[(int64_t)b * M + m];
    d += parity_u64(x & masks[m]) ? -g : g;
  }
  lam[i] = Cx<R>{(R)(d * (double)psi[i].x), (R)(d * (double)psi[i].y)};
}

// g = Im <lambda| P_q |psi> for P = X, Y, Z (type 0, 1, 2), per-block FP64
// partials; with ctl >= 0 the generator is |1><1|_ctl (x) P_q (a controlled
// rotation), so only pairs whose bit ctl is 1 contribute.
template <typename R>
__global__ void __launch_bounds__(kThreads)
    k_plain_grad(const Cx<R> *__restrict__ psi, const Cx<R> *__restrict__ lam, int n, int q,
                 int type, int occ, int n_occ, double *__restrict__ part, int nblk, int ctl) {
  __shared__ double red[kThreads / 64];
  const int b = blockIdx.y;
  const int64_t half = (int64_t)1 << (n - 1);
  const int64_t base = (int64_t)b << n;
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < half;
       p += (int64_t)nblk * kThreads) {
    int64_t lo = p & (((int64_t)1 << q) - 1);
    int64_t x0 = ((p >> q) << (q + 1)) | lo, x1 = x0 | ((int64_t)1 << q);
    if (ctl >= 0 && !((x0 >> ctl) & 1)) continue;
    double p0r = psi[base + x0].x, p0i = psi[base + x0].y;
    double p1r = psi[base + x1].x, p1i = psi[base + x1].y;
    double l0r = lam[base + x0].x, l0i = lam[base + x0].y;
    double l1r = lam[base + x1].x, l1i = lam[base + x1].y;
    // Im(conj(l) * v) = l.r * v.i - l.i * v.r
    if (type == 0) {  // X psi = (psi1, psi0)
      acc += l0r * p1i - l0i * p1r + l1r * p0i - l1i * p0r;
    } else if (type == 1) {  // Y psi = (-i psi1, i psi0)
      // -i psi1 = (p1i, -p1r); i psi0 = (-p0i, p0r)
      acc += l0r * (-p1r) - l0i * p1i + l1r * p0r - l1i * (-p0i);
    } else {  // Z psi = (psi0, -psi1)
      acc += (l0r * p0i - l0i * p0r) - (l1r * p1i - l1i * p1r);
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int wv = 0; wv < kThreads / 64; ++wv) t += red[wv];
    part[((int64_t)b * n_occ + occ) * nblk + blockIdx.x] = t;
  }
}

__global__ void k_plain_grad_final(const double *__restrict__ part, int B, int n_occ, int nblk,
                                   double *__restrict__ gocc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * n_occ) return;
  double acc = 0.0;
  for (int k = 0; k < nblk; ++k) acc += part[i * nblk + k];
  gocc[i] = acc;
}

// Scatter per-occurrence angle derivatives into parameter slots (fixed
// order), with the chain-rule factor of a scaled angle w[j] * x[b][i]:
// grad_w[j] = sum_b sum_{k in occ(w_j)} gocc[b][k] * (x[b][fac_k] or 1);
// grad_x[b][i] = sum_{k in occ(x_i)} gocc[b][k] * (w[fac_k] or 1).
// One launch: blocks [0, n_w) one per weight (samples over the threads,
// fixed-order block sum), the blocks after them one thread per (sample,
// input).
__global__ void __launch_bounds__(256) k_scatter(const double *__restrict__ gocc, int B, int n_occ, int n_w,
                                                 const int32_t *__restrict__ w_ptr,
                                                 const int32_t *__restrict__ w_list,
                                                 const int32_t *__restrict__ w_fac,
                                                 const int32_t *__restrict__ x_ptr,
                                                 const int32_t *__restrict__ x_list,
                                                 const int32_t *__restrict__ x_fac, const double *__restrict__ x,
                                                 const double *__restrict__ w, int n_in, double *__restrict__ gw,
                                                 double *__restrict__ gx) {
  if ((int)blockIdx.x < n_w) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < B; b += blockDim.x)
      for (int e = w_ptr[j]; e < w_ptr[j + 1]; ++e) {
        const int f = w_fac[e];
        const double g = gocc[(int64_t)b * n_occ + w_list[e]];
        acc += f < 0 ? g : g * x[(int64_t)b * n_in + f];
      }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) gw[j] = acc;
    return;
  }
  const int64_t i = (int64_t)(blockIdx.x - n_w) * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * n_in) return;
  const int b = (int)(i / n_in), k = (int)(i % n_in);
  double acc = 0.0;
  for (int e = x_ptr[k]; e < x_ptr[k + 1]; ++e) {
    const int f = x_fac[e];
    const double g = gocc[(int64_t)b * n_occ + x_list[e]];
    acc += f < 0 ? g : g * w[f];
  }
  gx[i] = acc;
}

// Upstream gradients of a Jacobian pass over `rows` = k x B rows: row r
// (sample r mod B) selects observable m0 + r / B.
__global__ void k_onehot(double *__restrict__ G, int rows, int B, int M, int m0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)rows * M) G[i] = (int)(i % M) == m0 + (int)(i / M) / B ? 1.0 : 0.0;
}

// `copies` back-to-back copies of n 8-byte words (a batch of states or of
// input rows, repeated for the rows of a Jacobian pass).
__global__ void k_replicate(uint64_t *__restrict__ dst, const uint64_t *__restrict__ src, int64_t n,
                            int copies) {
  const int64_t total = n * copies, step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) dst[i] = src[i % n];
}

// Rows of the Jacobian from a pass over `rows` = k x B rows (row r: sample
// b = r mod B, observable m = m0 + r / B): per sample, every weight and input
// slot sums its rotation occurrences (no sum over the batch).
__global__ void k_scatter_jac(const double *__restrict__ gocc, int rows, int B, int n_occ,
                              const int32_t *__restrict__ w_ptr, const int32_t *__restrict__ w_list,
                              const int32_t *__restrict__ w_fac, int n_w,
                              const int32_t *__restrict__ x_ptr, const int32_t *__restrict__ x_list,
                              const int32_t *__restrict__ x_fac, int n_in,
                              const double *__restrict__ x, const double *__restrict__ w, int m0,
                              int M, double *__restrict__ jw, double *__restrict__ jx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = n_w + (jx ? n_in : 0);
  if (i >= (int64_t)rows * per) return;
  const int r = (int)(i / per), j = (int)(i % per);
  const int b = r % B, m = m0 + r / B;
  const double *g = gocc + (int64_t)r * n_occ;
  double acc = 0.0;
  if (j < n_w) {
    for (int e = w_ptr[j]; e < w_ptr[j + 1]; ++e) {
      const int f = w_fac[e];
      acc += f < 0 ? g[w_list[e]] : g[w_list[e]] * x[(int64_t)b * n_in + f];
    }
    jw[((int64_t)b * M + m) * n_w + j] = acc;
  } else {
    const int k = j - n_w;
    for (int e = x_ptr[k]; e < x_ptr[k + 1]; ++e) {
      const int f = x_fac[e];
      acc += f < 0 ? g[x_list[e]] : g[x_list[e]] * w[f];
    }
    jx[((int64_t)b * M + m) * n_in + k] = acc;
  }
}

// ---------------------------------------------------------------------------
// Pauli strings with X or Y factors (Sec. II-A: any observable).  For the
// string (xm, zm), P|y> = i^nY (-1)^popcount(y & zm) |y ^ xm> with nY the
// number of Y factors, so <P> = i^nY sum_x conj(psi_x) s(x ^ xm) psi_(x ^ xm),
// s(v) = (-1)^popcount(v & zm).  With p the lowest qubit of xm, the pair
// (x, y = x ^ xm), bit p of x clear, contributes i^nY [a s(y) + conj(a) s(x)]
// for a = conj(psi_x) psi_y; s(x) s(y) = (-1)^nY, so this is
// (-1)^(nY/2) s(x) 2 Re a for even nY and (-1)^((nY+1)/2) s(y) 2 Im a for odd.

__device__ __forceinline__ uint64_t insert_zero_bit(uint64_t i, int p) {
  const uint64_t lo = i & ((1ull << p) - 1);
  return ((i >> p) << (p + 1)) | lo;
}

// Per (sample, block) FP64 partial sums of every off-diagonal string's pair
// terms, then (column n_nd) of |psi|^2: part[b][block][n_nd + 1].
template <typename R>
__global__ void __launch_bounds__(kThreads)
    k_pauli_partial(const Cx<R> *__restrict__ st, int n, int n_nd, const uint64_t *__restrict__ px,
                    const uint64_t *__restrict__ pz, double *__restrict__ part, int nblk) {
  __shared__ double red[kThreads / 64];
  const int b = blockIdx.y;
  const int64_t half = (int64_t)1 << (n - 1);
  const Cx<R> *s = st + ((int64_t)b << n);
  for (int j = 0; j <= n_nd; ++j) {
    double acc = 0.0;
    if (j < n_nd) {
      const uint64_t xm = px[j], zm = pz[j];
      const int p = __ffsll((unsigned long long)xm) - 1;
      const int ny = __popcll(xm & zm);
      const double sgn = ((ny + 1) >> 1) & 1 ? -1.0 : 1.0;  // (-1)^(nY/2) or (-1)^((nY+1)/2)
      for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < half;
           i += (int64_t)nblk * kThreads) {
        const uint64_t x = insert_zero_bit((uint64_t)i, p), y = x ^ xm;
        const double ax = s[x].x, bx = s[x].y, ay = s[y].x, by = s[y].y;
        if (ny & 1) {
          const double im = ax * by - bx * ay;
          acc += parity_u64(y & zm) ? -sgn * 2.0 * im : sgn * 2.0 * im;
        } else {
          const double re = ax * ay + bx * by;
          acc += parity_u64(x & zm) ? -sgn * 2.0 * re : sgn * 2.0 * re;
        }
      }
    } else {
      for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < half;
           i += (int64_t)nblk * kThreads) {
        const Cx<R> u = s[2 * i], v = s[2 * i + 1];
        acc += (double)u.x * u.x + (double)u.y * u.y + (double)v.x * v.x + (double)v.y * v.y;
      }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int wv = 0; wv < kThreads / 64; ++wv) t += red[wv];
      part[((int64_t)b * nblk + blockIdx.x) * (n_nd + 1) + j] = t;
    }
    __syncthreads();
  }
}

// out[b][idx_j] = (sum of column j) / (sum of column n_nd), fixed order;
// one workgroup per (string, sample).
__global__ void __launch_bounds__(256) k_pauli_final(const double *__restrict__ part, int nblk, int n_nd,
                                                     const int32_t *__restrict__ idx, int M,
                                                     double *__restrict__ out) {
  __shared__ double sh[4];
  const int j = blockIdx.x, b = blockIdx.y;
  const double *p = part + (int64_t)b * nblk * (n_nd + 1);
  double acc = 0.0, nrm = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    acc += p[(int64_t)k * (n_nd + 1) + j];
    nrm += p[(int64_t)k * (n_nd + 1) + n_nd];
  }
  acc = block_sum(acc, sh);
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) out[(int64_t)b * M + idx[j]] = acc / nrm;
}

// Bra term of the off-diagonal strings: sum_j G[b][idx_j] (P_j psi)_x minus
// (sum_j G[b][idx_j]) psi_x, the latter cancelling what the diagonal seed
// adds for their identity masks.  Written to lam, or added to it.
template <typename R>
__global__ void k_pauli_seed(const Cx<R> *__restrict__ psi, Cx<R> *__restrict__ lam, int B, int n,
                             int n_nd, const int32_t *__restrict__ idx, const uint64_t *__restrict__ px,
                             const uint64_t *__restrict__ pz, const double *__restrict__ G, int M,
                             int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ((int64_t)B << n)) return;
  const int b = (int)(i >> n);
  const uint64_t x = (uint64_t)i & ((1ull << n) - 1);
  const Cx<R> *s = psi + ((int64_t)b << n);
  double re = 0.0, im = 0.0, gsum = 0.0;
  for (int j = 0; j < n_nd; ++j) {
    const double g = G[(int64_t)b * M + idx[j]];
    gsum += g;
    const uint64_t y = x ^ px[j];
    double vr = s[y].x, vi = s[y].y;
    if (parity_u64(y & pz[j])) {
      vr = -vr;
      vi = -vi;
    }
    switch (__popcll(px[j] & pz[j]) & 3) {  // times i^nY
      case 0: re += g * vr; im += g * vi; break;
      case 1: re -= g * vi; im += g * vr; break;
      case 2: re -= g * vr; im -= g * vi; break;
      default: re += g * vi; im -= g * vr; break;
    }
  }
  re -= gsum * (double)s[x].x;
  im -= gsum * (double)s[x].y;
  if (accumulate) {
    re += (double)lam[i].x;
    im += (double)lam[i].y;
  }
  lam[i] = Cx<R>{(R)re, (R)im};
}

// ---------------------------------------------------------------------------
// host launchers

static inline unsigned nb(int64_t work) { return (unsigned)((work + kThreads - 1) / kThreads); }

hipError_t launch_half_angles(const DevCircuit &d, int B, const double *x, const double *w,
                              double2 *cs, hipStream_t s) {
  if (d.n_occ == 0) return hipSuccess;
  k_half_angles<<<nb((int64_t)B * d.n_occ), kThreads, 0, s>>>(B, d.n_occ, d.occ_src, d.occ_idx,
                                                              d.occ_widx, x, d.n_inputs, w, cs);
  return hipGetLastError();
}

static int plain_nblk(int B, int64_t work) {
  int64_t want = (2048 + B - 1) / B;
  int64_t cap = (work + kThreads - 1) / kThreads;
  int64_t v = want < cap ? want : cap;
  if (v > 256) v = 256;
  return (int)(v < 1 ? 1 : v);
}

int plain_norm_rows(int n, int B) { return plain_nblk(B, (int64_t)1 << n); }

// Squared norm of every sample's final state from the forward's partial sums
// (column M of part [B][rows][M + 1]); one workgroup per sample, fixed order.
__global__ void __launch_bounds__(256) k_norm_final(const double *__restrict__ part, int rows, int M,
                                                    double *__restrict__ out) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  const double *p = part + (int64_t)b * rows * (M + 1);
  double nrm = 0.0;
  for (int k = threadIdx.x; k < rows; k += blockDim.x) nrm += p[(int64_t)k * (M + 1) + M];
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) out[b] = nrm;
}

hipError_t launch_norms(const double *part, int B, int rows, int M, double *out, hipStream_t s) {
  k_norm_final<<<B, rows >= 256 ? 256u : 64u, 0, s>>>(part, rows, M, out);
  return hipGetLastError();
}

// First non-finite entry of the angle sources: index into inputs (0 ..
// nx - 1) or nx + index into weights; ~0 when every value is finite.
__global__ void k_nonfinite_init(unsigned long long *first) { *first = ~0ull; }
__global__ void k_first_nonfinite(const double *__restrict__ x, int64_t nx, const double *__restrict__ w,
                                  int64_t nw, unsigned long long *__restrict__ first) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nx + nw;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = i < nx ? x[i] : w[i - nx];
    if (!isfinite(v)) atomicMin(first, (unsigned long long)i);
  }
}

hipError_t launch_first_nonfinite(const double *x, int64_t nx, const double *w, int64_t nw,
                                  unsigned long long *first, hipStream_t s) {
  k_nonfinite_init<<<1, 1, 0, s>>>(first);
  const int64_t work = nx + nw;
  if (work > 0) {
    const int64_t blocks = std::min<int64_t>((work + kThreads - 1) / kThreads, 1024);
    k_first_nonfinite<<<(unsigned)blocks, kThreads, 0, s>>>(x, nx, w, nw, first);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t plain_forward(const DevCircuit &d, const HostCircuitInfo &h, int B, const double2 *cs,
                         void *state, double *part, double *out, bool normalise, hipStream_t s) {
  Cx<R> *st = (Cx<R> *)state;
  const int n = d.n;
  const int64_t dim = (int64_t)1 << n;
  k_plain_init<R><<<nb((int64_t)B * dim), kThreads, 0, s>>>(st, (int64_t)B * dim, dim);
  for (size_t k = 0; k < h.gates.size(); ++k) {
    const Gate &g = h.gates[k];
    if (is_rotation(g.type) || is_fixed(g.type))
      k_plain_1q<R><<<nb((int64_t)B * (dim / 2)), kThreads, 0, s>>>(st, nullptr, B, n, g.q0, g.type,
                                                                    h.gate_occ[k], cs, d.n_occ, 0, -1);
    else if (is_crot(g.type))
      k_plain_1q<R><<<nb((int64_t)B * (dim / 2)), kThreads, 0, s>>>(
          st, nullptr, B, n, g.q1, g.type - G_CRX, h.gate_occ[k], cs, d.n_occ, 0, g.q0);
    else if (g.type == G_CNOT)
      k_plain_cnot<R><<<nb((int64_t)B * (dim / 2)), kThreads, 0, s>>>(st, nullptr, B, n, g.q0, g.q1);
    else
      k_plain_cz<R><<<nb((int64_t)B * dim), kThreads, 0, s>>>(st, nullptr, B, n, g.q0, g.q1);
  }
  int nblk = plain_nblk(B, dim);
  k_plain_expval<R><<<dim3(nblk, B), kThreads, 0, s>>>(st, n, d.masks, d.n_obs, part, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_obs_final(part, B, nblk, d.n_obs, out, normalise, s);
}

template <typename R>
hipError_t plain_backward(const DevCircuit &d, const HostCircuitInfo &h, int B, const double2 *cs,
                          const double *x, const double *w, void *state, void *lam_buf,
                          const double *G, double *part, double *gocc, double *gw, double *gx,
                          hipStream_t s) {
  Cx<R> *psi = (Cx<R> *)state, *lam = (Cx<R> *)lam_buf;
  const int n = d.n;
  const int64_t dim = (int64_t)1 << n;
  k_plain_seed<R><<<nb((int64_t)B * dim), kThreads, 0, s>>>(psi, lam, B, n, d.masks, d.n_obs, G);
  hipError_t e0 = launch_pauli_seed<R>(d, B, psi, lam, G, true, s);
  if (e0 != hipSuccess) return e0;
  const int nblk = plain_nblk(B, dim / 2);
  for (int k = (int)h.gates.size() - 1; k >= 0; --k) {
    const Gate &g = h.gates[k];
    if (is_rotation(g.type) || is_crot(g.type)) {
      // a controlled rotation acts on its target q1 where the control q0 is 1
      const bool ctl = is_crot(g.type);
      const int q = ctl ? g.q1 : g.q0, t = ctl ? g.type - G_CRX : g.type, c = ctl ? g.q0 : -1;
      k_plain_grad<R><<<dim3(nblk, B), kThreads, 0, s>>>(psi, lam, n, q, t, h.gate_occ[k], d.n_occ,
                                                         part, nblk, c);
      k_plain_1q<R><<<nb((int64_t)B * (dim / 2)), kThreads, 0, s>>>(psi, lam, B, n, q, t,
                                                                    h.gate_occ[k], cs, d.n_occ, 1, c);
    } else if (is_fixed(g.type)) {
      k_plain_1q<R><<<nb((int64_t)B * (dim / 2)), kThreads, 0, s>>>(psi, lam, B, n, g.q0, g.type, -1,
                                                                    cs, d.n_occ, 1, -1);
    } else if (g.type == G_CNOT) {
      k_plain_cnot<R><<<nb((int64_t)B * (dim / 2)), kThreads, 0, s>>>(psi, lam, B, n, g.q0, g.q1);
    } else {
      k_plain_cz<R><<<nb((int64_t)B * dim), kThreads, 0, s>>>(psi, lam, B, n, g.q0, g.q1);
    }
  }
  if (d.n_occ > 0)
    k_plain_grad_final<<<nb((int64_t)B * d.n_occ), kThreads, 0, s>>>(part, B, d.n_occ, nblk, gocc);
  return launch_scatter(d, B, gocc, x, w, gw, gx, s);
}

static inline unsigned red_threads(int64_t n) { return n >= 256 ? 256u : 64u; }

hipError_t launch_obs_final(const double *part, int B, int nblk, int M, double *out,
                            bool normalise, hipStream_t s) {
  if (B <= 0 || M <= 0) return hipSuccess;
  k_obs_final<<<dim3(M, B), red_threads(nblk), 0, s>>>(part, nblk, M, out, normalise ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_scatter(const DevCircuit &d, int B, const double *gocc, const double *x,
                          const double *w, double *gw, double *gx, hipStream_t s) {
  const unsigned threads = red_threads(B);
  const int n_w = d.n_weights > 0 ? d.n_weights : 0;
  const int64_t nx = gx && d.n_inputs > 0 ? (int64_t)B * d.n_inputs : 0;
  const int64_t blocks = n_w + (nx + threads - 1) / threads;
  if (blocks == 0) return hipSuccess;
  k_scatter<<<(unsigned)blocks, threads, 0, s>>>(gocc, B, d.n_occ, n_w, d.w_ptr, d.w_list, d.w_fac, d.x_ptr,
                                                d.x_list, d.x_fac, x, w, nx ? d.n_inputs : 0, gw, gx);
  return hipGetLastError();
}

hipError_t launch_onehot(double *G, int rows, int B, int M, int m0, hipStream_t s) {
  k_onehot<<<nb((int64_t)rows * M), kThreads, 0, s>>>(G, rows, B, M, m0);
  return hipGetLastError();
}

hipError_t launch_replicate(void *dst, const void *src, size_t bytes, int copies, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / sizeof(uint64_t));
  if (n == 0 || copies <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n * copies + kThreads - 1) / kThreads, 4096);
  k_replicate<<<(int)blocks, kThreads, 0, s>>>((uint64_t *)dst, (const uint64_t *)src, n, copies);
  return hipGetLastError();
}

hipError_t launch_scatter_jac(const DevCircuit &d, int rows, int B, const double *gocc, const double *x,
                              const double *w, int m0, double *jw, double *jx, hipStream_t s) {
  const int64_t work = (int64_t)rows * (d.n_weights + (jx ? d.n_inputs : 0));
  if (work == 0) return hipSuccess;
  k_scatter_jac<<<nb(work), kThreads, 0, s>>>(gocc, rows, B, d.n_occ, d.w_ptr, d.w_list, d.w_fac,
                                              d.n_weights, d.x_ptr, d.x_list, d.x_fac, d.n_inputs, x,
                                              w, m0, d.n_obs, jw, jx);
  return hipGetLastError();
}

static int pauli_nblk(const DevCircuit &d, int B) { return plain_nblk(B, (int64_t)1 << (d.n - 1)); }

size_t pauli_part_doubles(const DevCircuit &d, int B) {
  return (size_t)B * pauli_nblk(d, B) * (d.n_nd + 1);
}

template <typename R>
hipError_t launch_pauli_expval(const DevCircuit &d, int B, const void *state, double *part, double *out,
                               hipStream_t s) {
  if (d.n_nd == 0) return hipSuccess;
  const int nblk = pauli_nblk(d, B);
  k_pauli_partial<R><<<dim3(nblk, B), kThreads, 0, s>>>((const Cx<R> *)state, d.n, d.n_nd, d.nd_x,
                                                       d.nd_z, part, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_pauli_final<<<dim3(d.n_nd, B), red_threads(nblk), 0, s>>>(part, nblk, d.n_nd, d.nd_idx, d.n_obs,
                                                             out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pauli_seed(const DevCircuit &d, int B, const void *psi, void *lam, const double *G,
                             bool accumulate, hipStream_t s) {
  if (d.n_nd == 0) return hipSuccess;
  k_pauli_seed<R><<<nb((int64_t)B << d.n), kThreads, 0, s>>>((const Cx<R> *)psi, (Cx<R> *)lam, B, d.n,
                                                            d.n_nd, d.nd_idx, d.nd_x, d.nd_z, G,
                                                            d.n_obs, accumulate ? 1 : 0);
  return hipGetLastError();
}

template hipError_t launch_pauli_expval<float>(const DevCircuit &, int, const void *, double *, double *,
                                               hipStream_t);
template hipError_t launch_pauli_expval<double>(const DevCircuit &, int, const void *, double *, double *,
                                                hipStream_t);
template hipError_t launch_pauli_seed<float>(const DevCircuit &, int, const void *, void *, const double *,
                                             bool, hipStream_t);
template hipError_t launch_pauli_seed<double>(const DevCircuit &, int, const void *, void *, const double *,
                                              bool, hipStream_t);

size_t plain_part_doubles(const DevCircuit &d, int B) {
  const int64_t dim = (int64_t)1 << d.n;
  size_t a = (size_t)B * plain_nblk(B, dim) * (d.n_obs + 1);
  size_t b = (size_t)B * d.n_occ * plain_nblk(B, dim / 2);
  return a > b ? a : b;
}

template hipError_t plain_forward<float>(const DevCircuit &, const HostCircuitInfo &, int,
                                         const double2 *, void *, double *, double *, bool,
                                         hipStream_t);
template hipError_t plain_forward<double>(const DevCircuit &, const HostCircuitInfo &, int,
                                          const double2 *, void *, double *, double *, bool,
                                          hipStream_t);
template hipError_t plain_backward<float>(const DevCircuit &, const HostCircuitInfo &, int,
                                          const double2 *, const double *, const double *, void *, void *, const double *,
                                          double *, double *, double *, double *, hipStream_t);
template hipError_t plain_backward<double>(const DevCircuit &, const HostCircuitInfo &, int,
                                           const double2 *, const double *, const double *, void *, void *, const double *,
                                           double *, double *, double *, double *, hipStream_t);

}  // namespace qtm
