// Shared-weight dense blocks on the matrix cores (forward only).
//
// In a layer of the layered ansatz (RX(x) encoding on every qubit, then
// RY(w) and RZ(w) on every qubit, then an open CZ chain), the weights are
// the same for every sample of the batch (Sec. II-B, Eq. (6)).  For a block
// of 4 consecutive qubits the weight part
//     W = CZ(in-block pairs) . (RZ RY) x (RZ RY) x (RZ RY) x (RZ RY)
// is one dense 16 x 16 complex unitary shared by the batch, i.e. a 32 x 32
// real operator applied to all B * 2^(n-4) vectors of 16 amplitudes: a
// dense contraction, run here with v_mfma_f32_16x16x4f32.  The per-sample RX
// encoding is applied before it on the VALU, and the CZ gates between
// blocks as signs of the global index.
//
// One pass per (layer, block) over the whole state: a wave takes 16 columns
// (vectors) of one sample.  Lane l holds, for column l % 16 and g = l / 16,
// the block amplitudes g, g + 4, g + 8, g + 12 (register r = amplitude
// 4 r + g): exactly the matrix-core B operand of K-steps 0-3 (real parts)
// and 4-7 (imaginary parts).  The output of M-tile 0 (real parts) and 1
// (imaginary parts) leaves amplitudes 4 g + r in lane l, register r.
//
// The last pass also reads every Pauli-Z string expectation value and the
// norm (FP64 partials per workgroup, reduced by k_obs_final).
#include "k9.h"

#include "sweep_ops.h"

namespace qtm {

typedef float k9f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// prep (FP64, rounded once to FP32)

// W of (layer, block) as the matrix-core A operand table
// tab[(lb * 2 + mt) * 8 + s][lane] = Wr[16 mt + lane % 16][4 s + lane / 16],
// Wr = [[Re W, -Im W], [Im W, Re W]].  One thread per (layer, block).
__global__ void k_k9_prep_w(int n_lb, int nb, const int32_t *__restrict__ ry, const int32_t *__restrict__ rz,
                            const double *__restrict__ w, float *__restrict__ tab) {
  const int lb = blockIdx.x * blockDim.x + threadIdx.x;
  if (lb >= n_lb) return;
  const int layer = lb / nb, blk = lb % nb;
  const int n = nb * 4;
  // per block qubit t: U_t = RZ(wz) RY(wy)
  MD U[4];
  for (int t = 0; t < 4; ++t) {
    const int q = 4 * blk + t;
    U[t] = md_mul(md_rot(2, w[rz[layer * n + q]]), md_rot(1, w[ry[layer * n + q]]));
  }
  float *o = tab + (size_t)lb * 2 * 8 * 64;
  for (int a = 0; a < 16; ++a) {
    // in-block CZ chain: sign (-1)^(a0 a1 + a1 a2 + a2 a3) on output a
    const int cz = ((a & (a >> 1)) & 7);
    const double sg = (__popc(cz) & 1) ? -1.0 : 1.0;
    for (int bcol = 0; bcol < 16; ++bcol) {
      CD e = {sg, 0.0};
      for (int t = 0; t < 4; ++t) e = cd_mul(e, U[t].m[(a >> t) & 1][(bcol >> t) & 1]);
      // Wr rows: a (real output), 16 + a (imaginary output); columns: b (real
      // input), 16 + b (imaginary input)
      const double wr[2][2] = {{e.x, -e.y}, {e.y, e.x}};
      for (int ro = 0; ro < 2; ++ro)
        for (int co = 0; co < 2; ++co) {
          const int row = 16 * ro + a, col = 16 * co + bcol;
          const int mt = row >> 4, s = col >> 2, lane = (row & 15) + 16 * (col & 3);
          o[(mt * 8 + s) * 64 + lane] = (float)wr[ro][co];
        }
    }
  }
}

// (cos, sin) of half the RX angle per (sample, layer, qubit).
__global__ void k_k9_prep_rx(int B, int L, int n, int n_in, const int32_t *__restrict__ rx,
                             const double *__restrict__ x, float2 *__restrict__ cs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * L * n) return;
  const int b = (int)(i / ((int64_t)L * n)), lq = (int)(i % ((int64_t)L * n));
  double s, c;
  sincos(0.5 * x[(int64_t)b * n_in + rx[lq]], &s, &c);
  cs[i] = make_float2((float)c, (float)s);
}

// |0...0> of every sample.
__global__ void k_k9_init(Cx<float> *__restrict__ st, int64_t total, int64_t dim) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) st[i] = Cx<float>{(i & (dim - 1)) == 0 ? 1.f : 0.f, 0.f};
}

// ---------------------------------------------------------------------------
// one pass: layer `layer`, block `blk`

struct K9PassArgs {
  Cx<float> *state;
  const float *tab;   // A operand tables
  const float2 *rx;   // [B][L][n]
  int n, L, layer, blk;
  uint32_t cross_in;  // CZ pairs (q, q + 1) between blocks applied before RX (bit q set), or 0
  uint32_t cross_out; // the same after the dense block (last pass)
  // last pass: observables
  int M;
  const uint64_t *masks;
  double *part;       // [B][rows][M + 1]
};

__device__ __forceinline__ uint32_t k9_sign(uint32_t x, uint32_t pairs) {
  return ((uint32_t)__popc(x & (x >> 1) & pairs) & 1u) << 31;
}

__global__ void __launch_bounds__(256) k_k9_pass(K9PassArgs a) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4;
  const int n = a.n, sh = 4 * a.blk;
  const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + (lane & 15);
  const int b = (int)(col >> (n - 4));
  const uint32_t r = (uint32_t)(col & (((int64_t)1 << (n - 4)) - 1));
  const uint32_t lo = r & ((1u << sh) - 1u), hi = r >> sh;
  const uint32_t base = (hi << (sh + 4)) | lo;  // index within the sample
  Cx<float> *st = a.state + ((int64_t)b << n);
  Cx<float> v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = st[base | ((uint32_t)(4 * k + g) << sh)];
  if (a.cross_in) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t z = k9_sign(base | ((uint32_t)(4 * k + g) << sh), a.cross_in);
      v[k] = Cx<float>{flip(v[k].x, z), flip(v[k].y, z)};
    }
  }
  // RX(x) of the block's qubits: out = c v - i s v_partner
  const float2 *cs = a.rx + ((int64_t)b * a.L + a.layer) * n + sh;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float c = cs[q].x, s = cs[q].y;
    if (q < 2) {
      // block bit q is lane bit 4 + q
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float px = __shfl_xor(v[k].x, 16 << q, 64), py = __shfl_xor(v[k].y, 16 << q, 64);
        v[k] = Cx<float>{c * v[k].x + s * py, c * v[k].y - s * px};
      }
    } else {
      // block bit q is register bit q - 2
      const int m = 1 << (q - 2);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (!(k & m)) {
          const Cx<float> v0 = v[k], v1 = v[k | m];
          v[k] = Cx<float>{c * v0.x + s * v1.y, c * v0.y - s * v1.x};
          v[k | m] = Cx<float>{c * v1.x + s * v0.y, c * v1.y - s * v0.x};
        }
    }
  }
  // W on the matrix cores: K = 32 real inputs in 8 steps of 4, two M-tiles
  const float *A = a.tab + (size_t)(a.layer * (n / 4) + a.blk) * 2 * 8 * 64 + lane;
  k9f4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float bv = s < 4 ? v[s].x : v[s - 4].y;
    re = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s * 64], bv, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_16x16x4f32(A[(8 + s) * 64], bv, im, 0, 0, 0);
  }
  Cx<float> o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[k] = Cx<float>{re[k], im[k]};
    if (a.cross_out) {
      const uint32_t z = k9_sign(base | ((uint32_t)(4 * g + k) << sh), a.cross_out);
      o[k] = Cx<float>{flip(o[k].x, z), flip(o[k].y, z)};
    }
    st[base | ((uint32_t)(4 * g + k) << sh)] = o[k];
  }
  if (!a.part) return;
  // observables and norm: FP32 per-thread partials over 4 amplitudes, FP64
  // across lanes and waves; one partial row per workgroup
  __shared__ double red[4];
  const int rows = 1 << (n - 10);  // workgroups per sample (64 columns each)
  const int row = (int)(blockIdx.x & (rows - 1));
  for (int m = 0; m <= a.M; ++m) {
    const uint32_t mask = m < a.M ? (uint32_t)a.masks[m] : 0u;
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float p = o[k].x * o[k].x + o[k].y * o[k].y;
      acc += (__popc((base | ((uint32_t)(4 * g + k) << sh)) & mask) & 1) ? -p : p;
    }
    const double d = wave_sum_d((double)acc);
    if (lane == 0) red[wave] = d;
    __syncthreads();
    if (t == 0) a.part[((int64_t)b * rows + row) * (a.M + 1) + m] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host

bool k9_detect(const CircuitDesc &d, K9Layout &out, std::string &why) {
  const int n = d.n;
  if (n < 12 || n % 4 != 0) {
    why = "the dense-block forward needs a multiple of 4 qubits, at least 12";
    return false;
  }
  const int per = 3 * n + (n - 1);
  const int G = (int)d.gates.size();
  if (G == 0 || G % per != 0) {
    why = "not a layered RX / RY / RZ / CZ-chain circuit";
    return false;
  }
  const int L = G / per;
  K9Layout k;
  k.n = n;
  k.L = L;
  k.rx.assign((size_t)L * n, 0);
  k.ry.assign((size_t)L * n, 0);
  k.rz.assign((size_t)L * n, 0);
  for (int l = 0; l < L; ++l) {
    const Gate *g = d.gates.data() + (size_t)l * per;
    for (int q = 0; q < n; ++q) {
      const Gate &x = g[q], &y = g[n + q], &z = g[2 * n + q];
      if (x.type != G_RX || x.q0 != q || x.src != S_INPUT || y.type != G_RY || y.q0 != q ||
          y.src != S_WEIGHT || z.type != G_RZ || z.q0 != q || z.src != S_WEIGHT) {
        why = "not a layered RX(input) / RY(weight) / RZ(weight) / CZ-chain circuit";
        return false;
      }
      k.rx[(size_t)l * n + q] = x.index;
      k.ry[(size_t)l * n + q] = y.index;
      k.rz[(size_t)l * n + q] = z.index;
    }
    for (int q = 0; q + 1 < n; ++q) {
      const Gate &c = g[3 * n + q];
      if (c.type != G_CZ || std::min(c.q0, c.q1) != q || std::max(c.q0, c.q1) != q + 1) {
        why = "the entangler is not the open CZ chain";
        return false;
      }
    }
  }
  out = std::move(k);
  return true;
}

size_t k9_tab_floats(const K9Layout &k) { return (size_t)k.L * (k.n / 4) * 2 * 8 * 64; }
int k9_part_rows(const K9Layout &k) { return 1 << (k.n - 10); }

hipError_t k9_forward(const K9Dev &k, const DevCircuit &d, int B, const double *x, const double *w, void *state,
                      float *tab, float2 *rxcs, double *part, double *out, hipStream_t s, SweepTimer *tm) {
  const int n = k.n, L = k.L, nb = n / 4;
  const int64_t dim = (int64_t)1 << n;
  Cx<float> *st = reinterpret_cast<Cx<float> *>(state);
  k_k9_init<<<(unsigned)((B * dim + 255) / 256), 256, 0, s>>>(st, B * dim, dim);
  k_k9_prep_w<<<(L * nb + 63) / 64, 64, 0, s>>>(L * nb, nb, k.ry, k.rz, w, tab);
  k_k9_prep_rx<<<(unsigned)(((int64_t)B * L * n + 255) / 256), 256, 0, s>>>(B, L, n, d.n_inputs, k.rx, x, rxcs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // CZ pairs between blocks: (4 j + 3, 4 j + 4)
  uint32_t cross = 0;
  for (int j = 0; j + 1 < nb; ++j) cross |= 1u << (4 * j + 3);
  const unsigned grid = (unsigned)((int64_t)B * (dim >> 4) / 64);
  for (int l = 0; l < L; ++l)
    for (int j = 0; j < nb; ++j) {
      K9PassArgs a;
      a.state = st;
      a.tab = tab;
      a.rx = rxcs;
      a.n = n;
      a.L = L;
      a.layer = l;
      a.blk = j;
      a.cross_in = (l > 0 && j == 0) ? cross : 0u;
      const bool last = l == L - 1 && j == nb - 1;
      a.cross_out = last ? cross : 0u;
      a.M = d.n_obs;
      a.masks = d.masks;
      a.part = last ? part : nullptr;
      if (tm) tm->before(0, s);
      k_k9_pass<<<grid, 256, 0, s>>>(a);
      if (tm) tm->after(0, s);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  return launch_obs_final(part, B, 1 << (n - 10), d.n_obs, out, true, s);
}

}  // namespace qtm
