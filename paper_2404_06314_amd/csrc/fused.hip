// Fused path: LDS-tiled, register-staged sweeps.
//
// A sweep loads a tile of 2^KT amplitudes of one sample (the `klo` lowest
// qubits contiguous, plus KT - klo others chosen by the planner), runs a
// chain of stages on it and writes it back.  In a stage every thread holds
// 16 amplitudes in registers: the ones that differ in the stage's 4 register
// bits.  Single-qubit blocks (the fused RZ RY RX of one wire and layer) and
// CNOT targets act on register bits; CZ gates act as a sign computed from
// the global index.  Between stages the tile is exchanged through LDS (an
// XOR-swizzled layout that keeps the per-stage index arithmetic separable).
//
// Forward: the last sweep also reads every Pauli-Z string expectation value
// (Sec. II-A: all observables from one evolved state) and the norm.
// Backward: the reverse sweeps carry the ket psi and the combined bra
// lambda = (sum_m G_m O_m) psi together; before un-applying a parameterised
// block on wire q they accumulate the three numbers Im Tr(P T) (P = X, Y, Z)
// of the 2x2 transition matrix T[a][b] = sum_r psi(b, r) conj(lambda(a, r));
// the derivative of every rotation inside the block follows from them and
// the block's later rotations (see k_fused_prep).
#include <mutex>
#include <type_traits>

#include "jit.h"
#include "kernels.h"
#include "sweep_ops.h"

namespace qtm {

constexpr int kMaxWgPerSample = 512;

int fused_wg_per_sample(int n, int kt) {
  int64_t tiles = (int64_t)1 << (n - kt);
  return (int)(tiles < kMaxWgPerSample ? tiles : kMaxWgPerSample);
}

size_t fused_part_obs_doubles(const DevCircuit &d, const DevPlan &p, int B) {
  return (size_t)B * fused_wg_per_sample(d.n, p.kt) * (d.n_obs + 1);
}
size_t fused_rn_doubles(const DevCircuit &d, const DevPlan &p, int B) {
  return (size_t)std::max(p.n_sweeps, 1) * B * fused_wg_per_sample(d.n, p.kt) * 5;
}
size_t fused_part_grad_doubles(const DevCircuit &d, const DevPlan &p, int B) {
  return (size_t)B * (size_t)(p.n_gslots > 0 ? p.n_gslots : 1) * fused_wg_per_sample(d.n, p.kt) * 3;
}

// ---------------------------------------------------------------------------
// matrix prep: U = G_last ... G_first per (sample, block), FP64, stored in R;
// for each rotation j of the block, P'_j = A_j P_j A_j^dag with A_j the
// block's rotations after j, stored as (px, py, pz): P'_j = px X + py Y + pz Z.
template <typename R>
__global__ void k_fused_prep(int B, int n_blocks, const int32_t *__restrict__ blk,
                             const int32_t *__restrict__ blk_off, const double *__restrict__ x,
                             int n_in, const double *__restrict__ w, M2<R> *__restrict__ mats,
                             double *__restrict__ coef, int n_occ) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * n_blocks) return;
  const int b = (int)(i / n_blocks), k = (int)(i % n_blocks);
  prep_block<R>(blk + blk_off[k], x + (int64_t)b * n_in, w, mats + i,
                coef ? coef + (int64_t)b * n_occ * 3 : nullptr);
}

// ---------------------------------------------------------------------------
// forward sweep

template <typename R, int KT>
__global__ void __launch_bounds__(1 << (KT - kRegBits), sizeof(R) == 4 ? 2 : 1) k_fused_fwd(FwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool FULL = true;
  constexpr int ntb = KT - kRegBits;
  constexpr bool active = true;
  const int b = blockIdx.y, wg = blockIdx.x, nwg = gridDim.x;
#include "sweep_fwd.inc"
}

// ---------------------------------------------------------------------------
// backward sweep

// (three workgroups per compute unit for the matrix-core kernels, which
// pass psi and lambda through one LDS tile)
template <typename R, int KT>
__global__ void __launch_bounds__(1 << (KT - kRegBits), sizeof(R) == 4 ? (KT - kRegBits >= 6 ? 3 : 2) : 1)
    k_fused_bwd(BwdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool FULL = true;
  constexpr int ntb = KT - kRegBits;
  constexpr bool active = true;
  const int b = blockIdx.y, wg = blockIdx.x, nwg = gridDim.x;
#include "sweep_bwd.inc"
}

// One workgroup per (gradient slot gs, sample b): the slot's transition-
// matrix components summed over the workgroup partials and the norm summed
// over the first backward sweep's partials (fixed order), then
// g[b][k] = (px TX + py TY + pz TZ) / norm for every rotation k of the slot.
__global__ void __launch_bounds__(64) k_fused_grad_slot(const double *__restrict__ part,
                                                        const double *__restrict__ pnorm,
                                                        const double *__restrict__ coef,
                                                        const int32_t *__restrict__ gs_ptr,
                                                        const int32_t *__restrict__ gs_occ, int n_occ,
                                                        int n_gslots, int nwg,
                                                        const int32_t *__restrict__ gs_rows,
                                                        double *__restrict__ gocc) {
  // one wave per (slot, sample)
  const int gs = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  // rows of the slot's partials: one per workgroup of its sweep (fewer than
  // nwg where the specialised sweep runs only the tiles that can be nonzero)
  const int rows = gs_rows ? gs_rows[gs] : nwg;
  // the slot's rows are contiguous (3 components each): consecutive lanes
  // read consecutive doubles; element e = t + 64 k is component e % 3
  const double *p = part + ((int64_t)b * n_gslots + gs) * nwg * 3;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = t, c = t % 3; e < rows * 3; e += 64, c = c == 2 ? 0 : c + 1) acc[c] += p[e];
  double nr = 0.0;
  for (int wg = t; wg < nwg; wg += 64) nr += pnorm[(int64_t)b * nwg + wg];
  const double tx = wave_sum_w<64>(acc[0]), ty = wave_sum_w<64>(acc[1]), tz = wave_sum_w<64>(acc[2]);
  nr = wave_sum_w<64>(nr);
  for (int e = gs_ptr[gs] + t; e < gs_ptr[gs + 1]; e += 64) {
    const int k = gs_occ[e];
    const double *cf = coef + ((int64_t)b * n_occ + k) * 3;
    gocc[(int64_t)b * n_occ + k] = (cf[0] * tx + cf[1] * ty + cf[2] * tz) / nr;
  }
}

// ---------------------------------------------------------------------------
// host side

template <typename R, int KT>
static size_t fwd_lds(int M) {
  constexpr int NW = ((1 << (KT - kRegBits)) + 63) / 64;
  return (sizeof(Cx<R>) << KT) + sizeof(M2<R>) * kMaxSweepBlocks + sizeof(double) * (size_t)(M + 1) * NW;
}
template <typename R, int KT>
static size_t bwd_lds(int ngs) {
  constexpr int NT = 1 << (KT - kRegBits);
  constexpr int NW = (NT + 63) / 64;
  // one tile for psi and lambda in turn in the matrix-core kernels, else two
  constexpr int tiles = sizeof(R) == 4 && NT >= 64 ? 1 : 2;
  const size_t acc = (size_t)ngs * 3 * NW;
  return (tiles * sizeof(Cx<R>) << KT) + sizeof(M2<R>) * kMaxSweepBlocks + sizeof(double) * (2 * NW + acc);
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// One sweep launch: the specialised kernel when there is one, else the
// compiled kernel for this tile size.
template <typename K, typename A>
static hipError_t launch_sweep(K kernel, const JitSweeps *js, int dir, int sw, int nwg, int B, int nt,
                               size_t lds, hipStream_t s, A &a) {
  if (js) {
    void *args[] = {&a};
    return hipModuleLaunchKernel(js->k[dir][sw].fn, js->nwg[dir][sw], B, 1, nt, 1, 1, 0, s, args, nullptr);
  }
  hipLaunchKernelGGL(kernel, dim3(nwg, B), dim3(nt), lds, s, a);
  return hipSuccess;
}

template <typename R, int KT>
static hipError_t run_fwd(const DevCircuit &d, const DevPlan &p, int B, const double *x, const double *w,
                          void *mats, double *coef, void *state, double *part_obs, double *out,
                          bool store_final, hipStream_t s, SweepTimer *tm, const JitSweeps *js,
                          const Renorm &rn) {
  const int nwg = fused_wg_per_sample(d.n, KT);
  const size_t lds = fwd_lds<R, KT>(d.n_obs);
  hipError_t e = allow_lds(k_fused_fwd<R, KT>, lds);
  if (e != hipSuccess) return e;
  for (int sw = 0; sw < p.n_sweeps; ++sw) {
    FwdArgs a;
    a.prog = p.code;
    a.thr = p.thr;
    a.sweep_off = p.sweep_off_fwd[sw];
    a.n = d.n;
    a.state = state;
    a.mats = mats;
    a.n_blocks = p.n_blocks;
    a.ntiles = 1 << (d.n - KT);
    a.first = sw == 0;
    a.last = sw == p.n_sweeps - 1;
    a.store = !a.last || store_final;
    a.masks = d.masks;
    a.M = d.n_obs;
    a.obs_sgn = p.obs_sgn_f;
    a.part_obs = part_obs;
    a.out = out;
    if (sw == 0 && js && js->loaded && js->direct_prep) {
      a.blk = p.blk;
      a.blk_off = p.blk_off;
      a.x = x;
      a.w = w;
      a.n_in = d.n_inputs;
      a.n_occ = d.n_occ;
      a.mats_out = mats;
      a.coef = coef;
    }
    if (rn.period > 0) {
      // sweep sw rescales when it is a positive multiple of the period; the
      // sweep before it records its end norm
      if (sw > 0 && sw % rn.period == 0) {
        a.rn_prev = rn.fwd + (size_t)(sw - 1) * B * nwg;
        a.rn_prev_n = js ? js->nwg[0][sw - 1] : nwg;
      }
      if (sw + 1 < p.n_sweeps && (sw + 1) % rn.period == 0) a.rn_out = rn.fwd + (size_t)sw * B * nwg;
    }
    if (tm) tm->before(0, s);
    e = launch_sweep(k_fused_fwd<R, KT>, js, 0, sw, nwg, B, 1 << (KT - kRegBits), lds, s, a);
    if (tm) tm->after(0, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <typename R, int KT>
static hipError_t run_bwd(const DevCircuit &d, const DevPlan &p, int B, const double *G, void *mats,
                          void *psi, const void *psi_in, void *lam, double *part_grad, double *part_norm,
                          const double *coef, double *gocc, hipStream_t s, SweepTimer *tm, const JitSweeps *js,
                          const Renorm &rn) {
  const int nwg = fused_wg_per_sample(d.n, KT);
  const size_t lds = bwd_lds<R, KT>(p.max_gslots);
  hipError_t e = allow_lds(k_fused_bwd<R, KT>, lds);
  if (e != hipSuccess) return e;
  for (int sw = 0; sw < p.n_sweeps; ++sw) {
    BwdArgs a;
    a.prog = p.code;
    a.thr = p.thr;
    a.sweep_off = p.sweep_off_bwd[sw];
    a.n = d.n;
    a.psi = psi;
    a.psi_in = sw == 0 ? psi_in : nullptr;
    a.coef = coef;
    a.gocc = gocc;
    a.n_occ = d.n_occ;
    a.lam = lam;
    a.mats = mats;
    a.n_blocks = p.n_blocks;
    a.ntiles = 1 << (d.n - KT);
    a.first = sw == 0;
    a.store = sw != p.n_sweeps - 1;
    a.masks = d.masks;
    a.M = d.n_obs;
    a.G = G;
    a.seed_sgn = p.seed_sgn;
    a.seed_add = sw == 0 && d.n_nd > 0;
    a.part_grad = part_grad;
    a.n_gslots = p.n_gslots > 0 ? p.n_gslots : 1;
    a.part_norm = part_norm;
    if (rn.period > 0) {
      a.rn_rec = rn.bwd;
      a.rn_i = sw;
      a.rn_period = rn.period;
      a.rn_rows = nwg;
    }
    if (tm) tm->before(1, s);
    e = launch_sweep(k_fused_bwd<R, KT>, js, 1, sw, nwg, B, 1 << (KT - kRegBits), lds, s, a);
    if (tm) tm->after(1, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

static inline unsigned nblocks256(int64_t w) { return (unsigned)((w + 255) / 256); }

template <typename R>
static hipError_t prep(const DevCircuit &d, const DevPlan &p, int B, const double *x,
                       const double *w, void *mats, double *coef, hipStream_t s) {
  if (p.n_blocks == 0) return hipSuccess;
  k_fused_prep<R><<<nblocks256((int64_t)B * p.n_blocks), 256, 0, s>>>(
      B, p.n_blocks, p.blk, p.blk_off, x, d.n_inputs, w, reinterpret_cast<M2<R> *>(mats), coef,
      d.n_occ);
  return hipGetLastError();
}

#define QTM_KT_DISPATCH(KTV, CALL) \
  switch (KTV) {                   \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    case 6: CALL(6); break;        \
    case 7: CALL(7); break;        \
    case 8: CALL(8); break;        \
    case 9: CALL(9); break;        \
    case 10: CALL(10); break;      \
    case 11: CALL(11); break;      \
    case 12: CALL(12); break;      \
    default: return hipErrorInvalidValue; \
  }

template <typename R>
hipError_t fused_forward(const DevCircuit &d, const DevPlan &p, int B, const double *x,
                         const double *w, void *mats, double *coef, void *state, double *part_obs,
                         double *out, bool store_final, hipStream_t s, SweepTimer *tm,
                         const JitSweeps *js, const Renorm &rn) {
  // (a specialised forward that prepares the matrices itself needs no prep launch)
  hipError_t e = js && js->loaded && js->direct_prep ? hipSuccess : prep<R>(d, p, B, x, w, mats, coef, s);
  if (e != hipSuccess) return e;
#define FWD_CALL(K) \
  e = run_fwd<R, K>(d, p, B, x, w, mats, coef, state, part_obs, out, store_final, s, tm, js, rn)
  QTM_KT_DISPATCH(p.kt, FWD_CALL)
#undef FWD_CALL
  if (e != hipSuccess) return e;
  // a specialised last sweep over single-tile samples has written out
  if (js && js->loaded && js->direct_obs) return hipSuccess;
  return launch_obs_final(part_obs, B, fused_wg_per_sample(d.n, p.kt), d.n_obs, out, true, s);
}

template <typename R>
hipError_t fused_backward(const DevCircuit &d, const DevPlan &p, int B, const double *x,
                          const double *w, const double *G, void *mats, double *coef, bool prepped,
                          void *state, const void *state_in, void *lam, double *part_grad,
                          double *part_norm, double *gocc, double *gw, double *gx, hipStream_t s,
                          SweepTimer *tm, const JitSweeps *js, const Renorm &rn) {
  // prepped: mats and coef still hold what the forward computed from the
  // same angles for this plan and batch
  hipError_t e = prepped ? hipSuccess : prep<R>(d, p, B, x, w, mats, coef, s);
  if (e != hipSuccess) return e;
  // bra term of observables with X or Y factors, added in the first sweep
  if ((e = launch_pauli_seed<R>(d, B, state_in ? state_in : state, lam, G, false, s)) != hipSuccess) return e;
#define BWD_CALL(K) \
  e = run_bwd<R, K>(d, p, B, G, mats, state, state_in, lam, part_grad, part_norm, coef, gocc, s, tm, js, rn)
  QTM_KT_DISPATCH(p.kt, BWD_CALL)
#undef BWD_CALL
  if (e != hipSuccess) return e;
  // (a specialised one-sweep backward over single-tile samples has written
  // the per-rotation gradients itself)
  if (d.n_occ > 0 && p.n_gslots > 0 && !(js && js->loaded && js->direct_grad)) {
    const int nwg = fused_wg_per_sample(d.n, p.kt);
    k_fused_grad_slot<<<dim3(p.n_gslots, B), 64, 0, s>>>(
        part_grad, part_norm, coef, p.gs_ptr, p.gs_occ, d.n_occ, p.n_gslots, nwg,
        js ? js->gs_rows_dev : nullptr, gocc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_scatter(d, B, gocc, x, w, gw, gx, s);
}

template hipError_t fused_forward<float>(const DevCircuit &, const DevPlan &, int, const double *,
                                         const double *, void *, double *, void *, double *, double *,
                                         bool, hipStream_t, SweepTimer *, const JitSweeps *, const Renorm &);
template hipError_t fused_forward<double>(const DevCircuit &, const DevPlan &, int, const double *,
                                          const double *, void *, double *, void *, double *, double *,
                                          bool, hipStream_t, SweepTimer *, const JitSweeps *, const Renorm &);
template hipError_t fused_backward<float>(const DevCircuit &, const DevPlan &, int, const double *,
                                          const double *, const double *, void *, double *, bool,
                                          void *, const void *, void *, double *, double *, double *, double *,
                                          double *, hipStream_t, SweepTimer *, const JitSweeps *,
                                          const Renorm &);
template hipError_t fused_backward<double>(const DevCircuit &, const DevPlan &, int, const double *,
                                           const double *, const double *, void *, double *, bool,
                                           void *, const void *, void *, double *, double *, double *, double *,
                                           double *, hipStream_t, SweepTimer *, const JitSweeps *,
                                           const Renorm &);

}  // namespace qtm
