// Uneven batch: many circuits of different width and depth, one sample each
// (Sec. II-B: batch elements are independent, so nothing forces them to share
// a circuit), run by one persistent kernel per direction.
//
// Work unit = one tile of one sweep of one circuit.  All units of a pass sit
// in one queue whose order comes from a list schedule of the sweep chains
// (longest remaining chain first).  A workgroup takes the next ticket from an
// atomic counter, waits until every tile of the previous sweep of the same
// circuit is done (a per-circuit counter), runs the tile with the same sweep
// body as the batched kernels, and bumps the counter.  Every dependency of a
// unit sits earlier in the queue and was taken by a running workgroup, so the
// waits always end; the wait is also bounded (on time-out the pass's outputs
// become NaN instead of the kernel spinning).
//
// Circuits narrower than the compiled tile run with the surplus threads idle
// on zeros: their LDS slots lie above the circuit's 2^kt amplitudes and are
// cleared when a unit starts.
//
// The forward pass is reset -> matrix prep -> persistent sweeps -> final
// reduction; the backward pass is reset -> prep (with rotation
// coefficients) -> persistent sweeps -> gradient assembly.  Each pass is one
// hipGraph built once per handle; only the caller's pointers change between
// calls, and they are patched into the kernel nodes before a launch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>

#include "multi.h"
#include "schedule.h"
#include "kernels.h"
#include "sweep_ops.h"

namespace qtm {

constexpr int kMultiKT = kMaxTileQubits;
constexpr int kMultiNT = 1 << (kMultiKT - kRegBits);
constexpr int kMultiMaxSpins = 1 << 21;

// Per-item descriptor: int64 words, read with scalar loads.
enum : int {
  MI_CODE, MI_THR, MI_SW, MI_NSW, MI_N, MI_KT, MI_NTILES, MI_NBLK,
  MI_NGS, MI_M, MI_MASKS, MI_OSG, MI_SSG, MI_BLK, MI_BLKOFF, MI_OCCG,
  MI_NOCC, MI_NIN, MI_NW, MI_WPTR, MI_WLIST, MI_XPTR, MI_XLIST, MI_ST,
  MI_MATS, MI_OCC, MI_POBS, MI_PGRAD, MI_PNORM, MI_INOFF, MI_WOFF, MI_OUTOFF,
  MI_WORDS
};

// Counters: [ticket_f, err_f, done_f[N]] then [ticket_b, err_b, done_b[N]].
struct MultiStatic {
  const int32_t *code, *thr, *sw, *blk, *csr, *occg;
  const int32_t *units;  // [n_units][4]: item, sweep, tile, 0
  const int64_t *items;
  const uint64_t *masks;
  const float *osg;
  const double *ssg;
  M2<float> *mats;
  double *coef, *gocc, *part_obs, *part_grad, *part_norm;
  Cx<float> *lam;
  int *ctr;  // this pass's counters: [0] ticket, [1] error, [2 ..) done per item
  int n_items, n_units;
};

struct MultiIO {
  const double *x, *w, *G;
  double *out, *gw, *gx;
  Cx<float> *state;
};

__global__ void k_multi_reset(int *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void __launch_bounds__(256) k_multi_prep(MultiStatic ms, MultiIO io, int with_coef) {
  const int64_t *I = ms.items + (int64_t)blockIdx.x * MI_WORDS;
  const int nb = (int)I[MI_NBLK];
  const int32_t *blk = ms.blk + I[MI_BLK];
  const int32_t *bo = ms.blk + I[MI_BLKOFF];
  const double *x = io.x ? io.x + I[MI_INOFF] : nullptr;
  const double *w = io.w ? io.w + I[MI_WOFF] : nullptr;
  for (int k = threadIdx.x; k < nb; k += blockDim.x)
    prep_block<float>(blk + bo[k], x, w, ms.mats + I[MI_MATS] + k,
                      with_coef ? ms.coef + 3 * I[MI_OCC] : nullptr);
}

// Thread 0 polls (relaxed, bounded) until *cnt >= target, then acquires at
// agent scope once; the cache invalidation that acquire performs is
// cache-wide, and the barrier orders the other threads' loads after it.
__device__ __forceinline__ void multi_wait(int *cnt, int target, int *err) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > kMultiMaxSpins) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// s_waitcnt vmcnt(0) (gfx9 encoding: expcnt and lgkmcnt left at their maxima)
constexpr int kWaitVmcnt0 = 0x0F70;

// Every thread waits until its own stores of the unit have completed; after
// the barrier thread 0 releases them at agent scope (one L2 write-back for
// the workgroup) and counts the unit as done.
__device__ __forceinline__ void multi_signal(int *cnt) {
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ int multi_ticket(int *ctr, int *slot) {
  __syncthreads();
  if (threadIdx.x == 0) *slot = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*slot);
}

// Clear the LDS slots above a narrow circuit's 2^kt amplitudes (nreg tiles).
__device__ __forceinline__ void zero_surplus(unsigned char *smem, int kt, int nreg) {
  Cx<float> *p = reinterpret_cast<Cx<float> *>(smem);
  for (int r = 0; r < nreg; ++r)
    for (int i = (1 << kt) + threadIdx.x; i < (1 << kMultiKT); i += kMultiNT)
      p[(r << kMultiKT) + i] = Cx<float>{0.f, 0.f};
}

__global__ void __launch_bounds__(kMultiNT, 2) k_multi_fwd(MultiStatic ms, MultiIO io) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tk;
  using R = float;
  constexpr int KT = kMultiKT;
  constexpr bool FULL = false;
  int *const done = ms.ctr + 2;
  for (;;) {
    const int tk = multi_ticket(ms.ctr, &s_tk);
    if (tk >= ms.n_units) break;
    const cptr<int32_t> U = as_const(ms.units) + 4 * (int64_t)tk;
    const int item = U[0], sweep = U[1], tile = U[2];
    const cptr<int64_t> I = as_const(ms.items) + (int64_t)item * MI_WORDS;
    const int ntiles = (int)I[MI_NTILES], kt = (int)I[MI_KT];
    if (sweep > 0) multi_wait(done + item, sweep * ntiles, ms.ctr + 1);
    if (kt < KT) zero_surplus(smem, kt, 1);
    FwdArgs a;
    a.prog = ms.code + I[MI_CODE];
    a.thr = ms.thr + I[MI_THR];
    a.sweep_off = as_const(ms.sw)[I[MI_SW] + sweep];
    a.n = (int)I[MI_N];
    a.state = io.state + I[MI_ST];
    a.mats = ms.mats + I[MI_MATS];
    a.n_blocks = (int)I[MI_NBLK];
    a.ntiles = ntiles;
    a.first = sweep == 0;
    a.last = sweep == (int)I[MI_NSW] - 1;
    a.store = 1;
    a.masks = ms.masks + I[MI_MASKS];
    a.M = (int)I[MI_M];
    a.obs_sgn = ms.osg + I[MI_OSG];
    a.part_obs = ms.part_obs + I[MI_POBS];
    const int ntb = kt - kRegBits;
    const bool active = (int)threadIdx.x < (1 << ntb);
    const int b = 0, wg = tile, nwg = ntiles;
#include "sweep_fwd.inc"
    multi_signal(done + item);
  }
}

// (three workgroups per compute unit: psi and lambda pass through one LDS
// tile in turn)
__global__ void __launch_bounds__(kMultiNT, 3) k_multi_bwd(MultiStatic ms, MultiIO io) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tk;
  using R = float;
  constexpr int KT = kMultiKT;
  constexpr bool FULL = false;
  int *const done = ms.ctr + 2;
  for (;;) {
    const int tk = multi_ticket(ms.ctr, &s_tk);
    if (tk >= ms.n_units) break;
    const cptr<int32_t> U = as_const(ms.units) + 4 * (int64_t)tk;
    const int item = U[0], sweep = U[1], tile = U[2];
    const cptr<int64_t> I = as_const(ms.items) + (int64_t)item * MI_WORDS;
    const int ntiles = (int)I[MI_NTILES], kt = (int)I[MI_KT];
    if (sweep > 0) multi_wait(done + item, sweep * ntiles, ms.ctr + 1);
    if (kt < KT) zero_surplus(smem, kt, 1);
    BwdArgs a;
    a.prog = ms.code + I[MI_CODE];
    a.thr = ms.thr + I[MI_THR];
    a.sweep_off = as_const(ms.sw)[I[MI_SW] + I[MI_NSW] + sweep];
    a.n = (int)I[MI_N];
    a.psi = io.state + I[MI_ST];
    a.lam = ms.lam + I[MI_ST];
    a.mats = ms.mats + I[MI_MATS];
    a.n_blocks = (int)I[MI_NBLK];
    a.ntiles = ntiles;
    a.first = sweep == 0;
    a.store = sweep != (int)I[MI_NSW] - 1;
    a.masks = ms.masks + I[MI_MASKS];
    a.M = (int)I[MI_M];
    a.G = io.G + I[MI_OUTOFF];
    a.seed_sgn = ms.ssg + I[MI_SSG];
    a.seed_add = 0;
    a.part_grad = ms.part_grad + I[MI_PGRAD];
    a.n_gslots = (int)I[MI_NGS];
    a.part_norm = ms.part_norm + I[MI_PNORM];
    const int ntb = kt - kRegBits;
    const bool active = (int)threadIdx.x < (1 << ntb);
    const int b = 0, wg = tile, nwg = ntiles;
#include "sweep_bwd.inc"
    multi_signal(done + item);
  }
}

// <Z-string m> = (sum over tiles of the partial) / (sum over tiles of the norm)
__global__ void __launch_bounds__(256) k_multi_fwd_final(MultiStatic ms, MultiIO io) {
  const int64_t *I = ms.items + (int64_t)blockIdx.x * MI_WORDS;
  const int M = (int)I[MI_M], T = (int)I[MI_NTILES];
  const double *p = ms.part_obs + I[MI_POBS];
  const bool bad = ms.ctr[1] != 0;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    double acc = 0.0, nrm = 0.0;
    for (int t = 0; t < T; ++t) {
      acc += p[(int64_t)t * (M + 1) + m];
      nrm += p[(int64_t)t * (M + 1) + M];
    }
    io.out[I[MI_OUTOFF] + m] = bad ? NAN : acc / nrm;
  }
}

// Per occurrence k: (px TX + py TY + pz TZ) / norm, then every input and
// weight slot of the item sums its occurrences (construction order), times
// the other factor for a weight-scaled input angle.
__global__ void __launch_bounds__(256) k_multi_bwd_final(MultiStatic ms, MultiIO io) {
  const int64_t *I = ms.items + (int64_t)blockIdx.x * MI_WORDS;
  const int T = (int)I[MI_NTILES], nocc = (int)I[MI_NOCC];
  const bool bad = ms.ctr[1] != 0;
  const double *pn = ms.part_norm + I[MI_PNORM];
  const double *pg = ms.part_grad + I[MI_PGRAD];
  const int32_t *occg = ms.occg + I[MI_OCCG];
  double *gocc = ms.gocc + I[MI_OCC];
  double nrm = 0.0;
  for (int t = 0; t < T; ++t) nrm += pn[t];
  for (int k = threadIdx.x; k < nocc; k += blockDim.x) {
    const int gs = occg[k];
    double tx = 0.0, ty = 0.0, tz = 0.0;
    for (int t = 0; t < T; ++t) {
      const double *q = pg + ((int64_t)gs * T + t) * 3;
      tx += q[0];
      ty += q[1];
      tz += q[2];
    }
    const double *cf = ms.coef + 3 * (I[MI_OCC] + k);
    gocc[k] = (cf[0] * tx + cf[1] * ty + cf[2] * tz) / nrm;
  }
  __syncthreads();
  const int nw = (int)I[MI_NW], nin = (int)I[MI_NIN];
  const int32_t *wp = ms.csr + I[MI_WPTR], *wl = ms.csr + I[MI_WLIST];
  const int32_t *xp = ms.csr + I[MI_XPTR], *xl = ms.csr + I[MI_XLIST];
  const int32_t *wf = wl + wp[nw], *xf = xl + xp[nin];
  const double *x = io.x ? io.x + I[MI_INOFF] : nullptr;
  const double *w = io.w ? io.w + I[MI_WOFF] : nullptr;
  for (int j = threadIdx.x; j < nw + nin; j += blockDim.x) {
    if (j < nw) {
      double acc = 0.0;
      for (int e = wp[j]; e < wp[j + 1]; ++e) acc += wf[e] < 0 ? gocc[wl[e]] : gocc[wl[e]] * x[wf[e]];
      io.gw[I[MI_WOFF] + j] = bad ? NAN : acc;
    } else if (io.gx) {
      const int i = j - nw;
      double acc = 0.0;
      for (int e = xp[i]; e < xp[i + 1]; ++e) acc += xf[e] < 0 ? gocc[xl[e]] : gocc[xl[e]] * w[xf[e]];
      io.gx[I[MI_INOFF] + i] = bad ? NAN : acc;
    }
  }
}

// ---------------------------------------------------------------------------
// host side

namespace {

size_t fwd_lds_bytes(int max_m) {
  constexpr int NW = (kMultiNT + 63) / 64;
  return (sizeof(Cx<float>) << kMultiKT) + sizeof(M2<float>) * kMaxSweepBlocks +
         sizeof(double) * (size_t)(max_m + 1) * NW;
}
size_t bwd_lds_bytes(int max_gs) {
  constexpr int NW = (kMultiNT + 63) / 64;
  // one tile: psi and lambda pass through it in turn
  return (sizeof(Cx<float>) << kMultiKT) + sizeof(M2<float>) * kMaxSweepBlocks +
         sizeof(double) * (size_t)(NW + (size_t)max_gs * 3 * NW);
}

template <typename T>
hipError_t dev_copy(T **dst, const std::vector<T> &src, std::vector<void *> &owned) {
  const size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
  hipError_t e = hipMalloc((void **)dst, bytes);
  if (e != hipSuccess) return e;
  owned.push_back(*dst);
  if (src.empty()) return hipSuccess;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

hipError_t dev_alloc(void **dst, size_t bytes, std::vector<void *> &owned) {
  hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
  if (e == hipSuccess) owned.push_back(*dst);
  return e;
}

struct ProgInfo {
  HostPlan hp;
  int64_t code, thr, sw, masks, osg, ssg, blk, blkoff, occg, wptr, wlist, xptr, xlist;
  int n, M, n_in, n_w, n_occ;
};

}  // namespace

struct MultiRuntime {
  std::vector<MultiItemIn> in;
  std::vector<ProgInfo> progs;
  std::vector<int> item_prog;
  // host tables
  std::vector<int32_t> code, thr, sw, blk, csr, occg;
  std::vector<uint64_t> masks;
  std::vector<float> osg;
  std::vector<double> ssg;
  std::vector<int64_t> items;
  int max_m = 0, max_gs = 0;
  int64_t n_mats = 0, n_occ = 0, n_pobs = 0, n_pgrad = 0, n_pnorm = 0, n_amps = 0;
  std::vector<std::vector<double>> cost_f, cost_b;
  std::vector<int> ntiles;
  // device
  int device = -1;
  bool uploaded = false;
  std::vector<void *> owned;
  MultiStatic sf{}, sb{};
  int grid_f = 0, grid_b = 0;
  size_t lds_f = 0, lds_b = 0;
  const char *where = "";  // the HIP call behind the last error
  struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node[4] = {};
    MultiIO io{};
    bool built = false;
  } graph[2];

  ~MultiRuntime() {
    for (auto &g : graph) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.g) (void)hipGraphDestroy(g.g);
    }
    for (void *p : owned) (void)hipFree(p);
  }

  std::string build(const std::vector<MultiItemIn> &items_in);
  hipError_t upload();
  hipError_t run(int pass, const MultiIO &io, hipStream_t s, SweepTimer *tm);
  void node_params(int pass, int k, const MultiIO &io, hipKernelNodeParams &p, void **args,
                   MultiStatic &ms_copy, MultiIO &io_copy, int &flag);
};

std::string MultiRuntime::build(const std::vector<MultiItemIn> &items_in) {
  in = items_in;
  std::map<std::string, int> seen;
  for (const MultiItemIn &it : in) {
    const CircuitDesc &d = *it.desc;
    std::string key;
    auto put = [&](const void *p, size_t n) { key.append(reinterpret_cast<const char *>(p), n); };
    const int32_t hdr[5] = {d.n, d.n_inputs, d.n_weights, it.kt, it.klo};
    put(hdr, sizeof(hdr));
    put(d.gates.data(), d.gates.size() * sizeof(Gate));
    put(d.masks.data(), d.masks.size() * sizeof(uint64_t));
    auto f = seen.find(key);
    if (f != seen.end()) {
      item_prog.push_back(f->second);
      continue;
    }
    ProgInfo pi;
    std::string why = build_host_plan(d, it.kt, it.klo, pi.hp);
    if (!why.empty()) return "internal planner error: " + why;
    pi.n = d.n;
    pi.M = (int)d.masks.size();
    pi.n_in = d.n_inputs;
    pi.n_w = d.n_weights;
    pi.n_occ = (int)d.occ_gate.size();
    pi.code = (int64_t)code.size();
    code.insert(code.end(), pi.hp.prog.code.begin(), pi.hp.prog.code.end());
    pi.thr = (int64_t)thr.size();
    thr.insert(thr.end(), pi.hp.prog.thr.begin(), pi.hp.prog.thr.end());
    pi.sw = (int64_t)sw.size();
    sw.insert(sw.end(), pi.hp.prog.sweep_off_fwd.begin(), pi.hp.prog.sweep_off_fwd.end());
    sw.insert(sw.end(), pi.hp.prog.sweep_off_bwd.begin(), pi.hp.prog.sweep_off_bwd.end());
    pi.masks = (int64_t)masks.size();
    masks.insert(masks.end(), d.masks.begin(), d.masks.end());
    pi.osg = (int64_t)osg.size();
    osg.insert(osg.end(), pi.hp.obs_sgn.begin(), pi.hp.obs_sgn.end());
    pi.ssg = (int64_t)ssg.size();
    ssg.insert(ssg.end(), pi.hp.seed_sgn.begin(), pi.hp.seed_sgn.end());
    pi.blk = (int64_t)blk.size();
    blk.insert(blk.end(), pi.hp.blk.begin(), pi.hp.blk.end());
    pi.blkoff = (int64_t)blk.size();
    blk.insert(blk.end(), pi.hp.blk_off.begin(), pi.hp.blk_off.end());
    pi.occg = (int64_t)occg.size();
    occg.insert(occg.end(), pi.hp.occ_gslot.begin(), pi.hp.occ_gslot.end());
    // parameter slot -> occurrences, construction order; each list is
    // followed by its chain-rule factor slots (same length)
    const ParamCsr pc = param_csr(d);
    auto put_csr = [&](const std::vector<int32_t> &ptr_, const std::vector<int32_t> &lst_,
                       const std::vector<int32_t> &fac_, int64_t &ptr, int64_t &lst) {
      ptr = (int64_t)csr.size();
      csr.insert(csr.end(), ptr_.begin(), ptr_.end());
      lst = (int64_t)csr.size();
      csr.insert(csr.end(), lst_.begin(), lst_.end());
      csr.insert(csr.end(), fac_.begin(), fac_.end());
    };
    put_csr(pc.w_ptr, pc.w_list, pc.w_fac, pi.wptr, pi.wlist);
    put_csr(pc.x_ptr, pc.x_list, pc.x_fac, pi.xptr, pi.xlist);
    // per-sweep cost estimates (tile loads + stages) for the list schedule
    seen.emplace(key, (int)progs.size());
    item_prog.push_back((int)progs.size());
    progs.push_back(std::move(pi));
  }
  // sweep costs per program, one entry per sweep
  std::vector<std::vector<double>> pcf(progs.size()), pcb(progs.size());
  for (size_t p = 0; p < progs.size(); ++p) {
    const Program &pr = progs[p].hp.prog;
    for (int32_t off : pr.sweep_off_fwd) pcf[p].push_back(2.0 + pr.code[off]);
    for (int32_t off : pr.sweep_off_bwd) pcb[p].push_back(4.0 + 2.0 * pr.code[off]);
  }
  for (size_t i = 0; i < in.size(); ++i) {
    const ProgInfo &pi = progs[item_prog[i]];
    const HostPlan &hp = pi.hp;
    const int T = 1 << (pi.n - hp.kt);
    const int ngs = std::max(hp.n_gslots, 1);
    int64_t w[MI_WORDS] = {};
    w[MI_CODE] = pi.code;
    w[MI_THR] = pi.thr;
    w[MI_SW] = pi.sw;
    w[MI_NSW] = hp.n_sweeps;
    w[MI_N] = pi.n;
    w[MI_KT] = hp.kt;
    w[MI_NTILES] = T;
    w[MI_NBLK] = hp.n_blocks;
    w[MI_NGS] = ngs;
    w[MI_M] = pi.M;
    w[MI_MASKS] = pi.masks;
    w[MI_OSG] = pi.osg;
    w[MI_SSG] = pi.ssg;
    w[MI_BLK] = pi.blk;
    w[MI_BLKOFF] = pi.blkoff;
    w[MI_OCCG] = pi.occg;
    w[MI_NOCC] = pi.n_occ;
    w[MI_NIN] = pi.n_in;
    w[MI_NW] = pi.n_w;
    w[MI_WPTR] = pi.wptr;
    w[MI_WLIST] = pi.wlist;
    w[MI_XPTR] = pi.xptr;
    w[MI_XLIST] = pi.xlist;
    w[MI_ST] = in[i].st_off;
    w[MI_MATS] = n_mats;
    w[MI_OCC] = n_occ;
    w[MI_POBS] = n_pobs;
    w[MI_PGRAD] = n_pgrad;
    w[MI_PNORM] = n_pnorm;
    w[MI_INOFF] = in[i].in_off;
    w[MI_WOFF] = in[i].w_off;
    w[MI_OUTOFF] = in[i].out_off;
    items.insert(items.end(), w, w + MI_WORDS);
    n_mats += std::max(hp.n_blocks, 1);
    n_occ += pi.n_occ;
    n_pobs += (int64_t)T * (pi.M + 1);
    n_pgrad += (int64_t)ngs * T * 3;
    n_pnorm += T;
    n_amps = std::max<int64_t>(n_amps, in[i].st_off + ((int64_t)1 << pi.n));
    max_m = std::max(max_m, pi.M);
    max_gs = std::max(max_gs, hp.max_gslots);
    cost_f.push_back(pcf[item_prog[i]]);
    cost_b.push_back(pcb[item_prog[i]]);
    ntiles.push_back(T);
  }
  return "";
}

#define QTM_TRY(call)         \
  do {                        \
    where = #call;            \
    if ((e = (call))) return e; \
  } while (0)

hipError_t MultiRuntime::upload() {
  hipError_t e;
  int cus = 0, occ_f = 0, occ_b = 0;
  QTM_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  lds_f = fwd_lds_bytes(max_m);
  lds_b = bwd_lds_bytes(max_gs);
  for (auto kl : {std::make_pair((const void *)k_multi_fwd, lds_f),
                  std::make_pair((const void *)k_multi_bwd, lds_b)})
    if (kl.second > 65536)
      QTM_TRY(hipFuncSetAttribute(kl.first, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kl.second));
  QTM_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, k_multi_fwd, kMultiNT, lds_f));
  QTM_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_b, k_multi_bwd, kMultiNT, lds_b));
  const int P_f = std::max(1, cus * std::max(occ_f, 1));
  const int P_b = std::max(1, cus * std::max(occ_b, 1));
  const std::vector<int32_t> uf = multi_schedule(cost_f, ntiles, P_f);
  const std::vector<int32_t> ub = multi_schedule(cost_b, ntiles, P_b);
  const int nu_f = (int)(uf.size() / 4), nu_b = (int)(ub.size() / 4);
  grid_f = std::max(1, std::min(P_f, nu_f));
  grid_b = std::max(1, std::min(P_b, nu_b));

  MultiStatic s{};
  int32_t *dcode, *dthr, *dsw, *dblk, *dcsr, *doccg, *duf, *dub;
  int64_t *ditems;
  uint64_t *dmasks;
  float *dosg;
  double *dssg;
  where = "device tables";
  if ((e = dev_copy(&dcode, code, owned)) || (e = dev_copy(&dthr, thr, owned)) ||
      (e = dev_copy(&dsw, sw, owned)) || (e = dev_copy(&dblk, blk, owned)) ||
      (e = dev_copy(&dcsr, csr, owned)) || (e = dev_copy(&doccg, occg, owned)) ||
      (e = dev_copy(&duf, uf, owned)) || (e = dev_copy(&dub, ub, owned)) ||
      (e = dev_copy(&ditems, items, owned)) || (e = dev_copy(&dmasks, masks, owned)) ||
      (e = dev_copy(&dosg, osg, owned)) || (e = dev_copy(&dssg, ssg, owned)))
    return e;
  void *mats, *coef, *gocc, *pobs, *pgrad, *pnorm, *lam, *ctr;
  const int N = (int)in.size();
  where = "device workspace";
  if ((e = dev_alloc(&mats, sizeof(M2<float>) * n_mats, owned)) ||
      (e = dev_alloc(&coef, sizeof(double) * 3 * n_occ, owned)) ||
      (e = dev_alloc(&gocc, sizeof(double) * n_occ, owned)) ||
      (e = dev_alloc(&pobs, sizeof(double) * n_pobs, owned)) ||
      (e = dev_alloc(&pgrad, sizeof(double) * n_pgrad, owned)) ||
      (e = dev_alloc(&pnorm, sizeof(double) * n_pnorm, owned)) ||
      (e = dev_alloc(&lam, sizeof(Cx<float>) * n_amps, owned)) ||
      (e = dev_alloc(&ctr, sizeof(int) * (size_t)(4 + 2 * N), owned)))
    return e;
  s.code = dcode;
  s.thr = dthr;
  s.sw = dsw;
  s.blk = dblk;
  s.csr = dcsr;
  s.occg = doccg;
  s.items = ditems;
  s.masks = dmasks;
  s.osg = dosg;
  s.ssg = dssg;
  s.mats = (M2<float> *)mats;
  s.coef = (double *)coef;
  s.gocc = (double *)gocc;
  s.part_obs = (double *)pobs;
  s.part_grad = (double *)pgrad;
  s.part_norm = (double *)pnorm;
  s.lam = (Cx<float> *)lam;
  s.n_items = N;
  sf = s;
  sf.units = duf;
  sf.n_units = nu_f;
  sf.ctr = (int *)ctr;
  sb = s;
  sb.units = dub;
  sb.n_units = nu_b;
  sb.ctr = (int *)ctr + 2 + N;
  uploaded = true;
  return hipSuccess;
}

// Kernel k of pass `pass` (0 forward, 1 backward): reset, prep, sweeps, final.
void MultiRuntime::node_params(int pass, int k, const MultiIO &io, hipKernelNodeParams &p,
                               void **args, MultiStatic &ms_copy, MultiIO &io_copy, int &flag) {
  const MultiStatic &ms = pass == 0 ? sf : sb;
  const int N = (int)in.size();
  ms_copy = ms;
  io_copy = io;
  p = hipKernelNodeParams{};
  p.blockDim = dim3(256);
  p.sharedMemBytes = 0;
  p.extra = nullptr;
  p.kernelParams = args;
  args[0] = &ms_copy;
  args[1] = &io_copy;
  switch (k) {
    case 0:
      p.func = (void *)k_multi_reset;
      p.gridDim = dim3((unsigned)std::max(1, (N + 2 + 255) / 256));
      // reset takes (int*, int): reuse the slots
      flag = N + 2;
      args[0] = &ms_copy.ctr;
      args[1] = &flag;
      break;
    case 1:
      p.func = (void *)k_multi_prep;
      p.gridDim = dim3((unsigned)N);
      flag = pass;
      args[2] = &flag;
      break;
    case 2:
      p.func = pass == 0 ? (void *)k_multi_fwd : (void *)k_multi_bwd;
      p.gridDim = dim3((unsigned)(pass == 0 ? grid_f : grid_b));
      p.blockDim = dim3(kMultiNT);
      p.sharedMemBytes = (unsigned)(pass == 0 ? lds_f : lds_b);
      break;
    default:
      p.func = pass == 0 ? (void *)k_multi_fwd_final : (void *)k_multi_bwd_final;
      p.gridDim = dim3((unsigned)N);
      break;
  }
}

hipError_t MultiRuntime::run(int pass, const MultiIO &io, hipStream_t s, SweepTimer *tm) {
  hipError_t e;
  int dev = 0;
  QTM_TRY(hipGetDevice(&dev));
  where = "multi handle used on a second device";
  if (device >= 0 && device != dev) return hipErrorInvalidDevice;
  device = dev;
  if (!uploaded && (e = upload())) return e;
  if (in.empty()) return hipSuccess;
  if (tm) {
    // eager launches, events around the persistent kernel
    for (int k = 0; k < 4; ++k) {
      hipKernelNodeParams p;
      void *args[3];
      MultiStatic msc;
      MultiIO ioc;
      int flag = 0;
      node_params(pass, k, io, p, args, msc, ioc, flag);
      if (k == 2) tm->before(pass, s);
      QTM_TRY(hipLaunchKernel(p.func, p.gridDim, p.blockDim, p.kernelParams, p.sharedMemBytes, s));
      if (k == 2) tm->after(pass, s);
    }
    return hipSuccess;
  }
  Graph &G = graph[pass];
  if (!G.built) {
    QTM_TRY(hipGraphCreate(&G.g, 0));
    for (int k = 0; k < 4; ++k) {
      hipKernelNodeParams p;
      void *args[3];
      MultiStatic msc;
      MultiIO ioc;
      int flag = 0;
      node_params(pass, k, io, p, args, msc, ioc, flag);
      QTM_TRY(hipGraphAddKernelNode(&G.node[k], G.g, k ? &G.node[k - 1] : nullptr, k ? 1 : 0, &p));
    }
    QTM_TRY(hipGraphInstantiate(&G.exec, G.g, nullptr, nullptr, 0));
    G.io = io;
    G.built = true;
  } else if (memcmp(&G.io, &io, sizeof(MultiIO)) != 0) {
    for (int k = 1; k < 4; ++k) {
      hipKernelNodeParams p;
      void *args[3];
      MultiStatic msc;
      MultiIO ioc;
      int flag = 0;
      node_params(pass, k, io, p, args, msc, ioc, flag);
      QTM_TRY(hipGraphExecKernelNodeSetParams(G.exec, G.node[k], &p));
    }
    G.io = io;
  }
  QTM_TRY(hipGraphLaunch(G.exec, s));
  return hipSuccess;
}

MultiRuntime *multi_runtime_create(const std::vector<MultiItemIn> &items, std::string &err) {
  MultiRuntime *m = new (std::nothrow) MultiRuntime();
  if (!m) {
    err = "out of host memory";
    return nullptr;
  }
  err = m->build(items);
  if (!err.empty()) {
    delete m;
    return nullptr;
  }
  return m;
}

void multi_runtime_destroy(MultiRuntime *m) { delete m; }

hipError_t multi_runtime_forward(MultiRuntime *m, const double *x, const double *w, double *out,
                                 void *state, hipStream_t s, SweepTimer *tm) {
  MultiIO io{x, w, nullptr, out, nullptr, nullptr, reinterpret_cast<Cx<float> *>(state)};
  return m->run(0, io, s, tm);
}

hipError_t multi_runtime_backward(MultiRuntime *m, const double *x, const double *w, const double *G,
                                  void *state, double *gw, double *gx, hipStream_t s, SweepTimer *tm) {
  MultiIO io{x, w, G, nullptr, gw, gx, reinterpret_cast<Cx<float> *>(state)};
  return m->run(1, io, s, tm);
}

const char *multi_runtime_where(const MultiRuntime *m) { return m->where; }

int multi_runtime_units(const MultiRuntime *m, int pass) {
  if (!m->uploaded) return -1;
  return pass == 0 ? m->sf.n_units : m->sb.n_units;
}

}  // namespace qtm
