// C ABI of libqtm (declared in include/qtm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "qtm.h"
#include "circuit.h"
#include "jit.h"
#include "k9.h"
#include "kernels.h"
#include "multi.h"
#include "tune.h"

using namespace qtm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const std::string &where) {
  g_err = where + ": " + hipGetErrorString(e);
  return QTM_ERR_HIP;
}

// Cap on one circuit handle's device workspace in bytes, from the
// environment variable QTM_MAX_WORKSPACE_BYTES (read whenever a workspace
// buffer has to grow); 0 = no cap.  Returns false for a value that is not a
// byte count.
bool workspace_cap(size_t *cap) {
  *cap = 0;
  const char *v = getenv("QTM_MAX_WORKSPACE_BYTES");
  if (!v || !*v) return true;
  char *end = nullptr;
  const unsigned long long x = strtoull(v, &end, 10);
  if (!end || *end != 0) return false;
  *cap = (size_t)x;
  return true;
}

// Grow-only device buffer; `total` (if set) counts the bytes of all buffers
// of the owning handle, which the cap above bounds.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t *total = nullptr;
  int ensure(size_t need) {
    if (need <= bytes) return QTM_OK;
    const size_t want = need < 256 ? 256 : need;
    size_t cap = 0;
    if (!workspace_cap(&cap)) return fail(QTM_ERR_WORKSPACE, "QTM_MAX_WORKSPACE_BYTES is not a byte count");
    const size_t others = total ? *total - bytes : 0;
    if (cap && others + want > cap)
      return fail(QTM_ERR_WORKSPACE, "workspace of " + std::to_string(others + want) +
                                         " bytes exceeds QTM_MAX_WORKSPACE_BYTES=" + std::to_string(cap));
    release();
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return fail(QTM_ERR_WORKSPACE, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    bytes = want;
    if (total) *total += want;
    return QTM_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    if (total) *total -= bytes;
    p = nullptr;
    bytes = 0;
  }
};

template <typename T>
int upload(T **dst, const std::vector<T> &src, std::vector<void *> &owned) {
  size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
  if (hipMalloc((void **)dst, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QTM_ERR_WORKSPACE, "device allocation failed");
  }
  owned.push_back(*dst);
  if (!src.empty()) {
    hipError_t e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  return QTM_OK;
}

struct StateTag {
  uint64_t circuit_id;
  int32_t batch, precision;
  uint64_t prep_gen;  // the circuit's prep_gen right after that forward
};
std::mutex g_reg_mu;
std::unordered_map<void *, StateTag> g_registry;
uint64_t g_next_id = 1;

// Events around sweep kernels (diagnostic timing, QTM_OPT_TIMING).
struct EventTimer : SweepTimer {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
  hipEvent_t cur = nullptr;
  hipError_t err = hipSuccess;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) err = r;
    return e;
  }
  void before(int kind, hipStream_t s) override {
    (void)kind;
    cur = get();
    if (cur) (void)hipEventRecord(cur, s);
  }
  void after(int kind, hipStream_t s) override {
    hipEvent_t e = get();
    if (e) (void)hipEventRecord(e, s);
    if (cur && e) pending[kind].push_back({cur, e});
    cur = nullptr;
  }
  ~EventTimer() override {
    for (auto &v : pending)
      for (auto &pr : v) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct qtm_circuit_s {
  uint64_t id = 0;
  CircuitDesc desc;
  HostCircuitInfo hinfo;
  int path = QTM_PATH_AUTO;
  int tile_qubits = 0;
  int low_qubits = 0;
  int renorm = 0;  // QTM_OPT_RENORM: rescale every `renorm` sweeps (0 = off)
  int device = -1;
  std::unique_ptr<EventTimer> timer;
  bool uploaded = false;
  DevCircuit dev;
  std::vector<void *> owned;
  // plans by (kt, klo, zero_skip): the specialised kernels skip all-zero
  // tiles and take plans chosen for that (QTM_OPT_JIT), the compiled ones not
  std::map<std::tuple<int, int, int>, DevPlan> plans;
  std::map<std::tuple<int, int, int>, HostPlan> hplans;
  int jit = 0;  // QTM_OPT_JIT
  int greedy_plan = 0;  // QTM_OPT_GREEDY_PLAN
  int plan_io = 12;     // QTM_OPT_PLAN_IO
  int jac_chunk = 0;    // QTM_OPT_JAC_CHUNK
  std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<JitSweeps>> jits;  // (kt, klo, precision, renorm, zero_skip)
  DevBuf cs, part, gocc, lam, state_ws, mats, coef, part_obs, part_grad, part_norm, part_pauli;
  DevBuf jac_state, jac_G, jac_gw, jac_out, jac_x, chk, rn;
  // shared-weight dense-block forward (QTM_OPT_DENSE_BLOCKS)
  int k9 = 0;
  K9Layout k9l;
  K9Dev k9d;
  DevBuf k9_tab, k9_rx, k9_part;
  size_t ws_total = 0;  // device workspace bytes of this handle
  int check_angles = 0;  // QTM_OPT_CHECK_ANGLES
  // The partial sums the last forward pass left for qtm_forward_norms:
  // [batch][rows][n_obs + 1] doubles with the squared norm in column n_obs.
  const double *norm_part = nullptr;
  int32_t norm_rows = 0, norm_B = 0;
  // What `mats` and `coef` hold: counted up by every forward (and by a
  // backward that prepares its own), with the fused plan, batch and
  // precision they were computed for (plan NULL: not by the fused path).
  uint64_t prep_gen = 0;
  const DevPlan *prep_plan = nullptr;
  int32_t prep_B = 0, prep_prec = -1;

  std::vector<DevBuf *> bufs() {
    return {&cs, &part, &gocc, &lam, &state_ws, &mats, &coef, &part_obs, &part_grad, &part_norm,
            &part_pauli, &jac_state, &jac_G, &jac_gw, &jac_out, &jac_x, &chk, &rn, &k9_tab, &k9_rx,
            &k9_part};
  }
  qtm_circuit_s() {
    for (DevBuf *b : bufs()) b->total = &ws_total;
  }
  ~qtm_circuit_s() {
    for (void *p : owned) (void)hipFree(p);
    for (DevBuf *b : bufs()) b->release();
  }
};

struct qtm_multi_s {
  std::vector<qtm_circuit_t> items;
  std::vector<int64_t> in_off, w_off, out_off, st_off;
  std::vector<int32_t> narrow;  // items run one by one: below 4 qubits, X / Y observables or
                                // controlled rotations
  MultiRuntime *rt = nullptr;   // every other item: persistent kernels
  std::unique_ptr<EventTimer> timer;
  ~qtm_multi_s() { multi_runtime_destroy(rt); }
};

namespace {

int ensure_device(qtm_circuit_t c) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (c->device >= 0 && c->device != dev)
    return fail(QTM_ERR_UNSUPPORTED, "circuit handle used on a second device");
  c->device = dev;
  if (c->uploaded) return QTM_OK;
  const CircuitDesc &d = c->desc;
  DevCircuit &g = c->dev;
  g.n = d.n;
  g.n_inputs = d.n_inputs;
  g.n_weights = d.n_weights;
  g.n_obs = (int)d.masks.size();
  g.n_occ = (int)d.occ_gate.size();
  std::vector<int32_t> src, idx, widx;
  for (int k : d.occ_gate) {
    src.push_back(d.gates[k].src);
    idx.push_back(d.gates[k].index);
    widx.push_back(d.gates[k].src == S_SCALED ? d.gates[k].q1 : 0);
  }
  const ParamCsr pc = param_csr(d);
  std::vector<int32_t> nd_idx;
  std::vector<uint64_t> nd_x, nd_z;
  for (size_t m = 0; m < d.pauli_x.size(); ++m)
    if (d.pauli_x[m]) {
      nd_idx.push_back((int32_t)m);
      nd_x.push_back(d.pauli_x[m]);
      nd_z.push_back(d.pauli_z[m]);
    }
  g.n_nd = (int)nd_idx.size();
  int rc;
  if ((rc = upload(&g.nd_idx, nd_idx, c->owned))) return rc;
  if ((rc = upload(&g.nd_x, nd_x, c->owned))) return rc;
  if ((rc = upload(&g.nd_z, nd_z, c->owned))) return rc;
  if ((rc = upload(&g.masks, d.masks, c->owned))) return rc;
  if ((rc = upload(&g.occ_src, src, c->owned))) return rc;
  if ((rc = upload(&g.occ_idx, idx, c->owned))) return rc;
  if ((rc = upload(&g.occ_widx, widx, c->owned))) return rc;
  if ((rc = upload(&g.w_ptr, pc.w_ptr, c->owned))) return rc;
  if ((rc = upload(&g.w_list, pc.w_list, c->owned))) return rc;
  if ((rc = upload(&g.w_fac, pc.w_fac, c->owned))) return rc;
  if ((rc = upload(&g.x_ptr, pc.x_ptr, c->owned))) return rc;
  if ((rc = upload(&g.x_list, pc.x_list, c->owned))) return rc;
  if ((rc = upload(&g.x_fac, pc.x_fac, c->owned))) return rc;
  c->uploaded = true;
  return QTM_OK;
}

// How the fused plans of this handle are chosen: 0 greedy, > 0 for kernels
// that skip all-zero tiles (the specialised ones) with that traffic weight,
// see QTM_OPT_GREEDY_PLAN and QTM_OPT_PLAN_IO.
int zero_skip_plan(const qtm_circuit_s *c) { return c->jit && !c->greedy_plan ? c->plan_io : 0; }

int default_kt(const qtm_circuit_s *c, int precision) {
  int kt = c->tile_qubits > 0 ? c->tile_qubits : (precision == QTM_C128 ? 11 : 12);
  kt = std::min(kt, kMaxTileQubits);
  kt = std::min(kt, c->desc.n);
  return std::max(kt, kMinTileQubits);
}

// Host plan for (kt, klo) of this precision (planned once, kept).
int get_host_plan(qtm_circuit_t c, int precision, const HostPlan **out) {
  if (c->desc.has_crot())
    return fail(QTM_ERR_UNSUPPORTED, "controlled rotations run on the per-gate path only");
  const int kt = default_kt(c, precision);
  const int klo = std::min(c->low_qubits > 0 ? c->low_qubits : 5, kt);
  const int zs = zero_skip_plan(c);
  auto key = std::make_tuple(kt, klo, zs);
  auto it = c->hplans.find(key);
  if (it == c->hplans.end()) {
    HostPlan hp;
    std::string why = build_host_plan(c->desc, kt, klo, hp, zs);
    if (!why.empty()) return fail(QTM_ERR_UNSUPPORTED, "internal planner error: " + why);
    it = c->hplans.emplace(key, std::move(hp)).first;
  }
  *out = &it->second;
  return QTM_OK;
}

int get_plan(qtm_circuit_t c, int precision, DevPlan **out) {
  const HostPlan *hpp = nullptr;
  int rc = get_host_plan(c, precision, &hpp);
  if (rc) return rc;
  const HostPlan &hp = *hpp;
  auto key = std::make_tuple(hp.kt, hp.klo, hp.zero_skip);
  auto it = c->plans.find(key);
  if (it != c->plans.end()) {
    *out = &it->second;
    return QTM_OK;
  }
  DevPlan dp;
  dp.kt = hp.kt;
  dp.klo = hp.klo;
  dp.n_blocks = hp.n_blocks;
  dp.n_gslots = hp.n_gslots;
  dp.max_gslots = hp.max_gslots;
  dp.n_sweeps = hp.n_sweeps;
  dp.sweep_off_fwd = hp.prog.sweep_off_fwd;
  dp.sweep_off_bwd = hp.prog.sweep_off_bwd;
  if ((rc = upload(&dp.code, hp.prog.code, c->owned))) return rc;
  if ((rc = upload(&dp.thr, hp.prog.thr, c->owned))) return rc;
  if ((rc = upload(&dp.blk, hp.blk, c->owned))) return rc;
  if ((rc = upload(&dp.blk_off, hp.blk_off, c->owned))) return rc;
  if ((rc = upload(&dp.occ_gslot, hp.occ_gslot, c->owned))) return rc;
  {
    std::vector<int32_t> ptr(std::max(hp.n_gslots, 0) + 1, 0), occ(hp.occ_gslot.size());
    for (int32_t g : hp.occ_gslot) ++ptr[g + 1];
    for (int g = 0; g < hp.n_gslots; ++g) ptr[g + 1] += ptr[g];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t k = 0; k < hp.occ_gslot.size(); ++k) occ[fill[hp.occ_gslot[k]]++] = (int32_t)k;
    if ((rc = upload(&dp.gs_ptr, ptr, c->owned))) return rc;
    if ((rc = upload(&dp.gs_occ, occ, c->owned))) return rc;
  }
  if ((rc = upload(&dp.obs_sgn_f, hp.obs_sgn, c->owned))) return rc;
  if ((rc = upload(&dp.seed_sgn, hp.seed_sgn, c->owned))) return rc;
  auto ins = c->plans.emplace(key, dp);
  *out = &ins.first->second;
  return QTM_OK;
}

JitSpec jit_spec(qtm_circuit_t c, int precision, const HostPlan &hp) {
  JitSpec sp;
  sp.n = c->desc.n;
  sp.kt = hp.kt;
  sp.dbl = precision == QTM_C128;
  sp.M = (int)c->desc.masks.size();
  sp.n_blocks = hp.n_blocks;
  sp.masks = c->desc.masks;
  sp.seed_add = c->desc.has_offdiag();
  sp.nwg_full = fused_wg_per_sample(sp.n, sp.kt);
  sp.renorm = c->renorm;
  sp.hp = &hp;
  return sp;
}

// Compile (once) the sweep kernels specialised for this circuit's plan at
// `precision`; with load, also load them on the current device.
int get_jit(qtm_circuit_t c, int precision, bool load, const JitSweeps **out) {
  *out = nullptr;
  const HostPlan *hp = nullptr;
  int rc = get_host_plan(c, precision, &hp);
  if (rc) return rc;
  const auto key = std::make_tuple(hp->kt, hp->klo, precision, c->renorm, hp->zero_skip);
  auto it = c->jits.find(key);
  if (it == c->jits.end()) {
    std::unique_ptr<JitSweeps> js(new JitSweeps());
    std::string err = jit_compile(jit_spec(c, precision, *hp), *js);
    if (!err.empty()) return fail(QTM_ERR_UNSUPPORTED, "specialised sweep kernels: " + err);
    it = c->jits.emplace(key, std::move(js)).first;
  }
  if (load) {
    hipError_t e = jit_load(*it->second);
    if (e != hipSuccess) return hip_fail(e, "loading the specialised sweep kernels");
  }
  *out = it->second.get();
  return QTM_OK;
}

bool use_fused(const qtm_circuit_s *c) {
  if (c->path == QTM_PATH_PLAIN) return false;
  return c->desc.n >= kMinTileQubits && !c->desc.has_crot();
}

int check_common(qtm_circuit_t c, int32_t batch, int32_t precision) {
  if (!c) return fail(QTM_ERR_INVALID_ARG, "NULL circuit");
  if (batch <= 0) return fail(QTM_ERR_INVALID_ARG, "batch must be >= 1");
  if (precision != QTM_C64 && precision != QTM_C128)
    return fail(QTM_ERR_INVALID_ARG, "precision must be QTM_C64 or QTM_C128");
  if (c->path == QTM_PATH_FUSED && c->desc.n < kMinTileQubits)
    return fail(QTM_ERR_UNSUPPORTED, "the fused path needs at least 4 qubits");
  if (c->path == QTM_PATH_FUSED && c->desc.has_crot())
    return fail(QTM_ERR_UNSUPPORTED, "controlled rotations run on the per-gate path only");
  size_t amps = (size_t)batch << c->desc.n;
  if (amps / (size_t)batch != ((size_t)1 << c->desc.n))
    return fail(QTM_ERR_INVALID_ARG, "batch too large");
  return QTM_OK;
}

size_t elem_bytes(int precision) { return precision == QTM_C128 ? 16 : 8; }

// Device buffers of one forward pass: the library's workspace (qtm_forward)
// or the no-allocation scratch array (qtm_forward_noalloc).
struct FwdBufs {
  void *mats = nullptr;         // fused: [B][n_blocks] gate matrices
  double *coef = nullptr;       // fused: [B][n_occ][3] derivative coefficients
  double *part_obs = nullptr;   // fused: observable partial sums
  double2 *cs = nullptr;        // per-gate: half-angle cosines and sines
  double *part = nullptr;       // per-gate: observable partial sums
  double *part_pauli = nullptr; // observables with X or Y factors
  double *rn = nullptr;         // fused, QTM_OPT_RENORM: the forward's norm records
};

// Byte sizes of those buffers for (B, plan); p = NULL on the per-gate path.
struct FwdSizes {
  size_t mats = 0, coef = 0, part_obs = 0, cs = 0, part = 0, part_pauli = 0, rn = 0;
};
FwdSizes fwd_sizes(const DevCircuit &d, const DevPlan *p, int32_t B, int renorm) {
  FwdSizes z;
  if (p) {
    z.mats = (size_t)B * std::max(p->n_blocks, 1) * sizeof(M2<double>);
    z.part_obs = fused_part_obs_doubles(d, *p, B) * sizeof(double);
    z.coef = (size_t)B * std::max(d.n_occ, 1) * 3 * sizeof(double);
    if (renorm) z.rn = fused_rn_doubles(d, *p, B) * sizeof(double);
  } else {
    z.cs = (size_t)B * std::max(d.n_occ, 1) * sizeof(double2);
    z.part = plain_part_doubles(d, B) * sizeof(double);
  }
  if (d.n_nd > 0) z.part_pauli = pauli_part_doubles(d, B) * sizeof(double);
  return z;
}

// The forward's launches: the sweeps (p != NULL; js = specialised kernels or
// NULL) or the per-gate kernels, with the diagonal observables, then the
// observables with X or Y factors (read from the stored final states).
hipError_t launch_forward(qtm_circuit_t c, const DevPlan *p, const JitSweeps *js, int32_t B, int32_t prec,
                          const double *x, const double *w, double *out, void *state, bool keep,
                          const FwdBufs &b, SweepTimer *tm, hipStream_t s) {
  const DevCircuit &d = c->dev;
  if (d.n_nd > 0) keep = true;
  hipError_t e;
  if (p) {
    Renorm rn;
    if (c->renorm) {
      rn.period = c->renorm;
      rn.fwd = b.rn;
    }
    e = prec == QTM_C64
            ? fused_forward<float>(d, *p, B, x, w, b.mats, b.coef, state, b.part_obs, out, keep, s, tm, js, rn)
            : fused_forward<double>(d, *p, B, x, w, b.mats, b.coef, state, b.part_obs, out, keep, s, tm, js, rn);
  } else {
    e = launch_half_angles(d, B, x, w, b.cs, s);
    if (e == hipSuccess)
      e = prec == QTM_C64 ? plain_forward<float>(d, c->hinfo, B, b.cs, state, b.part, out, false, s)
                          : plain_forward<double>(d, c->hinfo, B, b.cs, state, b.part, out, false, s);
  }
  if (e != hipSuccess) return e;
  return prec == QTM_C64 ? launch_pauli_expval<float>(d, B, state, b.part_pauli, out, s)
                         : launch_pauli_expval<double>(d, B, state, b.part_pauli, out, s);
}

// The shared-weight dense-block forward (complex64): uploads the slot
// tables once, sizes its workspace, runs k9_forward.
int k9_run(qtm_circuit_t c, int32_t B, const double *x, const double *w, double *out, void *state,
           hipStream_t s) {
  const DevCircuit &d = c->dev;
  int rc;
  if (c->k9d.n == 0) {
    int32_t *rx = nullptr, *ry = nullptr, *rz = nullptr;
    if ((rc = upload(&rx, c->k9l.rx, c->owned)) || (rc = upload(&ry, c->k9l.ry, c->owned)) ||
        (rc = upload(&rz, c->k9l.rz, c->owned)))
      return rc;
    c->k9d.rx = rx;
    c->k9d.ry = ry;
    c->k9d.rz = rz;
    c->k9d.L = c->k9l.L;
    c->k9d.n = c->k9l.n;
  }
  const int rows = k9_part_rows(c->k9l);
  if ((rc = c->k9_tab.ensure(k9_tab_floats(c->k9l) * sizeof(float))) ||
      (rc = c->k9_rx.ensure((size_t)B * c->k9l.L * c->k9l.n * sizeof(float2))) ||
      (rc = c->k9_part.ensure((size_t)B * rows * (d.n_obs + 1) * sizeof(double))))
    return rc;
  c->prep_gen++;
  c->prep_plan = nullptr;
  c->norm_part = nullptr;
  hipError_t e = k9_forward(c->k9d, d, B, x, w, state, (float *)c->k9_tab.p, (float2 *)c->k9_rx.p,
                            (double *)c->k9_part.p, out, s, c->timer.get());
  if (e != hipSuccess) return hip_fail(e, "dense-block forward launch");
  c->norm_part = (const double *)c->k9_part.p;
  c->norm_rows = rows;
  c->norm_B = B;
  return QTM_OK;
}

// Forward pass on the library's workspace.
int do_forward(qtm_circuit_t c, int32_t B, int32_t prec, const double *x, const double *w,
               double *out, void *state, bool keep, hipStream_t s) {
  const DevCircuit &d = c->dev;
  int rc;
  if (c->k9 && prec == QTM_C64 && use_fused(c)) return k9_run(c, B, x, w, out, state, s);
  DevPlan *p = nullptr;
  const JitSweeps *js = nullptr;
  if (use_fused(c)) {
    if ((rc = get_plan(c, prec, &p))) return rc;
    if (c->jit && (rc = get_jit(c, prec, true, &js))) return rc;
  }
  const FwdSizes z = fwd_sizes(d, p, B, c->renorm);
  FwdBufs b;
  if (p) {
    // the derivative coefficients too, so that the backward can reuse both
    if ((rc = c->mats.ensure(z.mats)) || (rc = c->part_obs.ensure(z.part_obs)) || (rc = c->coef.ensure(z.coef)))
      return rc;
    b.mats = c->mats.p;
    b.coef = (double *)c->coef.p;
    b.part_obs = (double *)c->part_obs.p;
    if (z.rn) {
      // the forward's records, then the backward's (fused_rn_doubles)
      if ((rc = c->rn.ensure(z.rn))) return rc;
      b.rn = (double *)c->rn.p;
    }
  } else {
    if ((rc = c->cs.ensure(z.cs)) || (rc = c->part.ensure(z.part))) return rc;
    b.cs = (double2 *)c->cs.p;
    b.part = (double *)c->part.p;
  }
  if (z.part_pauli) {
    if ((rc = c->part_pauli.ensure(z.part_pauli))) return rc;
    b.part_pauli = (double *)c->part_pauli.p;
  }
  c->prep_gen++;
  c->prep_plan = nullptr;
  c->norm_part = nullptr;
  hipError_t e = launch_forward(c, p, js, B, prec, x, w, out, state, keep, b, c->timer.get(), s);
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  if (p) {
    c->prep_plan = p;
    c->prep_B = B;
    c->prep_prec = prec;
  }
  c->norm_part = p ? b.part_obs : b.part;
  c->norm_rows = p ? fused_wg_per_sample(d.n, p->kt) : plain_norm_rows(d.n, B);
  c->norm_B = B;
  return QTM_OK;
}

// With QTM_OPT_CHECK_ANGLES: every input and weight must be finite.  Runs a
// check kernel on the stream, copies its result to the host and waits.
int check_angles(qtm_circuit_t c, int32_t B, const double *x, const double *w, hipStream_t s) {
  if (!c->check_angles) return QTM_OK;
  const int64_t nx = x ? (int64_t)B * c->desc.n_inputs : 0, nw = w ? c->desc.n_weights : 0;
  int rc = c->chk.ensure(sizeof(unsigned long long));
  if (rc) return rc;
  unsigned long long first = 0;
  hipError_t e = launch_first_nonfinite(x, nx, w, nw, (unsigned long long *)c->chk.p, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&first, c->chk.p, sizeof first, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "angle check");
  if (first == ~0ull) return QTM_OK;
  if ((int64_t)first < nx)
    return fail(QTM_ERR_INVALID_ARG, "non-finite angle source: inputs[" +
                                         std::to_string(first / c->desc.n_inputs) + "][" +
                                         std::to_string(first % c->desc.n_inputs) + "]");
  return fail(QTM_ERR_INVALID_ARG, "non-finite angle source: weights[" + std::to_string(first - nx) + "]");
}

// Adjoint backward from the final states in psi (consumed).  Leaves the
// per-sample, per-rotation derivatives in c->gocc.
// prepped: no forward has run on c since the one that filled psi, so mats
// and coef may still hold its matrices (checked against the plan, batch and
// precision here).
// psi_in: the final states, if not in psi (the fused path reads them there
// and leaves psi overwritten; the per-gate path works in psi, so they are
// copied there first)
int run_backward(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                 const double *weights, const double *grad_expvals, void *psi, const void *psi_in,
                 double *grad_weights, double *grad_inputs, bool prepped, hipStream_t s) {
  const DevCircuit &d = c->dev;
  const size_t sbytes = ((size_t)batch << c->desc.n) * elem_bytes(precision);
  int rc;
  if ((rc = c->lam.ensure(sbytes))) return rc;
  if ((rc = c->gocc.ensure((size_t)batch * std::max(std::max(d.n_occ, d.n_obs), 1) * sizeof(double))))
    return rc;
  hipError_t e;
  if (use_fused(c)) {
    DevPlan *p = nullptr;
    if ((rc = get_plan(c, precision, &p))) return rc;
    if ((rc = c->mats.ensure((size_t)batch * std::max(p->n_blocks, 1) * sizeof(M2<double>)))) return rc;
    if ((rc = c->coef.ensure((size_t)batch * std::max(d.n_occ, 1) * 3 * sizeof(double)))) return rc;
    if ((rc = c->part_grad.ensure(fused_part_grad_doubles(d, *p, batch) * sizeof(double)))) return rc;
    const JitSweeps *js = nullptr;
    if (c->jit && (rc = get_jit(c, precision, true, &js))) return rc;
    if ((rc = c->part_norm.ensure((size_t)batch * fused_wg_per_sample(d.n, p->kt) * sizeof(double))))
      return rc;
    const bool reuse = prepped && c->prep_plan == p && c->prep_B == batch && c->prep_prec == precision;
    if (!reuse) {
      // this backward prepares mats and coef itself
      c->prep_gen++;
      c->prep_plan = p;
      c->prep_B = batch;
      c->prep_prec = precision;
    }
    Renorm rn;
    if (c->renorm) {
      const size_t nrn = fused_rn_doubles(d, *p, batch);
      if ((rc = c->rn.ensure(nrn * sizeof(double)))) return rc;
      rn.period = c->renorm;
      rn.bwd = (double *)c->rn.p + nrn / 5;  // after the forward's records
    }
    e = precision == QTM_C64
            ? fused_backward<float>(d, *p, batch, inputs, weights, grad_expvals, c->mats.p,
                                    (double *)c->coef.p, reuse, psi, psi_in, c->lam.p, (double *)c->part_grad.p,
                                    (double *)c->part_norm.p, (double *)c->gocc.p, grad_weights,
                                    grad_inputs, s, c->timer.get(), js, rn)
            : fused_backward<double>(d, *p, batch, inputs, weights, grad_expvals, c->mats.p,
                                     (double *)c->coef.p, reuse, psi, psi_in, c->lam.p, (double *)c->part_grad.p,
                                     (double *)c->part_norm.p, (double *)c->gocc.p, grad_weights,
                                     grad_inputs, s, c->timer.get(), js, rn);
  } else {
    if ((rc = c->cs.ensure((size_t)batch * std::max(d.n_occ, 1) * sizeof(double2)))) return rc;
    if ((rc = c->part.ensure(plain_part_doubles(d, batch) * sizeof(double)))) return rc;
    if (psi_in && (e = hipMemcpyAsync(psi, psi_in, sbytes, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return hip_fail(e, "state copy");
    // the per-gate backward reuses the forward's partial-sum buffer
    c->norm_part = nullptr;
    e = launch_half_angles(d, batch, inputs, weights, (double2 *)c->cs.p, s);
    if (e == hipSuccess)
      e = precision == QTM_C64
              ? plain_backward<float>(d, c->hinfo, batch, (double2 *)c->cs.p, inputs, weights, psi, c->lam.p,
                                      grad_expvals, (double *)c->part.p, (double *)c->gocc.p,
                                      grad_weights, grad_inputs, s)
              : plain_backward<double>(d, c->hinfo, batch, (double2 *)c->cs.p, inputs, weights, psi, c->lam.p,
                                       grad_expvals, (double *)c->part.p, (double *)c->gocc.p,
                                       grad_weights, grad_inputs, s);
  }
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return QTM_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the no-allocation forward: one array per GPU, in the library's
// code object, held until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device (with that device current).
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(QTM_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(QTM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return QTM_OK;
}

}  // namespace

extern "C" {

const char *qtm_last_error(void) { return g_err.c_str(); }

const char *qtm_version(void) { return "qtm 0.1 (gfx950)"; }

int qtm_circuit_create(int32_t n_qubits, const qtm_gate *gates, int32_t n_gates, int32_t n_inputs,
                       int32_t n_weights, const uint64_t *obs_zmask, int32_t n_obs,
                       qtm_circuit_t *out) {
  return qtm_circuit_create_pauli(n_qubits, gates, n_gates, n_inputs, n_weights, nullptr, obs_zmask,
                                  n_obs, out);
}

int qtm_circuit_create_pauli(int32_t n_qubits, const qtm_gate *gates, int32_t n_gates,
                             int32_t n_inputs, int32_t n_weights, const uint64_t *obs_xmask,
                             const uint64_t *obs_zmask, int32_t n_obs, qtm_circuit_t *out) {
  if (!out) return fail(QTM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::unique_ptr<qtm_circuit_s> c(new (std::nothrow) qtm_circuit_s());
  if (!c) return fail(QTM_ERR_WORKSPACE, "out of host memory");
  std::string err;
  int rc = validate_and_build(n_qubits, reinterpret_cast<const Gate *>(gates), n_gates, n_inputs,
                              n_weights, obs_zmask, obs_xmask, n_obs, c->desc, err);
  if (rc) return fail(rc, err);
  c->hinfo.gates = c->desc.gates;
  c->hinfo.gate_occ = c->desc.gate_occ;
  {
    std::lock_guard<std::mutex> g(g_reg_mu);
    c->id = g_next_id++;
  }
  *out = c.release();
  return QTM_OK;
}

int qtm_circuit_destroy(qtm_circuit_t c) {
  if (!c) return QTM_OK;
  {
    std::lock_guard<std::mutex> g(g_reg_mu);
    for (auto it = g_registry.begin(); it != g_registry.end();)
      it = it->second.circuit_id == c->id ? g_registry.erase(it) : std::next(it);
  }
  delete c;
  return QTM_OK;
}

int qtm_set_option(qtm_circuit_t c, int32_t option, int64_t value) {
  if (!c) return fail(QTM_ERR_INVALID_ARG, "NULL circuit");
  switch (option) {
    case QTM_OPT_PATH:
      if (value < QTM_PATH_AUTO || value > QTM_PATH_FUSED) return fail(QTM_ERR_INVALID_ARG, "bad path");
      c->path = (int)value;
      return QTM_OK;
    case QTM_OPT_TILE_QUBITS:
      if (value != 0 && (value < kMinTileQubits || value > kMaxTileQubits))
        return fail(QTM_ERR_INVALID_ARG, "tile qubits must be 0 or 4..12");
      c->tile_qubits = (int)value;
      return QTM_OK;
    case QTM_OPT_LOW_QUBITS:
      if (value < 0 || value > kMaxTileQubits) return fail(QTM_ERR_INVALID_ARG, "low qubits must be 0..12");
      c->low_qubits = (int)value;
      return QTM_OK;
    case QTM_OPT_RENORM:
      if (value < 0 || value > 1024) return fail(QTM_ERR_INVALID_ARG, "renormalisation period must be 0..1024");
      c->renorm = (int)value;
      return QTM_OK;
    case QTM_OPT_TIMING:
      if (value && !c->timer) c->timer.reset(new EventTimer());
      if (!value) c->timer.reset();
      return QTM_OK;
    case QTM_OPT_JIT:
      c->jit = value ? 1 : 0;
      return QTM_OK;
    case QTM_OPT_GREEDY_PLAN:
      c->greedy_plan = value ? 1 : 0;
      return QTM_OK;
    case QTM_OPT_PLAN_IO:
      if (value < 1 || value > 64) return fail(QTM_ERR_INVALID_ARG, "QTM_OPT_PLAN_IO must be in 1..64");
      c->plan_io = (int)value;
      return QTM_OK;
    case QTM_OPT_JAC_CHUNK:
      if (value < 0 || value > 65535) return fail(QTM_ERR_INVALID_ARG, "QTM_OPT_JAC_CHUNK must be in 0..65535");
      c->jac_chunk = (int)value;
      return QTM_OK;
    case QTM_OPT_CHECK_ANGLES:
      c->check_angles = value ? 1 : 0;
      return QTM_OK;
    case QTM_OPT_DENSE_BLOCKS:
      if (value) {
        std::string why;
        K9Layout k;
        if (!k9_detect(c->desc, k, why)) return fail(QTM_ERR_UNSUPPORTED, "dense blocks: " + why);
        if (c->desc.has_offdiag()) return fail(QTM_ERR_UNSUPPORTED, "dense blocks: Z-string observables only");
        if (c->k9d.n == 0) c->k9l = std::move(k);
      }
      c->k9 = value ? 1 : 0;
      return QTM_OK;
    default:
      return fail(QTM_ERR_UNSUPPORTED, "unknown option");
  }
}

int qtm_state_bytes(qtm_circuit_t c, int32_t batch, int32_t precision, size_t *bytes) {
  int rc = check_common(c, batch, precision);
  if (rc) return rc;
  if (!bytes) return fail(QTM_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = ((size_t)batch << c->desc.n) * elem_bytes(precision);
  return QTM_OK;
}

int qtm_forward(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                const double *weights, double *expvals, void *state, void *stream) {
  int rc = check_common(c, batch, precision);
  if (rc) return rc;
  if (!expvals) return fail(QTM_ERR_INVALID_ARG, "expvals is NULL");
  if (c->desc.n_inputs > 0 && !inputs) return fail(QTM_ERR_INVALID_ARG, "inputs is NULL");
  if (c->desc.n_weights > 0 && !weights) return fail(QTM_ERR_INVALID_ARG, "weights is NULL");
  if ((rc = ensure_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_angles(c, batch, inputs, weights, s))) return rc;
  const size_t sbytes = ((size_t)batch << c->desc.n) * elem_bytes(precision);
  void *st = state;
  if (!st) {
    if ((rc = c->state_ws.ensure(sbytes))) return rc;
    st = c->state_ws.p;
  }
  rc = do_forward(c, batch, precision, inputs, weights, expvals, st, state != nullptr, s);
  if (rc) return rc;
  if (state) {
    std::lock_guard<std::mutex> g(g_reg_mu);
    g_registry[state] = StateTag{c->id, batch, precision, c->prep_gen};
  }
  return QTM_OK;
}

int qtm_forward_noalloc(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                        const double *weights, double *expvals, void *state, void *stream) {
  int rc = check_common(c, batch, precision);
  if (rc) return rc;
  if (!expvals || !state) return fail(QTM_ERR_INVALID_ARG, "expvals and state are required");
  if (c->desc.n_inputs > 0 && !inputs) return fail(QTM_ERR_INVALID_ARG, "inputs is NULL");
  if (c->desc.n_weights > 0 && !weights) return fail(QTM_ERR_INVALID_ARG, "weights is NULL");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (c->k9 && precision == QTM_C64 && use_fused(c))
    return fail(QTM_ERR_UNSUPPORTED, "qtm_forward_noalloc does not run the dense-block forward");
  // the circuit's constant tables and plan must already be on this device
  if (!c->uploaded || c->device != dev)
    return fail(QTM_ERR_STATE, "the circuit's tables are not on this device: call qtm_forward once first");
  const DevCircuit &d = c->dev;
  const DevPlan *p = nullptr;
  const JitSweeps *js = nullptr;
  if (use_fused(c)) {
    // the plan key as get_host_plan forms it; nothing is planned here
    const int kt = default_kt(c, precision);
    const int klo = std::min(c->low_qubits > 0 ? c->low_qubits : 5, kt);
    const int zs = zero_skip_plan(c);
    auto it = c->plans.find(std::make_tuple(kt, klo, zs));
    if (it == c->plans.end())
      return fail(QTM_ERR_STATE, "the circuit's plan for this tile configuration is not on the device: "
                                 "call qtm_forward once first");
    p = &it->second;
    // specialised kernels only if already compiled and loaded here; else the compiled ones
    if (c->jit) {
      auto jt = c->jits.find(std::make_tuple(kt, klo, (int)precision, c->renorm, zs));
      if (jt != c->jits.end() && jt->second->loaded && jt->second->device == dev) js = jt->second.get();
    }
  }
  const FwdSizes z = fwd_sizes(d, p, batch, c->renorm);
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t need =
      up(z.mats) + up(z.coef) + up(z.part_obs) + up(z.cs) + up(z.part) + up(z.part_pauli) + up(z.rn);
  if (need > kScratchBytes)
    return fail(QTM_ERR_WORKSPACE, "qtm_forward_noalloc needs " + std::to_string(need) +
                                       " bytes of scratch for this batch; the maximum is " +
                                       std::to_string(kScratchBytes));
  void *base = nullptr;
  if ((rc = scratch_address(dev, &base))) return rc;
  unsigned char *q = (unsigned char *)base;
  FwdBufs b;
  b.mats = z.mats ? q : nullptr;
  q += up(z.mats);
  b.coef = z.coef ? (double *)q : nullptr;
  q += up(z.coef);
  b.part_obs = z.part_obs ? (double *)q : nullptr;
  q += up(z.part_obs);
  b.cs = z.cs ? (double2 *)q : nullptr;
  q += up(z.cs);
  b.part = z.part ? (double *)q : nullptr;
  q += up(z.part);
  b.part_pauli = z.part_pauli ? (double *)q : nullptr;
  q += up(z.part_pauli);
  b.rn = z.rn ? (double *)q : nullptr;
  // the library's matrices (a backward may reuse them) and the norm partials
  // are not this pass's; a state tag of this buffer no longer describes it
  c->prep_gen++;
  c->prep_plan = nullptr;
  c->norm_part = nullptr;
  {
    std::lock_guard<std::mutex> g(g_reg_mu);
    g_registry.erase(state);
  }
  e = launch_forward(c, p, js, batch, precision, inputs, weights, expvals, state, true, b, nullptr,
                     (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "no-allocation forward launch");
  return QTM_OK;
}

int qtm_backward(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                 const double *weights, const double *grad_expvals, void *state,
                 double *grad_weights, double *grad_inputs, void *stream) {
  int rc = check_common(c, batch, precision);
  if (rc) return rc;
  if (!grad_expvals) return fail(QTM_ERR_INVALID_ARG, "grad_expvals is NULL");
  if (c->desc.n_weights > 0 && !grad_weights) return fail(QTM_ERR_INVALID_ARG, "grad_weights is NULL");
  if (c->desc.n_inputs > 0 && !inputs) return fail(QTM_ERR_INVALID_ARG, "inputs is NULL");
  if (c->desc.n_weights > 0 && !weights) return fail(QTM_ERR_INVALID_ARG, "weights is NULL");
  if ((rc = ensure_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_angles(c, batch, inputs, weights, s))) return rc;
  const DevCircuit &d = c->dev;
  const size_t sbytes = ((size_t)batch << c->desc.n) * elem_bytes(precision);
  void *psi = state;
  bool prepped = true;
  if (state) {
    std::lock_guard<std::mutex> g(g_reg_mu);
    auto it = g_registry.find(state);
    if (it == g_registry.end() || it->second.circuit_id != c->id || it->second.batch != batch ||
        it->second.precision != precision)
      return fail(QTM_ERR_STATE, "state buffer was not filled by qtm_forward for this circuit, batch and precision");
    prepped = it->second.prep_gen == c->prep_gen;
    g_registry.erase(it);
  } else {
    // recompute the forward into the workspace (expectation values go to a scratch area)
    if ((rc = c->state_ws.ensure(sbytes))) return rc;
    psi = c->state_ws.p;
    if ((rc = c->gocc.ensure((size_t)batch * std::max(std::max(d.n_occ, d.n_obs), 1) * sizeof(double))))
      return rc;
    if ((rc = do_forward(c, batch, precision, inputs, weights, (double *)c->gocc.p, psi, true, s)))
      return rc;
  }
  return run_backward(c, batch, precision, inputs, weights, grad_expvals, psi, nullptr, grad_weights,
                      grad_inputs, prepped, s);
}

namespace {
// Observables per adjoint pass of qtm_jacobian: QTM_OPT_JAC_CHUNK, else as
// many as keep one pass's repeated final states within kJacPassBytes (at
// least one); the rows of a pass stay within a grid dimension.  A batch
// whose states alone exceed that fills the GPU in a pass of its own, and
// repeating its states would only add copies (n = 20, batch 64: 36.8 ms with
// one observable per pass, 39.9 ms with two); small batches gain (n = 12,
// batch 48, 32 observables: 0.24 ms in one pass, 1.43 ms in 32).
constexpr size_t kJacPassBytes = (size_t)64 << 20;
int jacobian_chunk(const qtm_circuit_s *c, int32_t batch, size_t sbytes) {
  const int M = c->dev.n_obs;
  int64_t k = c->jac_chunk > 0 ? c->jac_chunk : (int64_t)(kJacPassBytes / std::max<size_t>(sbytes, 1));
  k = std::min<int64_t>(k, 65535 / batch);
  return (int)std::max<int64_t>(1, std::min<int64_t>(k, M));
}
}  // namespace

int qtm_jacobian(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                 const double *weights, double *expvals, double *jac_weights, double *jac_inputs,
                 void *stream) {
  int rc = check_common(c, batch, precision);
  if (rc) return rc;
  const CircuitDesc &cd = c->desc;
  if (cd.n_weights > 0 && !jac_weights) return fail(QTM_ERR_INVALID_ARG, "jac_weights is NULL");
  if (cd.n_inputs > 0 && !inputs) return fail(QTM_ERR_INVALID_ARG, "inputs is NULL");
  if (cd.n_weights > 0 && !weights) return fail(QTM_ERR_INVALID_ARG, "weights is NULL");
  if ((rc = ensure_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_angles(c, batch, inputs, weights, s))) return rc;
  const DevCircuit &d = c->dev;
  const int M = d.n_obs;
  const size_t sbytes = ((size_t)batch << cd.n) * elem_bytes(precision);
  const int k = jacobian_chunk(c, batch, sbytes);
  const size_t xbytes = (size_t)batch * cd.n_inputs * sizeof(double);
  if ((rc = c->state_ws.ensure(sbytes * k)) || (rc = c->jac_state.ensure(sbytes)) ||
      (rc = c->jac_G.ensure((size_t)batch * k * M * sizeof(double))) ||
      (rc = c->jac_gw.ensure((size_t)std::max(cd.n_weights, 1) * sizeof(double))) ||
      (rc = c->jac_out.ensure((size_t)batch * M * sizeof(double))) ||
      (k > 1 && xbytes > 0 && (rc = c->jac_x.ensure(xbytes * k))))
    return rc;
  double *out = expvals ? expvals : (double *)c->jac_out.p;
  // the forward leaves the final states in jac_state
  if ((rc = do_forward(c, batch, precision, inputs, weights, out, c->jac_state.p, true, s))) return rc;
  hipError_t e;
  for (int m0 = 0; m0 < M; m0 += k) {
    const int kk = std::min(k, M - m0), rows = kk * batch;
    if ((e = launch_onehot((double *)c->jac_G.p, rows, batch, M, m0, s))) return hip_fail(e, "jacobian seed");
    if (kk == 1) {
      // one observable: the pass reads the final states in jac_state and
      // works in state_ws (nothing copied)
      if ((rc = run_backward(c, batch, precision, inputs, weights, (double *)c->jac_G.p, c->state_ws.p,
                             c->jac_state.p, (double *)c->jac_gw.p, nullptr, true, s)))
        return rc;
    } else {
      // kk observables in one pass over kk x batch rows: the final states and
      // the input rows repeated kk times (row r is sample r mod batch); the
      // pass prepares its own gate matrices for the repeated rows
      if ((e = launch_replicate(c->state_ws.p, c->jac_state.p, sbytes, kk, s)))
        return hip_fail(e, "jacobian state copies");
      const double *xr = nullptr;
      if (xbytes > 0) {
        if ((e = launch_replicate(c->jac_x.p, inputs, xbytes, kk, s))) return hip_fail(e, "jacobian input copies");
        xr = (const double *)c->jac_x.p;
      }
      if ((rc = run_backward(c, rows, precision, xr, weights, (double *)c->jac_G.p, c->state_ws.p, nullptr,
                             (double *)c->jac_gw.p, nullptr, false, s)))
        return rc;
    }
    if ((e = launch_scatter_jac(d, rows, batch, (double *)c->gocc.p, inputs, weights, m0, jac_weights,
                                jac_inputs, s)))
      return hip_fail(e, "jacobian scatter");
  }
  return QTM_OK;
}

namespace {
int read_timer(EventTimer *tp, int32_t kind, double *total_ms, int64_t *launches) {
  *total_ms = 0.0;
  *launches = 0;
  if (!tp) return fail(QTM_ERR_INVALID_ARG, "timing is not enabled (QTM_OPT_TIMING)");
  EventTimer &t = *tp;
  if (t.err != hipSuccess) return hip_fail(t.err, "hipEventCreate");
  for (auto &pr : t.pending[kind]) {
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    *total_ms += ms;
    *launches += 1;
    t.pool.push_back(pr.first);
    t.pool.push_back(pr.second);
  }
  t.pending[kind].clear();
  return QTM_OK;
}
}  // namespace

int qtm_timing_read(qtm_circuit_t c, int32_t kind, double *total_ms, int64_t *launches) {
  if (!c || kind < 0 || kind > 1 || !total_ms || !launches)
    return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  return read_timer(c->timer.get(), kind, total_ms, launches);
}

int qtm_forward_norms(qtm_circuit_t c, int32_t batch, double *norms, void *stream) {
  if (!c || !norms) return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  if (!c->norm_part || c->norm_B != batch)
    return fail(QTM_ERR_STATE, "no forward pass with this batch has run on the circuit");
  hipError_t e = launch_norms(c->norm_part, batch, c->norm_rows, c->dev.n_obs, norms, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "norms launch");
  return QTM_OK;
}

// Diagnostics: JSON description of the fused plan for (precision) into buf.
int qtm_plan_json(qtm_circuit_t c, int32_t precision, char *buf, size_t len, size_t *needed) {
  if (!c) return fail(QTM_ERR_INVALID_ARG, "NULL circuit");
  if (c->desc.n < kMinTileQubits) return fail(QTM_ERR_UNSUPPORTED, "no fused plan below 4 qubits");
  if (c->desc.has_crot())
    return fail(QTM_ERR_UNSUPPORTED, "controlled rotations run on the per-gate path only");
  const int kt = default_kt(c, precision);
  const int klo = std::min(c->low_qubits > 0 ? c->low_qubits : 5, kt);
  Plan plan = make_plan(c->desc, kt, klo, zero_skip_plan(c));
  std::string why = check_plan(c->desc, plan);
  std::string js = plan_json(c->desc, plan);
  if (!why.empty()) {
    js = "{\"error\":\"" + why + "\"}";
  } else {
    // append the encoded device program (for layout checks)
    Program prog = encode_program(c->desc, plan);
    std::string extra = ",\"code\":[";
    for (size_t i = 0; i < prog.code.size(); ++i) extra += (i ? "," : "") + std::to_string(prog.code[i]);
    extra += "],\"thr\":[";
    for (size_t i = 0; i < prog.thr.size(); ++i) extra += (i ? "," : "") + std::to_string(prog.thr[i]);
    extra += "],\"sweep_off_fwd\":[";
    for (size_t i = 0; i < prog.sweep_off_fwd.size(); ++i)
      extra += (i ? "," : "") + std::to_string(prog.sweep_off_fwd[i]);
    extra += "],\"sweep_off_bwd\":[";
    for (size_t i = 0; i < prog.sweep_off_bwd.size(); ++i)
      extra += (i ? "," : "") + std::to_string(prog.sweep_off_bwd[i]);
    extra += "],\"excited\":[";
    for (size_t i = 0; i < prog.excited.size(); ++i) extra += (i ? "," : "") + std::to_string(prog.excited[i]);
    extra += "]}";
    js.pop_back();
    js += extra;
  }
  if (needed) *needed = js.size() + 1;
  if (buf && len > 0) {
    size_t k = std::min(len - 1, js.size());
    memcpy(buf, js.data(), k);
    buf[k] = 0;
  }
  return why.empty() ? QTM_OK : fail(QTM_ERR_UNSUPPORTED, why);
}

// Diagnostics: source of a specialised sweep kernel.
int qtm_jit_source(qtm_circuit_t c, int32_t precision, int32_t dir, int32_t sweep, char *buf, size_t len,
                   size_t *needed) {
  if (!c || (precision != QTM_C64 && precision != QTM_C128) || dir < 0 || dir > 1)
    return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  if (c->desc.n < kMinTileQubits) return fail(QTM_ERR_UNSUPPORTED, "no fused plan below 4 qubits");
  const HostPlan *hp = nullptr;
  int rc = get_host_plan(c, precision, &hp);
  if (rc) return rc;
  if (sweep < 0 || sweep >= hp->n_sweeps) return fail(QTM_ERR_INVALID_ARG, "sweep out of range");
  const std::string src = jit_source(jit_spec(c, precision, *hp), dir, sweep);
  if (needed) *needed = src.size() + 1;
  if (buf && len > 0) {
    size_t k = std::min(len - 1, src.size());
    memcpy(buf, src.data(), k);
    buf[k] = 0;
  }
  return QTM_OK;
}

// Compile the specialised sweep kernels of a circuit (no device needed).
int qtm_jit_compile(qtm_circuit_t c, int32_t precision) {
  if (!c || (precision != QTM_C64 && precision != QTM_C128)) return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  if (c->desc.n < kMinTileQubits) return fail(QTM_ERR_UNSUPPORTED, "no fused plan below 4 qubits");
  const JitSweeps *js = nullptr;
  return get_jit(c, precision, false, &js);
}

// Diagnostics: registers and scratch bytes of a loaded specialised kernel.
int qtm_jit_info(qtm_circuit_t c, int32_t precision, int32_t dir, int32_t sweep, int32_t *vgprs,
                 int32_t *scratch) {
  if (!c || (precision != QTM_C64 && precision != QTM_C128) || dir < 0 || dir > 1 || !vgprs || !scratch)
    return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  const HostPlan *hp = nullptr;
  int rc = get_host_plan(c, precision, &hp);
  if (rc) return rc;
  auto it = c->jits.find(std::make_tuple(hp->kt, hp->klo, (int)precision, c->renorm, hp->zero_skip));
  if (it == c->jits.end() || !it->second->loaded) return fail(QTM_ERR_INVALID_ARG, "specialised kernels not loaded");
  if (sweep < 0 || sweep >= (int)it->second->k[dir].size()) return fail(QTM_ERR_INVALID_ARG, "sweep out of range");
  *vgprs = it->second->k[dir][sweep].vgprs;
  *scratch = it->second->k[dir][sweep].scratch;
  return QTM_OK;
}

int qtm_autotune(qtm_circuit_t c, int32_t batch, int32_t precision, void *stream, int32_t flags, char *report,
                 size_t len, size_t *needed) {
  int rc = check_common(c, batch, precision);
  if (rc) return rc;
  if (c->desc.n < kMinTileQubits) return fail(QTM_ERR_UNSUPPORTED, "no fused path below 4 qubits");
  if (c->desc.has_crot())
    return fail(QTM_ERR_UNSUPPORTED, "controlled rotations run on the per-gate path only");
  TuneInfo info;
  info.n = c->desc.n;
  info.n_inputs = c->desc.n_inputs;
  info.n_weights = c->desc.n_weights;
  info.n_obs = (int)c->desc.masks.size();
  {
    // FNV-1a over the sizes, gate records and masks
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
      const unsigned char *b = (const unsigned char *)p;
      for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 1099511628211ull;
    };
    const int32_t sz[4] = {info.n, info.n_inputs, info.n_weights, info.n_obs};
    mix(sz, sizeof sz);
    mix(c->desc.gates.data(), c->desc.gates.size() * sizeof(Gate));
    mix(c->desc.masks.data(), c->desc.masks.size() * sizeof(uint64_t));
    mix(c->desc.pauli_x.data(), c->desc.pauli_x.size() * sizeof(uint64_t));
    char buf[40];
    snprintf(buf, sizeof buf, "n%d_%016llx", info.n, (unsigned long long)h);
    info.signature = buf;
  }
  std::string rep;
  rc = autotune(c, info, batch, precision, (hipStream_t)stream, (flags & 1) != 0, rep);
  if (needed) *needed = rep.size() + 1;
  if (report && len > 0) {
    size_t k = std::min(len - 1, rep.size());
    memcpy(report, rep.data(), k);
    report[k] = 0;
  }
  if (rc == QTM_ERR_UNSUPPORTED) return fail(rc, "autotune: no candidate reproduced the reference");
  if (rc) return rc == QTM_ERR_HIP ? hip_fail(hipGetLastError(), "autotune") : rc;
  return QTM_OK;
}

// --- uneven batch --------------------------------------------------------

int qtm_multi_create(const qtm_circuit_t *items, int32_t count, qtm_multi_t *out) {
  if (!out || count < 0 || (count > 0 && !items)) return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  *out = nullptr;
  std::unique_ptr<qtm_multi_s> m(new (std::nothrow) qtm_multi_s());
  if (!m) return fail(QTM_ERR_WORKSPACE, "out of host memory");
  int64_t io = 0, wo = 0, oo = 0, so = 0;
  std::vector<MultiItemIn> wide;
  for (int32_t i = 0; i < count; ++i) {
    qtm_circuit_t c = items[i];
    if (!c) return fail(QTM_ERR_INVALID_ARG, "NULL item");
    m->items.push_back(c);
    m->in_off.push_back(io);
    m->w_off.push_back(wo);
    m->out_off.push_back(oo);
    m->st_off.push_back(so);
    if (c->desc.n >= kMinTileQubits && !c->desc.has_offdiag() && !c->desc.has_crot()) {
      const int kt = default_kt(c, QTM_C64);
      const int klo = std::min(c->low_qubits > 0 ? c->low_qubits : 5, kt);
      wide.push_back(MultiItemIn{&c->desc, kt, klo, io, wo, oo, so / 8});
    } else {
      m->narrow.push_back(i);
    }
    io += c->desc.n_inputs;
    wo += c->desc.n_weights;
    oo += (int64_t)c->desc.masks.size();
    so += (int64_t)8 << c->desc.n;
  }
  m->in_off.push_back(io);
  m->w_off.push_back(wo);
  m->out_off.push_back(oo);
  m->st_off.push_back(so);
  if (!wide.empty()) {
    std::string err;
    m->rt = multi_runtime_create(wide, err);
    if (!m->rt) return fail(QTM_ERR_UNSUPPORTED, err);
  }
  *out = m.release();
  return QTM_OK;
}

int qtm_multi_destroy(qtm_multi_t m) {
  delete m;
  return QTM_OK;
}

int qtm_multi_layout(qtm_multi_t m, int64_t *in_off, int64_t *w_off, int64_t *out_off,
                     size_t *state_bytes) {
  if (!m) return fail(QTM_ERR_INVALID_ARG, "NULL multi handle");
  size_t n = m->items.size() + 1;
  if (in_off) memcpy(in_off, m->in_off.data(), n * sizeof(int64_t));
  if (w_off) memcpy(w_off, m->w_off.data(), n * sizeof(int64_t));
  if (out_off) memcpy(out_off, m->out_off.data(), n * sizeof(int64_t));
  if (state_bytes) *state_bytes = (size_t)m->st_off.back();
  return QTM_OK;
}

int qtm_multi_set_option(qtm_multi_t m, int32_t option, int64_t value) {
  if (!m) return fail(QTM_ERR_INVALID_ARG, "NULL multi handle");
  if (option != QTM_OPT_TIMING) return fail(QTM_ERR_UNSUPPORTED, "unknown multi option");
  if (value && !m->timer) m->timer.reset(new EventTimer());
  if (!value) m->timer.reset();
  return QTM_OK;
}

int qtm_multi_timing_read(qtm_multi_t m, int32_t kind, double *total_ms, int64_t *launches) {
  if (!m || kind < 0 || kind > 1 || !total_ms || !launches)
    return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  return read_timer(m->timer.get(), kind, total_ms, launches);
}

namespace {
int check_multi_io(qtm_multi_t m, const double *inputs, const double *weights) {
  if (m->in_off.back() > 0 && !inputs) return fail(QTM_ERR_INVALID_ARG, "inputs is NULL");
  if (m->w_off.back() > 0 && !weights) return fail(QTM_ERR_INVALID_ARG, "weights is NULL");
  return QTM_OK;
}
}  // namespace

int qtm_multi_forward(qtm_multi_t m, const double *inputs, const double *weights, double *expvals,
                      void *state, void *stream) {
  if (!m || !expvals || !state) return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  int rc = check_multi_io(m, inputs, weights);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (m->rt) {
    hipError_t e = multi_runtime_forward(m->rt, inputs, weights, expvals, state, s, m->timer.get());
    if (e != hipSuccess)
      return hip_fail(e, std::string("multi forward: ") + multi_runtime_where(m->rt));
  }
  for (int32_t i : m->narrow) {
    qtm_circuit_t c = m->items[i];
    rc = qtm_forward(c, 1, QTM_C64, inputs ? inputs + m->in_off[i] : nullptr,
                     weights ? weights + m->w_off[i] : nullptr, expvals + m->out_off[i],
                     (char *)state + m->st_off[i], stream);
    if (rc) return rc;
  }
  return QTM_OK;
}

int qtm_multi_backward(qtm_multi_t m, const double *inputs, const double *weights,
                       const double *grad_expvals, void *state, double *grad_weights,
                       double *grad_inputs, void *stream) {
  if (!m || !grad_expvals || !state) return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  if (m->w_off.back() > 0 && !grad_weights) return fail(QTM_ERR_INVALID_ARG, "grad_weights is NULL");
  int rc = check_multi_io(m, inputs, weights);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (m->rt) {
    hipError_t e = multi_runtime_backward(m->rt, inputs, weights, grad_expvals, state, grad_weights,
                                          grad_inputs, s, m->timer.get());
    if (e != hipSuccess)
      return hip_fail(e, std::string("multi backward: ") + multi_runtime_where(m->rt));
  }
  for (int32_t i : m->narrow) {
    qtm_circuit_t c = m->items[i];
    rc = qtm_backward(c, 1, QTM_C64, inputs ? inputs + m->in_off[i] : nullptr,
                      weights ? weights + m->w_off[i] : nullptr, grad_expvals + m->out_off[i],
                      (char *)state + m->st_off[i], grad_weights ? grad_weights + m->w_off[i] : nullptr,
                      grad_inputs ? grad_inputs + m->in_off[i] : nullptr, stream);
    if (rc) return rc;
  }
  return QTM_OK;
}

int qtm_multi_units(qtm_multi_t m, int32_t kind, int64_t *units) {
  if (!m || kind < 0 || kind > 1 || !units) return fail(QTM_ERR_INVALID_ARG, "bad arguments");
  *units = m->rt ? multi_runtime_units(m->rt, kind) : 0;
  return QTM_OK;
}

}  // extern "C"
