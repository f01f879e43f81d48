// Launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "circuit.h"
#include "device_common.h"

namespace qtm {

struct JitSweeps;

// Device copies of a circuit's static data (owned by the circuit handle).
struct DevCircuit {
  int n = 0, n_inputs = 0, n_weights = 0, n_obs = 0, n_occ = 0;
  uint64_t *masks = nullptr;
  int32_t *occ_src = nullptr, *occ_idx = nullptr, *occ_widx = nullptr;
  // parameter slot -> occurrences with the other factor of a scaled angle
  int32_t *w_ptr = nullptr, *w_list = nullptr, *w_fac = nullptr;
  int32_t *x_ptr = nullptr, *x_list = nullptr, *x_fac = nullptr;
  // observables with X or Y factors: their indices and Pauli strings
  int n_nd = 0;
  int32_t *nd_idx = nullptr;
  uint64_t *nd_x = nullptr, *nd_z = nullptr;
};

struct HostCircuitInfo {
  std::vector<Gate> gates;
  std::vector<int32_t> gate_occ;
};

// Device copy of a fused plan for one (kt, klo).
struct DevPlan {
  int kt = 0, klo = 0, n_blocks = 0, n_gslots = 0, max_gslots = 0;
  int n_sweeps = 0;
  std::vector<int32_t> sweep_off_fwd, sweep_off_bwd;
  int32_t *code = nullptr;      // program
  int32_t *thr = nullptr;       // per-stage per-thread global offsets
  int32_t *blk = nullptr;       // block records for the matrix prep
  int32_t *blk_off = nullptr;   // block -> offset in blk
  int32_t *occ_gslot = nullptr; // occurrence -> gradient slot
  int32_t *gs_ptr = nullptr;    // gradient slot -> its occurrences (CSR, [n_gslots + 1])
  int32_t *gs_occ = nullptr;
  float *obs_sgn_f = nullptr;   // [(M+1)][16] signs of the last forward stage (float)
  double *seed_sgn = nullptr;   // [M][16] signs of the first backward load layout (double)
};

// Optional hook around every sweep-kernel launch (kind 0 = forward sweep,
// 1 = backward sweep); used to time the kernels with events on the stream.
struct SweepTimer {
  virtual void before(int kind, hipStream_t s) = 0;
  virtual void after(int kind, hipStream_t s) = 0;
  virtual ~SweepTimer() = default;
};

hipError_t launch_half_angles(const DevCircuit &d, int B, const double *x, const double *w,
                              double2 *cs, hipStream_t s);
hipError_t launch_obs_final(const double *part, int B, int nblk, int M, double *out,
                            bool normalise, hipStream_t s);
hipError_t launch_scatter(const DevCircuit &d, int B, const double *gocc, const double *x,
                          const double *w, double *gw, double *gx, hipStream_t s);
size_t plain_part_doubles(const DevCircuit &d, int B);
// Observables with X or Y factors, from the final states: out[b][idx_j]
// (normalised).  part: pauli_part_doubles(d, B) doubles.
size_t pauli_part_doubles(const DevCircuit &d, int B);
template <typename R>
hipError_t launch_pauli_expval(const DevCircuit &d, int B, const void *state, double *part, double *out,
                               hipStream_t s);
// Their bra term (see k_pauli_seed), written to lam or added to it.
template <typename R>
hipError_t launch_pauli_seed(const DevCircuit &d, int B, const void *psi, void *lam, const double *G,
                             bool accumulate, hipStream_t s);
// Diagnostics: rows of the forward's observable partials on the per-gate
// path; every sample's squared state norm from such partials ([B][rows][M + 1],
// the norm in column M); the first non-finite angle source (see k_first_nonfinite).
int plain_norm_rows(int n, int B);
hipError_t launch_norms(const double *part, int B, int rows, int M, double *out, hipStream_t s);
hipError_t launch_first_nonfinite(const double *x, int64_t nx, const double *w, int64_t nw,
                                  unsigned long long *first, hipStream_t s);
// Jacobian passes over rows = k x B rows (row r: sample r mod B, observable
// m0 + r / B): the one-hot upstream gradients, `copies` back-to-back copies of
// a buffer (bytes a multiple of 8), and the rows' per-sample gradients
// scattered into [B][M][n_weights] and [B][M][n_inputs].
hipError_t launch_onehot(double *G, int rows, int B, int M, int m0, hipStream_t s);
hipError_t launch_replicate(void *dst, const void *src, size_t bytes, int copies, hipStream_t s);
hipError_t launch_scatter_jac(const DevCircuit &d, int rows, int B, const double *gocc, const double *x,
                              const double *w, int m0, double *jw, double *jx, hipStream_t s);

template <typename R>
hipError_t plain_forward(const DevCircuit &d, const HostCircuitInfo &h, int B, const double2 *cs,
                         void *state, double *part, double *out, bool normalise, hipStream_t s);
template <typename R>
hipError_t plain_backward(const DevCircuit &d, const HostCircuitInfo &h, int B, const double2 *cs,
                          const double *x, const double *w, void *state, void *lam,
                          const double *G, double *part, double *gocc, double *gw, double *gx,
                          hipStream_t s);

// Fused path workspace sizes and entry points.
int fused_wg_per_sample(int n, int kt);
size_t fused_part_obs_doubles(const DevCircuit &d, const DevPlan &p, int B);
size_t fused_part_grad_doubles(const DevCircuit &d, const DevPlan &p, int B);

// Periodic renormalisation of the fused sweeps: every `period` sweeps (0 =
// off) the loads are rescaled by norms recorded by the sweeps before (see
// FwdArgs / BwdArgs).  fwd: [n_sweeps][B][workgroups per sample] doubles,
// bwd: [n_sweeps][B][workgroups per sample][4] doubles (fused_rn_doubles).
struct Renorm {
  int period = 0;
  double *fwd = nullptr, *bwd = nullptr;
};
size_t fused_rn_doubles(const DevCircuit &d, const DevPlan &p, int B);

// js: kernels specialised for this plan (nullptr: the compiled sweep kernels).
// The forward's prep also writes the derivative coefficients when coef is
// not NULL; the backward skips its prep when `prepped` (mats and coef hold
// what a forward computed from the same angles, plan and batch).  The
// backward reads the final states from state_in when it is not NULL (else
// from state) and leaves intermediate states in state.
template <typename R>
hipError_t fused_forward(const DevCircuit &d, const DevPlan &p, int B, const double *x,
                         const double *w, void *mats, double *coef, void *state, double *part_obs,
                         double *out, bool store_final, hipStream_t s, SweepTimer *tm,
                         const JitSweeps *js, const Renorm &rn);
template <typename R>
hipError_t fused_backward(const DevCircuit &d, const DevPlan &p, int B, const double *x,
                          const double *w, const double *G, void *mats, double *coef, bool prepped,
                          void *state, const void *state_in, void *lam, double *part_grad,
                          double *part_norm, double *gocc, double *gw, double *gx, hipStream_t s,
                          SweepTimer *tm, const JitSweeps *js, const Renorm &rn);

}  // namespace qtm
