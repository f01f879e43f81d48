/*
 * qtm.h -- C ABI of libqtm: batched exact statevector forward and adjoint
 * vector-Jacobian product of parameterised circuits on one gfx950 GPU.
 *
 * The operations are those of "Qiskit-Torch-Module" (arXiv 2404.06314):
 *   - a circuit is a gate list whose rotation angles index into an input
 *     vector (data encoding s) or a weight vector (trainable Theta), plus a
 *     list of observables (Sec. II-D: encoding and variational parameters
 *     given separately, indexed in construction order, Sec. II-C);
 *   - qtm_forward evolves |0...0> once per sample and reads every observable
 *     from that one state (Sec. II-A, Eq. (3)-(4)), for a batch of inputs with
 *     shared weights (Sec. II-B, Eq. (6));
 *   - qtm_backward is the reverse-mode ("adjoint") gradient the paper extends
 *     to several observables (Sec. II-A, Eq. (5)), returned as a vector-
 *     Jacobian product: given G = dL/d<O> of shape (B, M) it writes
 *     dL/dweights = sum_b sum_m G[b][m] d<O_m>_b/dweights and
 *     dL/dinputs[b] = sum_m G[b][m] d<O_m>_b/dinputs[b].
 *
 * Conventions.  Basis index x = sum_q b_q 2^q (qubit q is bit q).
 * RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2).
 * CNOT(q0 -> q1) flips bit q1 where bit q0 is 1; CZ(q0, q1) negates the
 * amplitudes whose bits q0 and q1 are both 1.  An observable is a Pauli-Z
 * string given as a bitmask S: <Z_S> = sum_x (-1)^popcount(x & S) |psi_x|^2.
 *
 * Memory.  Every array argument named "dev" is device memory owned by the
 * caller; the library never frees it.  Host arrays are read during the call
 * only.  Circuit and multi handles, their plans and the internal workspace
 * (second state buffer, partial sums, matrices) are owned by the library
 * and released by the matching *_destroy.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Calls are
 * asynchronous on it: launch errors are returned, execution errors surface
 * at the caller's next synchronisation.  A handle's workspace is shared by
 * all calls on that handle, so calls on one handle must be ordered (same
 * stream, or synchronised by the caller); calls that overlap on one handle
 * race.
 *
 * Errors.  Every function returns QTM_OK (0) or a negative code and never
 * throws; qtm_last_error() gives a message for the calling thread's last
 * failure.
 */
#ifndef QTM_PUBLIC_HEADER_
#define QTM_PUBLIC_HEADER_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QTM_OK 0
#define QTM_ERR_INVALID_ARG (-1) /* bad qubit, control == target, index out of range,
                                    batch <= 0, NULL where required, bad mask */
#define QTM_ERR_UNSUPPORTED (-2) /* n_qubits > 30, unknown gate type or option */
#define QTM_ERR_WORKSPACE (-3)   /* device allocation of the workspace failed, or it would
                                    take a circuit handle's workspace beyond the byte count in
                                    the environment variable QTM_MAX_WORKSPACE_BYTES (read when
                                    a workspace buffer grows; unset or 0 = no cap) */
#define QTM_ERR_HIP (-4)         /* a HIP call failed; message in qtm_last_error */
#define QTM_ERR_STATE (-5)       /* state buffer not produced by qtm_forward for
                                    this (circuit, batch, precision) */

enum { QTM_RX = 0, QTM_RY = 1, QTM_RZ = 2, QTM_CNOT = 3, QTM_CZ = 4 };
/* Fixed one-qubit gates (on q0): Hadamard, Pauli X, Y, Z, S = diag(1, i),
 * S^dag, T = diag(1, e^{i pi/4}), T^dag, SX = sqrt(X) = [[1+i, 1-i],
 * [1-i, 1+i]] / 2.  They fuse into the per-wire blocks of the fused path. */
enum { QTM_H = 5, QTM_X = 6, QTM_Y = 7, QTM_Z = 8, QTM_S = 9, QTM_SDG = 10, QTM_T = 11,
       QTM_TDG = 12, QTM_SX = 13 };
/* Controlled rotations: q0 = control, q1 = target, src = QTM_SRC_INPUT or
 * QTM_SRC_WEIGHT; the rotation exp(-i t P / 2) acts on the target where the
 * control bit is 1.  Circuits with them run on the per-gate path
 * (QTM_PATH_FUSED returns QTM_ERR_UNSUPPORTED for them, and so do the
 * fused-plan diagnostics and qtm_autotune); in an uneven batch they run one
 * by one after the persistent kernels. */
enum { QTM_CRX = 14, QTM_CRY = 15, QTM_CRZ = 16 };
enum { QTM_SRC_NONE = 0, QTM_SRC_INPUT = 1, QTM_SRC_WEIGHT = 2, QTM_SRC_SCALED = 3 };
enum { QTM_C64 = 0, QTM_C128 = 1 }; /* state amplitudes: complex float / complex double */

/* Kernel path (option QTM_OPT_PATH). */
enum { QTM_PATH_AUTO = 0, QTM_PATH_PLAIN = 1, QTM_PATH_FUSED = 2 };

/* Options for qtm_set_option. */
enum {
  QTM_OPT_PATH = 0,        /* QTM_PATH_*; AUTO = fused */
  QTM_OPT_TILE_QUBITS = 1, /* fused path: qubits per LDS tile (0 = default) */
  QTM_OPT_LOW_QUBITS = 2,  /* fused path: contiguous low qubits always in a tile */
  QTM_OPT_RENORM = 3,      /* fused path: R >= 1 rescales the states every R sweeps with FP64
                              norms (see the note at qtm_forward); 0 (default): no rescale.  The
                              expectation values and gradients are divided by the FP64 norm in
                              either case.  0 <= R <= 1024, else QTM_ERR_INVALID_ARG. */
  QTM_OPT_TIMING = 4,      /* 1: record HIP events around every sweep kernel (qtm_timing_read) */
  QTM_OPT_JIT = 5          /* fused path: 1 = run sweep kernels specialised for this circuit
                              (generated from its plan and compiled with hiprtc on the first
                              call per precision, which takes seconds; errors surface as
                              QTM_ERR_UNSUPPORTED with the compiler's message), 0 = the
                              compiled generic sweep kernels (default) */,
  QTM_OPT_CHECK_ANGLES = 6 /* 1: qtm_forward, qtm_backward and qtm_jacobian first check that every
                              input and weight is finite (a check kernel on the stream, then a
                              copy to the host and a wait for the stream); a NaN or infinity
                              returns QTM_ERR_INVALID_ARG naming the first such entry, and
                              nothing else is launched.  0 (default): no check, no wait. */,
  QTM_OPT_DENSE_BLOCKS = 7 /* 1: complex64 forwards apply the weight part of each layer, RZ RY on
                              4 consecutive qubits with the CZ gates inside the block, as one dense
                              16 x 16 unitary shared by the batch (Sec. II-B, Eq. (6)) on the
                              matrix cores, one pass over the state per (layer, block), with the
                              per-sample RX encoding on the vector units and the CZ gates between
                              blocks as signs.  Only for layered circuits (per layer RX(input),
                              RY(weight), RZ(weight) on every qubit in qubit order, then the open
                              CZ chain) of 12, 16, ... qubits with Z-string observables, else
                              QTM_ERR_UNSUPPORTED; the backward is unchanged (it prepares its own
                              gate matrices).  0 (default): the fused sweeps. */,
  QTM_OPT_GREEDY_PLAN = 8  /* fused path, sweep planning.  0 (default): with QTM_OPT_JIT the sweeps
                              are planned for the specialised kernels, which skip the tiles whose
                              amplitudes are all zero (a qubit not yet acted on by a non-diagonal
                              gate holds |0>): a search over tile sequences by an estimated cost
                              that counts only the tiles that run; the generic kernels take the
                              greedy plan.  1: the greedy plan (each sweep runs the most ops a
                              tile allows) for both.  Results agree within rounding either way. */,
  QTM_OPT_PLAN_IO = 9      /* fused path, the zero-skip planning of QTM_OPT_GREEDY_PLAN = 0: the HBM
                              traffic of a sweep over the whole state, forward and backward, in
                              units of one fused block applied to the whole state, as the planner's
                              cost estimate weighs it against the block work (1..64, default 12;
                              larger values favour fewer, fuller sweeps).  The autotuner tries 8
                              and 16 beside the default.  Results agree within rounding. */,
  QTM_OPT_JAC_CHUNK = 10   /* qtm_jacobian: observables per adjoint pass, 1..65535 (capped at
                              n_obs and at 65535 / batch rows).  0 (default): as many as keep one
                              pass's copies of the final states within 64 MiB, so one per pass
                              for batches whose states exceed that.  Results agree within
                              rounding for every value. */
};

/* One gate.  Rotations (RX, RY, RZ): q0 = qubit, src = QTM_SRC_INPUT or
 * QTM_SRC_WEIGHT, index = slot in that vector (q1 ignored); or
 * src = QTM_SRC_SCALED: the angle is weights[q1] * inputs[index], the
 * trainable input scaling lambda * s of the paper's ansatz (Sec. III-A,
 * Eq. (7)); the gradients follow the chain rule (dL/dweights[q1] gains
 * g * inputs[index], dL/dinputs[index] gains g * weights[q1] for the angle
 * derivative g).
 * CNOT: q0 = control, q1 = target.  CZ: q0, q1 (symmetric).  src/index
 * ignored for entanglers. */
typedef struct {
  int32_t type, q0, q1, src, index;
} qtm_gate;

typedef struct qtm_circuit_s *qtm_circuit_t;
typedef struct qtm_multi_s *qtm_multi_t;

/* Validate and copy a circuit (host arrays).  1 <= n_qubits <= 30; gate
 * types as above (an unknown type is QTM_ERR_UNSUPPORTED);
 * obs_zmask[m] must have no bit >= n_qubits and n_obs >= 1.  Gates are
 * applied in list order (paper Eq. (7): the ansatz is a product of layers).
 * *out receives a new handle on success. */
int qtm_circuit_create(int32_t n_qubits, const qtm_gate *gates, int32_t n_gates,
                       int32_t n_inputs, int32_t n_weights, const uint64_t *obs_zmask,
                       int32_t n_obs, qtm_circuit_t *out);

/* As qtm_circuit_create, with observables that are general Pauli strings
 * (the paper admits any observable, Sec. II-A; its benchmarks use Z only).
 * Observable m has, on qubit q, the factor I, X, Z or Y for bits
 * (obs_xmask[m], obs_zmask[m]) at q = (0, 0), (1, 0), (0, 1) or (1, 1).
 * obs_xmask may be NULL (every observable a Z string: qtm_circuit_create).
 * Neither mask may have a bit >= n_qubits.  Z strings are evaluated inside
 * the sweeps; each string with X or Y factors costs one more read pass over
 * the final states in the forward and adds its term to the backward's
 * initial bra (one more read of the states and a write of the bra), and
 * the final states are then always stored (in the workspace when
 * qtm_forward gets state = NULL).  In an uneven batch (qtm_multi_create)
 * such circuits run one by one after the persistent kernels. */
int qtm_circuit_create_pauli(int32_t n_qubits, const qtm_gate *gates, int32_t n_gates,
                             int32_t n_inputs, int32_t n_weights, const uint64_t *obs_xmask,
                             const uint64_t *obs_zmask, int32_t n_obs, qtm_circuit_t *out);
int qtm_circuit_destroy(qtm_circuit_t c);

/* Tune the kernel path of a circuit (see QTM_OPT_*). */
int qtm_set_option(qtm_circuit_t c, int32_t option, int64_t value);

/* Bytes of the caller-owned state buffer for (batch, precision):
 * batch * 2^n amplitudes of 8 (C64) or 16 (C128) bytes, sample-major.  The
 * library remembers (host side) which circuit, batch and precision last
 * filled a buffer, and qtm_backward checks it (QTM_ERR_STATE). */
int qtm_state_bytes(qtm_circuit_t c, int32_t batch, int32_t precision, size_t *bytes);

/* Forward pass (Sec. II-A, II-B).
 * Periodic renormalisation (QTM_OPT_RENORM = R >= 1, fused path): forward
 * sweep s, for s a positive multiple of R, scales the state it loads by
 * 1 / sqrt(N), N the FP64 norm the sweep before it stored; backward sweep i
 * (a positive multiple of R) scales psi and lambda by the square roots of
 * the products of their FP64 load / end norm ratios over the R sweeps
 * before it, undoing the rounding drift of those sweeps.  Every gate is
 * linear, so the results change by rounding only.  Ignored by the per-gate
 * path and the uneven batch.
 *   inputs   dev [batch][n_inputs]  float64 (may be NULL if n_inputs == 0)
 *   weights  dev [n_weights]        float64 (may be NULL if n_weights == 0)
 *   expvals  dev [batch][n_obs]     float64, written
 *   state    dev, qtm_state_bytes(); receives the final states for a later
 *            qtm_backward.  NULL: not kept (a library workspace is used). */
int qtm_forward(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                const double *weights, double *expvals, void *state, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass as qtm_forward, with every workspace buffer (gate matrices,
 * derivative coefficients, partial sums) carved from a scratch array of
 * 16 MiB that the library's code object holds on each GPU until the process
 * ends.  It calls no hipMalloc, hipFree or other allocating routine.
 *   state    dev, qtm_state_bytes(); required (receives the final states).
 *   others   as qtm_forward.
 * Preconditions: one qtm_forward (or qtm_backward / qtm_autotune) with the
 * same precision and tile options has run on this device, so that the
 * circuit's constant tables and plan are resident (else QTM_ERR_STATE).  With
 * QTM_OPT_JIT the specialised kernels are used if that call loaded them,
 * otherwise the compiled ones.  A batch whose buffers exceed the scratch
 * (error message gives both sizes) returns QTM_ERR_WORKSPACE.
 * Every call on a GPU shares that GPU's scratch array, which keeps the last
 * call's contents: calls that overlap on one GPU (other streams, other
 * threads, other handles) race.  A state buffer filled here is not accepted
 * by qtm_backward (QTM_ERR_STATE), and qtm_forward_norms does not report
 * this pass. */
int qtm_forward_noalloc(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                        const double *weights, double *expvals, void *state, void *stream);

/* Adjoint VJP (Sec. II-A, reverse gradient).
 *   grad_expvals  dev [batch][n_obs] float64: G = dL/d<O>
 *   state         dev buffer written by qtm_forward with the same circuit, batch,
 *                 precision and angles; the backward consumes it: it works in
 *                 place and does not un-compute the states back to |0...0>
 *                 (the last un-apply of each qubit is skipped and the final
 *                 sweep stores nothing), so its contents on return are
 *                 unspecified and one forward serves one backward.  The
 *                 rounding drift of the evolution is reported instead by
 *                 qtm_forward_norms.
 *                 NULL: the forward is recomputed into the workspace.
 *   grad_weights  dev [n_weights] float64, overwritten (summed over the batch)
 *   grad_inputs   dev [batch][n_inputs] float64, overwritten; may be NULL. */
int qtm_backward(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                 const double *weights, const double *grad_expvals, void *state,
                 double *grad_weights, double *grad_inputs, void *stream);

/* Full Jacobian of the expectation values (the paper's (B, M, |Theta|)
 * result, Sec. II-A, Eq. (5)-(6)): forward once, then adjoint backward passes
 * with one-hot upstream gradients e_m.  A pass takes k observables
 * (QTM_OPT_JAC_CHUNK) over k x batch rows, row r being sample r mod batch
 * with observable m0 + r / batch, and starts from k copies of the final
 * states; with k = 1 it reads them in place.  Library workspace: the final
 * states plus two buffers of k x batch states (and k copies of the inputs).
 * Every row's gradient is computed by the same kernels as in a
 * one-observable pass; a pass of k > 1 prepares its own gate matrices for
 * the repeated input rows.
 *   expvals      dev [batch][n_obs] float64, overwritten; may be NULL
 *   jac_weights  dev [batch][n_obs][n_weights] float64: d<O_m>(sample b)/dw_j
 *                (per sample, not summed over the batch)
 *   jac_inputs   dev [batch][n_obs][n_inputs] float64, or NULL
 * Cost ~ forward + n_obs backward passes.  Same stream semantics as
 * qtm_backward. */
int qtm_jacobian(qtm_circuit_t c, int32_t batch, int32_t precision, const double *inputs,
                 const double *weights, double *expvals, double *jac_weights, double *jac_inputs,
                 void *stream);

/* Uneven batch (one sample per circuit, circuits of different size and depth,
 * Sec. II-B: batch elements are independent; each circuit has its own
 * weights, so no gradient is summed across items).  Amplitudes are complex64.
 *
 * qtm_multi_create copies the item list (the item handles must stay alive
 * while the multi handle exists) and plans every distinct circuit once
 * (items with equal gates, observables and tile options share one program).
 * Packed caller arrays: item i reads inputs[in_off[i] ...] (n_inputs of item
 * i), weights[w_off[i] ...] (n_weights), writes expvals[out_off[i] ...]
 * (n_obs values), grad_inputs / grad_weights at the input / weight offsets,
 * and reads grad_expvals at the expval offsets.  qtm_multi_layout fills the
 * offsets (arrays of `count` + 1 entries; the last entry is the total
 * length) and the state bytes (8 * 2^n per item, packed in item order).
 *
 * Items with at least 4 qubits run in one persistent kernel per direction
 * (tile units of all circuits in one queue, longest remaining chain first),
 * launched together with its prep and reduction kernels as one HIP graph
 * built on the first call; the graph's pointer arguments are updated when
 * the caller's pointers change.  Items below 4 qubits run one by one on the
 * per-gate kernels after the graph.
 *
 * qtm_multi_forward keeps every item's final state in `state` (dev, caller
 * owned, qtm_multi_layout bytes); qtm_multi_backward needs the state of the
 * preceding qtm_multi_forward on the same handle and inputs, and consumes it
 * (the adjoint un-computes it).  inputs / weights / grad_inputs may be NULL
 * only when the corresponding total length is 0 (grad_inputs: always).
 * If a persistent kernel's dependency wait ever times out (an internal
 * error), the pass's outputs are NaN. */
int qtm_multi_create(const qtm_circuit_t *items, int32_t count, qtm_multi_t *out);
int qtm_multi_destroy(qtm_multi_t m);
int qtm_multi_layout(qtm_multi_t m, int64_t *in_off, int64_t *w_off, int64_t *out_off,
                     size_t *state_bytes);
int qtm_multi_forward(qtm_multi_t m, const double *inputs, const double *weights,
                      double *expvals, void *state, void *stream);
int qtm_multi_backward(qtm_multi_t m, const double *inputs, const double *weights,
                       const double *grad_expvals, void *state, double *grad_weights,
                       double *grad_inputs, void *stream);
/* Only QTM_OPT_TIMING: with it set, the multi kernels are launched one by one
 * (no graph) and events bracket each persistent kernel; read them with
 * qtm_multi_timing_read (kind 0 forward, 1 backward; same contract as
 * qtm_timing_read). */
int qtm_multi_set_option(qtm_multi_t m, int32_t option, int64_t value);
int qtm_multi_timing_read(qtm_multi_t m, int32_t kind, double *total_ms, int64_t *launches);
/* Number of tile work units in the persistent queue of a pass (kind 0
 * forward, 1 backward); -1 before the first call has built the queue. */
int qtm_multi_units(qtm_multi_t m, int32_t kind, int64_t *units);

/* Diagnostics (norm-drift watchdog): every sample's squared norm <psi|psi>
 * of the final state of the last forward pass on c (qtm_forward, or the
 * forward that qtm_backward with state = NULL or qtm_jacobian runs), taken
 * from that pass's own FP64 reduction (no further pass over the states).
 * The evolution is unitary (Eq. (1)-(2): a normalised state), so the exact
 * value is 1 and its distance from 1 is the rounding drift of the amplitude
 * arithmetic; the expectation values are divided by it.
 *   norms  dev [batch] float64, written (asynchronously on `stream`).
 * QTM_ERR_STATE if the last forward pass on c had another batch, or if a
 * per-gate-path backward has reused its partial sums since. */
int qtm_forward_norms(qtm_circuit_t c, int32_t batch, double *norms, void *stream);

/* Diagnostics: with QTM_OPT_TIMING set, the library records a pair of HIP
 * events on the call's stream around every sweep kernel it launches.
 * qtm_timing_read waits for those events, returns the summed kernel time in
 * milliseconds and the number of launches of `kind` (0 = forward sweep,
 * 1 = backward sweep) since the last read, and forgets them. */
int qtm_timing_read(qtm_circuit_t c, int32_t kind, double *total_ms, int64_t *launches);

/* Tune the fused path of c for (batch, precision) on the current device:
 * tile qubits, contiguous low qubits, the compiled generic versus the
 * specialised sweep kernels (QTM_OPT_JIT), for the fastest specialised
 * configuration also the greedy sweep plan (QTM_OPT_GREEDY_PLAN) and the
 * zero-skip plans with traffic weights 8 and 16 (QTM_OPT_PLAN_IO), and for
 * complex64 layered CZ-chain circuits the dense-block forward
 * (QTM_OPT_DENSE_BLOCKS).  Every candidate must reproduce
 * the per-gate complex128 result on seeded synthetic inputs within the
 * precision's tolerances (<Z> 1e-5 absolute and gradients 1e-4 relative for
 * complex64; 1e-12 / 1e-10 for complex128) before it is timed; the fastest
 * is installed with qtm_set_option (among the candidates within 3% of it:
 * the most contiguous low qubits, then the larger tile, then the default
 * sweep plan).  flags bit 0: read and update the JSON
 * cache ($QTM_AUTOTUNE_CACHE, else ~/.cache/qtm_autotune.json), keyed by the
 * circuit's gates and observables, batch, precision and GPU architecture.
 * report (may be NULL): JSON summary of the candidates (truncated to len - 1
 * bytes); *needed = its full length + 1.  Allocates device memory for the
 * trial inputs and one state, synchronises `stream`, takes seconds (minutes
 * at 26 qubits); with QTM_AUTOTUNE_LOG=1 in the environment it prints one
 * line per candidate to stderr as each finishes.
 * QTM_ERR_UNSUPPORTED if no candidate passed (options reset to defaults). */
int qtm_autotune(qtm_circuit_t c, int32_t batch, int32_t precision, void *stream, int32_t flags,
                 char *report, size_t len, size_t *needed);

/* Diagnostics: the HIP source of the specialised kernel of forward (dir 0)
 * or backward (dir 1) sweep `sweep` at `precision` into buf (truncated to
 * len - 1 bytes, NUL-terminated); *needed = full length + 1.  Host only. */
int qtm_jit_source(qtm_circuit_t c, int32_t precision, int32_t dir, int32_t sweep, char *buf,
                   size_t len, size_t *needed);
/* Compile (without loading) the specialised sweep kernels of c at
 * `precision`; host only, no device needed.  QTM_ERR_UNSUPPORTED with the
 * compiler's message on failure.  The compiled code is kept for later calls
 * with QTM_OPT_JIT. */
int qtm_jit_compile(qtm_circuit_t c, int32_t precision);
/* Diagnostics: vector registers and scratch bytes per thread of a loaded
 * specialised kernel (after a call with QTM_OPT_JIT on this device). */
int qtm_jit_info(qtm_circuit_t c, int32_t precision, int32_t dir, int32_t sweep, int32_t *vgprs,
                 int32_t *scratch);

/* Diagnostics: JSON description of the fused-path plan (sweeps, tile qubits,
 * stages and the gate indices each stage runs) for the given precision, the
 * encoded device program, and per sweep the qubits excited by its end
 * ("excited": a bit mask; the specialised kernels take amplitudes with a
 * bit of an unexcited qubit as 0).  Writes at most len bytes (NUL-
 * terminated) into buf and the full size into *needed; buf may be NULL to
 * query the size. */
int qtm_plan_json(qtm_circuit_t c, int32_t precision, char *buf, size_t len, size_t *needed);

/* Message for the calling thread's last non-OK return ("" if none). */
const char *qtm_last_error(void);

/* Library version string. */
const char *qtm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QTM_PUBLIC_HEADER_ */
