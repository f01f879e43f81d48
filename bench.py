#!/usr/bin/env python3
"""Throughput of the batched statevector forward + adjoint VJP on one GPU.

One step = qtm_forward (keeping the final states) + qtm_backward (adjoint
vector-Jacobian product to dL/dweights and dL/dinputs) over one batch of
synthetic inputs already resident in HBM.  Default workload: n = 20 qubits,
8 layers (RX encoding, RY + RZ trainable, CZ ladder), batch 64, complex64
amplitudes, Z_i observables on every qubit.

Prints one JSON line (metric, value, roofline of the dominant kernel and the
CPU oracle's throughput on a bounded sample); progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "circuit evals/s (fwd+adjoint grad) n=20 depth 8 batch 64; % peak HBM GB/s"
HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
# FP32 vector FMA peak without packed math: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that determine a sweep kernel family's memory traffic: the HBM
# byte counts recorded under profiles/ hold for a kernel only while these are
# unchanged.
_COMMON = ["sweep_ops.h", "device_common.h", "layout.h", "circuit.cpp"]
KERNEL_SOURCES = {
    "qtm_jit": ["jit.cpp"] + _COMMON,
    "k_fused": ["fused.hip", "sweep_fwd.inc", "sweep_bwd.inc"] + _COMMON,
    "k_multi": ["multi.hip", "schedule.cpp", "sweep_fwd.inc", "sweep_bwd.inc"] + _COMMON,
    "k_k9": ["k9.hip", "sweep_ops.h", "device_common.h"],
}


def kernel_digest(kernel: str) -> str:
    import hashlib
    fam = next(k for k in KERNEL_SOURCES if kernel.startswith(k))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[fam]:
        with open(os.path.join(ROOT, "paper_2404_06314_amd", "csrc", f), "rb") as fh:
            # whole-line comments do not change a kernel
            for line in fh:
                if not line.lstrip().startswith(b"//"):
                    h.update(line)
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str, plan: str = ""):
    """HBM bytes per launch of `kernel` on `workload` from the counter summaries
    in profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a device copy), or None
    when none was recorded for the current kernel sources and, for kernels
    whose sweeps depend on the sweep plan, for this plan ("io12": zero-skip
    planning with traffic weight 12, "greedy")."""
    import glob
    digest = kernel_digest(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) < 6 or f[0] != "traffic_bytes_per_launch" or f[1] != kernel or f[2] != workload \
                        or f[4] != "sources" or f[5] != digest:
                    continue
                if (f[6:] == ["plan", plan]) if plan else len(f) == 6:
                    return int(f[3])
    return None


def block_ops(plan, kind: int = 0) -> float:
    """Fused single-qubit blocks the program applies as matrices, in units of
    a full 2x2 gate: in the forward (kind 0) every block, the first block on
    each qubit counting half (op code 5: its |1> inputs are 0, so half the
    products); in the backward (kind 1) the blocks it un-applies, i.e.
    without the last block on each qubit, whose un-apply the method does not
    need (op code 4: transition-matrix sums only)."""
    code = plan["code"]
    n = 0.0
    for off in plan["sweep_off_fwd" if kind == 0 else "sweep_off_bwd"]:
        nst = code[off]
        for s in range(nst):
            so = code[off + 90 + s]
            nops = code[so]
            for o in range(nops):
                c = code[so + 40 + 4 * o]
                n += 1.0 if c == 1 else 0.5 if c == 5 else 0.0
    return n


def _sweep_block_ops(plan, kind: int, unapply_first: bool):
    """block_ops per sweep of the pass (in its own order); with
    unapply_first, the backward also counts each qubit's last block where
    the specialised kernels un-apply it (every sweep but the one the
    backward ends with, see live_work)."""
    code = plan["code"]
    offs = plan["sweep_off_fwd" if kind == 0 else "sweep_off_bwd"]
    out = []
    for i, off in enumerate(offs):
        n = 0.0
        nst = code[off]
        for s in range(nst):
            so = code[off + 90 + s]
            for o in range(code[so]):
                c = code[so + 40 + 4 * o]
                n += 1.0 if c == 1 else 0.5 if c == 5 else \
                    (1.0 if c == 4 and unapply_first and i < len(offs) - 1 else 0.0)
        out.append(n)
    return out


def live_work(plan, n: int, kind: int, jit: bool):
    """(state passes, block units) of one pass: the state-array reads and
    writes per amplitude of the register, and the fused blocks applied as
    full 2x2 gates over the whole register (block_ops), both summed over
    the sweeps and counting only the work the kernels do.

    The state starts at |0...0>; with D_in / D_out the qubits not excited
    before / after forward sweep s (plan["excited"]), the amplitudes with a
    bit of D_out set are 0 throughout sweep s.  The specialised kernels
    (jit) run only tiles with no D_out bit among their outer qubits (all
    tiles in the last forward sweep), read psi (and lambda) only where no
    bit of D_in (forward) / D_out (backward) is set, and store only where
    the next sweep reads: no D_out bit (forward, but all of the final
    state) / no D_in bit (backward).  The compiled kernels do all of it."""
    S = len(plan["sweeps"])
    full = (1 << n) - 1
    ex = plan["excited"]
    frac = lambda m: 2.0 ** -bin(m).count("1")
    blocks = _sweep_block_ops(plan, kind, jit)
    passes = units = 0.0
    for i in range(S):
        s = i if kind == 0 else S - 1 - i  # forward index
        din = full if s == 0 else full & ~ex[s - 1]
        dout = full & ~ex[s]
        if not jit:
            din = dout = 0
        tile = sum(1 << q for q in plan["sweeps"][s]["tile"])
        skip = 0 if s == S - 1 else dout & ~tile
        units += blocks[i] * frac(skip)
        if kind == 0:
            passes += (0.0 if s == 0 else frac(din)) + (1.0 if s == S - 1 else frac(dout))
        else:
            passes += frac(dout) * (1 if s == S - 1 else 2)   # psi (and lambda) read
            passes += 0.0 if s == 0 else 2 * frac(din)         # psi and lambda stored
    return passes, units


def grad_units(plan, n: int, jit: bool) -> float:
    """Parameterised blocks whose transition-matrix sums the backward takes
    (op codes 1 and 4 with a gradient slot), in units of a block over the
    whole register, counting only the tiles the kernels run (as live_work)."""
    code = plan["code"]
    offs = plan["sweep_off_bwd"]
    S = len(offs)
    full = (1 << n) - 1
    ex = plan["excited"]
    units = 0.0
    for i, off in enumerate(offs):
        s = S - 1 - i  # forward index
        g = 0
        for st in range(code[off]):
            so = code[off + 90 + st]
            for o in range(code[so]):
                c, gs = code[so + 40 + 4 * o], code[so + 40 + 4 * o + 3]
                g += 1 if c in (1, 4) and gs >= 0 else 0
        tile = sum(1 << q for q in plan["sweeps"][s]["tile"])
        dout = full & ~ex[s]
        skip = 0 if (s == S - 1 or not jit) else dout & ~tile
        units += g * 2.0 ** -bin(skip).count("1")
    return units


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(wl, threads: int, samples: int):
    import numpy as np
    import oracle
    oracle.build(force=False)
    s = min(samples, wl.batch)
    x, G = wl.inputs[:s], wl.grad_out[:s]
    t0 = time.perf_counter()
    oracle.vjp(wl.circuit, x, wl.weights, G, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": s / dt, "unit": "circuit evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{s} of {wl.batch} samples of the same workload, forward + adjoint VJP "
                      f"in complex128, samples split over {threads} threads; {dt:.1f} s"}


def cpu_baselines(wl, threads: int, samples: int, samples_1: int):
    """The oracle on all `threads` cores (the reported value) and on one core,
    with the host's CPU model and core count."""
    allc = cpu_baseline(wl, threads, samples)
    one = cpu_baseline(wl, 1, samples_1)
    model, nproc = cpu_info()
    allc["single_core"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    allc["cpu_model"] = model
    allc["nproc"] = nproc
    return allc


def bench_jacobian(args, c, wl, prec, x, w, G, state, tuned):
    """Full Jacobian (B, M, |Theta|): the forward once, then one adjoint pass
    per observable.  Timed against one forward and one backward (VJP) pass of
    the same configuration: the ratio to M backward passes says what sharing
    psi across the M bras could at most save."""
    import torch
    import workloads as W
    import paper_2404_06314_amd as q

    def timed(fn, reps):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    M = wl.circuit.n_obs
    if args.jac_chunk:
        c.set_option(q.QTM_OPT_JAC_CHUNK, args.jac_chunk)
    fwd_ms = timed(lambda: c.forward(x, w, prec, state=state), args.steps)

    def vjp():
        c.forward(x, w, prec, state=state)
        c.backward(x, w, G, prec, state=state)

    step_ms = timed(vjp, args.steps)
    bwd_ms = step_ms - fwd_ms
    jac_ms = timed(lambda: c.jacobian(x, w, prec), max(1, args.steps // 4))
    log(f"jacobian: {jac_ms:.3f} ms; forward {fwd_ms:.3f} ms, backward {bwd_ms:.3f} ms, "
        f"M = {M}: {jac_ms / (M * bwd_ms):.3f} of M backward passes")
    out = {"metric": "full Jacobian (B, M, |Theta|) ms per batch", "value": round(jac_ms, 3),
           "unit": "ms", "higher_is_better": False, "n_gpus": 1, "dtype": prec, "data": "synthetic",
           "config": {"workload": W.WORKLOAD_NAMES[args.config], "batch": wl.batch, "observables": M,
                      "observables_per_pass": args.jac_chunk or "auto", "autotuned": tuned is not None},
           "forward_ms": round(fwd_ms, 3), "backward_ms": round(bwd_ms, 3),
           "ratio_to_M_backward": round(jac_ms / (M * bwd_ms), 4),
           "ratio_to_forward_plus_M_backward": round(jac_ms / (fwd_ms + M * bwd_ms), 4)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--precision", default=None, choices=[None, "c64", "c128"])
    ap.add_argument("--path", default="fused", choices=["fused", "plain"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--klo", type=int, default=0)
    ap.add_argument("--jit", type=int, default=1, choices=[0, 1],
                    help="1: sweep kernels specialised for the circuit at run time (QTM_OPT_JIT, "
                         "the default); 0: the compiled generic sweep kernels")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="1: run the autotuner (tile size, low qubits, generic/specialised) first; "
                         "its time is not part of the timed steps")
    ap.add_argument("--dense", type=int, default=0, choices=[0, 1],
                    help="1: complex64 forwards with the shared-weight dense blocks on the matrix cores "
                         "(QTM_OPT_DENSE_BLOCKS; layered CZ-chain circuits); implies --autotune 0")
    ap.add_argument("--greedy-plan", type=int, default=0, choices=[0, 1],
                    help="1: the greedy sweep plan for the specialised kernels (QTM_OPT_GREEDY_PLAN) "
                         "instead of the plan chosen for skipping zero tiles; implies --autotune 0")
    ap.add_argument("--plan-io", type=int, default=12,
                    help="HBM weight of a full-state sweep in the zero-skip planner's cost estimate "
                         "(QTM_OPT_PLAN_IO, 1..64); other than 12 implies --autotune 0")
    ap.add_argument("--renorm", type=int, default=0,
                    help="periodic renormalisation every R sweeps (QTM_OPT_RENORM); implies --autotune 0")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-gate complex128 step timed beside the fused one")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--cpu-samples", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--paper-sweep", default="", choices=["", "fig1", "fig2", "tab1", "all"],
                    help="time the paper's benchmark shapes (Eq. (7) ansatz with input scaling) "
                         "instead of the default workload; one JSON line per shape")
    ap.add_argument("--jacobian", action="store_true",
                    help="time the full Jacobian (qtm_jacobian) of the workload against one forward "
                         "and one backward pass; one JSON line")
    ap.add_argument("--jac-chunk", type=int, default=0,
                    help="with --jacobian: observables per adjoint pass (0: the library's choice)")
    ap.add_argument("--digest", default="",
                    help="print the digest of the sources of this kernel (traffic records refer to it)")
    args = ap.parse_args()
    if args.digest:
        print(kernel_digest(args.digest))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batch would be "
              "split across GPUs with one all-reduce of dL/dweights, which is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_2404_06314_amd as q

    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 copies of 1 GiB")
        return
    if args.paper_sweep:
        return bench_paper_shapes(args)
    if args.config == "c4":
        return bench_uneven(args)
    wl = W.config_workload(args.config)
    prec = args.precision or wl.meta["precision"]
    circ = wl.circuit
    c = q.Circuit.from_workload(circ)
    c.set_path(q.QTM_PATH_FUSED if args.path == "fused" else q.QTM_PATH_PLAIN)
    if args.tile:
        c.set_option(q.QTM_OPT_TILE_QUBITS, args.tile)
    if args.klo:
        c.set_option(q.QTM_OPT_LOW_QUBITS, args.klo)
    if args.jit and args.path == "fused":
        c.set_option(q.QTM_OPT_JIT, 1)
    if args.greedy_plan:
        args.autotune = 0
        c.set_option(q.QTM_OPT_GREEDY_PLAN, 1)
    if args.plan_io != 12:
        args.autotune = 0
        c.set_option(q.QTM_OPT_PLAN_IO, args.plan_io)
    if args.dense or args.renorm:
        args.autotune = 0
        c.set_option(q.QTM_OPT_DENSE_BLOCKS, args.dense)
        c.set_option(q.QTM_OPT_RENORM, args.renorm)
    tuned = None
    if args.autotune and args.path == "fused":
        os.environ.setdefault("QTM_AUTOTUNE_LOG", "1")  # progress: one line per candidate
        t0 = time.perf_counter()
        tuned = c.autotune(wl.batch, prec, cache=False)
        args.jit = tuned["jit"]
        args.greedy_plan = tuned.get("greedy", 0)
        args.plan_io = tuned.get("io", 12)
        log(f"autotune ({time.perf_counter() - t0:.1f} s): tile {tuned['tile']} klo {tuned['klo']} "
            f"jit {tuned['jit']} greedy plan {args.greedy_plan} plan io {args.plan_io} "
            f"({len(tuned['candidates'])} candidates)")
    dev = torch.device("cuda:0")
    x = torch.as_tensor(wl.inputs, device=dev)
    w = torch.as_tensor(wl.weights, device=dev)
    G = torch.as_tensor(wl.grad_out, device=dev)
    B = wl.batch
    state = c.alloc_state(B, prec)
    if args.jacobian:
        return bench_jacobian(args, c, wl, prec, x, w, G, state, tuned)
    log(f"workload {circ.name}: n={circ.n} gates={circ.n_gates} B={B} precision={prec} "
        f"path={args.path}")

    def step():
        c.forward(x, w, prec, state=state)
        c.backward(x, w, G, prec, state=state)

    t0 = time.perf_counter()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps, {time.perf_counter() - t0:.1f} s"
        f"{', including compiling the specialised kernels' if args.jit else ''})")

    c.set_option(q.QTM_OPT_TIMING, 1 if args.path == "fused" else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = B * args.steps / (t1 - t0)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} evals/s")

    roof = None
    plan_kt = plan_klo = None
    if args.path == "fused":
        pl = c.plan(prec)
        plan_kt, plan_klo = pl["kt"], pl["klo"]
    elem = 8 if prec == "c64" else 16
    if args.path == "fused":
        import ctypes
        lib = q._lib.load()
        plan = c.plan(prec)
        S = len(plan["sweeps"])
        res = {}
        for kind in (0, 1):
            ms = ctypes.c_double()
            nl = ctypes.c_int64()
            q._lib.check(lib.qtm_timing_read(c.handle, kind, ctypes.byref(ms), ctypes.byref(nl)))
            res[kind] = (ms.value, nl.value)
        c.set_option(q.QTM_OPT_TIMING, 0)
        kind = 1 if res[1][0] >= res[0][0] else 0
        ms_tot, launches = res[kind]
        use_jit = args.jit and args.path == "fused"
        dense_fwd = kind == 0 and args.dense and prec == "c64"
        # the specialised kernels' sweeps, and so their traffic, depend on the
        # sweep plan; the compiled ones always take the greedy plan
        plan_tag = ("greedy" if args.greedy_plan else f"io{args.plan_io}") if use_jit and not dense_fwd else ""
        avg_s = ms_tot / launches / 1e3
        if dense_fwd:
            # one pass per (layer, block of 4 qubits): the state read and
            # written once; a dense 32 x 32 real operator on every column of
            # 16 amplitudes (2048 flop)
            per_launch_bytes = B * (1 << circ.n) * elem * 2
            per_launch_flop = B * (1 << (circ.n - 4)) * 2048
            units = 0.0
        else:
            passes, units = live_work(plan, circ.n, kind, use_jit)
            bytes_per_step = B * (1 << circ.n) * elem * passes
            per_launch_bytes = bytes_per_step / S
            # algorithmic matrix-core work: every fused block is a 2x2 complex
            # gate on each of the B * 2^(n-1) pairs = 16 real MACs (32 flop) per
            # pair, applied to psi in the forward and un-applied on psi and
            # lambda in the backward (except each qubit's last block there),
            # over the tiles the kernels run (live_work)
            flop_step = int(B * (1 << (circ.n - 1)) * units * 32 * (2 if kind == 1 else 1))
            per_launch_flop = flop_step / S
        gbs = per_launch_bytes / avg_s / 1e9
        tfs = per_launch_flop / avg_s / 1e12
        sfx = f"_t{plan_kt}l{plan_klo}" + ("_c128" if prec == "c128" else "") + ("_rn" if args.renorm else "")
        name = "k_k9_pass" if dense_fwd else \
            (("qtm_jit_bwd" if kind == 1 else "qtm_jit_fwd") + sfx) if use_jit else \
            ("k_fused_bwd" if kind == 1 else "k_fused_fwd")
        if use_jit:
            for d in (0, 1):
                info = [c.jit_info(prec, d, s_) for s_ in range(S)]
                log(f"specialised {'bwd' if d else 'fwd'} kernels (VGPRs, scratch bytes): {info}")
        log(f"{name}: {launches} launches, avg {avg_s * 1e6:.1f} us, {per_launch_bytes / 1e6:.1f} MB "
            f"and {per_launch_flop / 1e9:.1f} GFLOP per launch -> {gbs:.1f} GB/s, {tfs:.2f} TFLOP/s; "
            f"fwd sweeps {res[0][0] / args.steps:.3f} ms/step, "
            f"bwd sweeps {res[1][0] / args.steps:.3f} ms/step ({S} sweeps)")
        # serial issue floor of the sweeps: matrix-core products at the FP32
        # matrix peak plus, in the backward, the transition-matrix FMAs (12
        # per amplitude pair and parameterised block, 24 flop) at the FP32
        # vector peak without packed math; gfx950 issues the two one after the
        # other within a wave
        gflop_step = B * (1 << (circ.n - 1)) * grad_units(plan, circ.n, use_jit) * 24 \
            if kind == 1 else 0.0
        floor_s = per_launch_flop / (MFMA_F32_PEAK_TFLOPS * 1e12) + \
            gflop_step / S / (VALU_F32_PEAK_TFLOPS * 1e12)
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(name, W.WORKLOAD_NAMES[args.config], plan_tag),
                "kernel": name, "avg_launch_us": round(avg_s * 1e6, 2),
                "bytes_per_launch": int(per_launch_bytes), "sweeps": S,
                "mfma": {"achieved": round(tfs, 3), "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tfs / MFMA_F32_PEAK_TFLOPS, 4), "flop_per_launch": int(per_launch_flop)},
                "issue": {"floor_us": round(floor_s * 1e6, 2), "frac": round(floor_s / avg_s, 4),
                          "valu_flop_per_launch": int(gflop_step / S)}}
        log(f"{name}: HBM {gbs / HBM_PEAK_GBS:.3f} of peak, matrix cores {tfs / MFMA_F32_PEAK_TFLOPS:.3f}, "
            f"serial issue floor {floor_s * 1e6:.1f} us ({floor_s / avg_s:.3f} of the launch)")

    # the plain per-sample complex128 form (one launch per gate) beside the
    # fused one: its step time, and how far the fused result is from it
    plain = None
    if args.path == "fused" and prec == "c64" and circ.n <= 20 and not args.no_plain:
        plain = plain_c128_beside(c, circ, x, w, G, state, B, prec, q)

    cpu = None
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        samples = args.cpu_samples or 3 * threads
        log(f"cpu baseline: oracle on {samples} samples with {threads} threads, then on one core ...")
        cpu = cpu_baselines(wl, threads, samples, samples_1=max(1, min(3, samples)))
        log(f"cpu baseline: {cpu['value']:.3f} evals/s on {threads} threads, "
            f"{cpu['single_core']['value']:.3f} on one core ({cpu['cpu_model']}, nproc {cpu['nproc']})")

    out = {
        "metric": METRIC if args.config == "c3" else f"circuit evals/s (fwd+adjoint grad) {circ.name}",
        "value": round(value, 2),
        "unit": "circuit evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": W.WORKLOAD_NAMES[args.config], "n_qubits": circ.n,
                   "layers": W.CONFIGS[args.config]["layers"],
                   "entangler": W.CONFIGS[args.config]["entangler"], "batch": B,
                   "observables": circ.n_obs, "precision": prec, "path": args.path,
                   "specialised_kernels": bool(args.jit and args.path == "fused"),
                   "tile_qubits": plan_kt, "low_qubits": plan_klo,
                   "sweep_plan": "greedy" if (args.greedy_plan or not args.jit) else f"zero-skip, io {args.plan_io}",
                   "autotuned": tuned is not None, "dense_blocks": bool(args.dense),
                   "renorm_period": args.renorm},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if plain is not None:
        out["plain_c128"] = plain
    print(json.dumps(out), flush=True)


def plain_c128_beside(c, circ, x, w, G, state, B, prec, q, steps=2):
    """One forward + VJP step of the plain per-gate complex128 kernels on the
    same inputs (timed over `steps` after one warm-up), and the largest
    differences of the fused result from it: absolute on <Z>, and per
    gradient vector relative to that vector's largest entry."""
    import torch
    cp = q.Circuit.from_workload(circ)
    cp.set_path(q.QTM_PATH_PLAIN)
    st = cp.alloc_state(B, "c128")

    def run(cc, p, s):
        ev = cc.forward(x, w, p, state=s)
        gw, gx = cc.backward(x, w, G, p, state=s)
        return ev, gw, gx

    ref = run(cp, "c128", st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run(cp, "c128", st)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    got = run(c, prec, state)
    torch.cuda.synchronize()
    ev_err = float((got[0] - ref[0]).abs().max())

    def rel(a, b):
        scale = float(b.abs().max()) if b.numel() else 0.0
        return float((a - b).abs().max()) / scale if scale > 0 else 0.0

    gx_err = max((rel(got[2][i], ref[2][i]) for i in range(B)), default=0.0) if got[2] is not None else None
    out = {"ms_per_step": round(ms, 2), "value": round(B / (ms / 1e3), 2), "unit": "circuit evals/s",
           "dtype": "c128", "path": "per-gate", "steps": steps,
           "fused_c64_max_abs_err_expval": ev_err, "fused_c64_max_rel_err_grad_w": rel(got[1], ref[1]),
           "fused_c64_max_rel_err_grad_x": gx_err}
    log(f"plain complex128 per-gate form: {ms:.1f} ms/step; fused complex64 against it: "
        f"<Z> {ev_err:.2e} abs, dL/dw {out['fused_c64_max_rel_err_grad_w']:.2e} rel, dL/dx {gx_err:.2e} rel")
    del st
    cp.close()
    return out


# The paper's benchmark shapes for its Eq. (7) ansatz (batch 48 throughout):
# Fig. 1 sweeps the qubit count at depth 3 with Z on every qubit, Fig. 2 the
# depth at 12 qubits, Tab. I the number of observables at 12 qubits, depth 3.
PAPER_SHAPES = {
    "fig1": [(n, 3, 48, n) for n in range(4, 19, 2)],
    "fig2": [(12, d, 48, 12) for d in range(1, 12)],
    "tab1": [(12, 3, 48, m) for m in (1, 2, 4, 8, 12, 16, 24, 32)],
}


def bench_paper_shapes(args):
    """Forward and adjoint-gradient times of the paper's ansatz at its own
    benchmark shapes (complex64, fused path, default tiles; the specialised
    kernels unless --jit 0).  Forward and backward are timed separately with
    events on the launch stream."""
    import torch
    import workloads as W
    import paper_2404_06314_amd as q

    sweeps = list(PAPER_SHAPES) if args.paper_sweep == "all" else [args.paper_sweep]
    prec = args.precision or "c64"
    dev = torch.device("cuda:0")
    for sw in sweeps:
        for i, (n, d, B, M) in enumerate(PAPER_SHAPES[sw]):
            wl = W.paper_workload(n, d, B, seed=500 + 37 * i + n, n_obs=M)
            c = q.Circuit.from_workload(wl.circuit)
            if args.jit:
                c.set_option(q.QTM_OPT_JIT, 1)
            x = torch.as_tensor(wl.inputs, device=dev)
            w = torch.as_tensor(wl.weights, device=dev)
            G = torch.as_tensor(wl.grad_out, device=dev)
            state = c.alloc_state(B, prec)
            for _ in range(max(args.warmup, 1)):
                c.forward(x, w, prec, state=state)
                c.backward(x, w, G, prec, state=state)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            tf = tb = 0.0
            for _ in range(args.steps):
                ev[0].record()
                c.forward(x, w, prec, state=state)
                ev[1].record()
                c.backward(x, w, G, prec, state=state)
                ev[2].record()
                ev[2].synchronize()
                tf += ev[0].elapsed_time(ev[1])
                tb += ev[1].elapsed_time(ev[2])
            tf /= args.steps
            tb /= args.steps
            # the same step captured once in a HIP graph and replayed: the
            # entry points only launch kernels once their workspaces exist,
            # so at these sizes the graph removes most of the launch cost
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                c.forward(x, w, prec, state=state)
                c.backward(x, w, G, prec, state=state)
            torch.cuda.current_stream().wait_stream(side)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                c.forward(x, w, prec, state=state)
                c.backward(x, w, G, prec, state=state)
            graph.replay()
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(args.steps):
                graph.replay()
            ev[1].record()
            ev[1].synchronize()
            tg = ev[0].elapsed_time(ev[1]) / args.steps
            line = {"sweep": sw, "n_qubits": n, "depth": d, "batch": B, "observables": M,
                    "parameters": wl.circuit.n_weights, "gates": wl.circuit.n_gates,
                    "ms_forward": round(tf, 4), "ms_backward": round(tb, 4),
                    "evals_per_s": round(B / ((tf + tb) / 1e3), 1),
                    "ms_step_graph": round(tg, 4), "evals_per_s_graph": round(B / (tg / 1e3), 1),
                    "dtype": prec, "specialised_kernels": bool(args.jit)}
            msg = ""
            if sw == "tab1":
                # the paper's reverse gradient returns the full Jacobian
                # (B, M, |Theta|): every observable in one adjoint pass (the
                # default at these sizes) against one pass per observable
                def jac_ms(k):
                    c.set_option(q.QTM_OPT_JAC_CHUNK, k)
                    for _ in range(max(args.warmup, 1)):
                        c.jacobian(x, w, prec)
                    torch.cuda.synchronize()
                    ev[0].record()
                    for _ in range(args.steps):
                        c.jacobian(x, w, prec)
                    ev[1].record()
                    ev[1].synchronize()
                    return ev[0].elapsed_time(ev[1]) / args.steps
                tj, tj1 = jac_ms(0), jac_ms(1)
                line["ms_jacobian"] = round(tj, 4)
                line["ms_jacobian_one_observable_per_pass"] = round(tj1, 4)
                msg = f"; Jacobian {tj:.3f} ms (one observable per pass: {tj1:.3f} ms)"
            print(json.dumps(line), flush=True)
            log(f"{sw} n={n} d={d} M={M}: fwd {tf:.3f} ms, bwd {tb:.3f} ms; graph-launched step {tg:.3f} ms{msg}")
            del graph
            c.close()


def bench_uneven(args):
    """1024 circuits (n 8..16, 2..10 layers, CNOT ring), one sample each, in one
    persistent kernel per direction.  The timed region launches the two HIP
    graphs; a second pass with per-kernel events (kernels launched one by one)
    gives the persistent kernels' durations for the roofline."""
    import ctypes
    import numpy as np
    import torch
    import workloads as W
    import paper_2404_06314_amd as q

    items = W.uneven_items(1024)
    circs = [q.Circuit.from_workload(wl.circuit) for wl in items]
    m = q.Multi(circs)
    dev = torch.device("cuda:0")
    cat = lambda k: torch.as_tensor(np.concatenate([getattr(wl, k).reshape(-1) for wl in items]),
                                    dtype=torch.float64, device=dev)
    x, w, G = cat("inputs"), cat("weights"), cat("grad_out")
    st = m.alloc_state()
    N = len(items)
    log(f"workload uneven batch: {N} circuits, n 8..16, 2..10 layers, ring; "
        f"state {m.state_bytes / 2**20:.1f} MiB")

    def step():
        m.forward(x, w, st)
        m.backward(x, w, G, st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps); units fwd {m.units(0)} bwd {m.units(1)}")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = N * args.steps / (t1 - t0)
    log(f"timed {args.steps} steps (graphs): {ms_per_step:.3f} ms/step, {value:.1f} circuits/s")

    m.set_timing(True)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    e1 = time.perf_counter()
    res = {k: m.timing_read(k) for k in (0, 1)}
    m.set_timing(False)
    kind = 1 if res[1][0] >= res[0][0] else 0
    ms_tot, launches = res[kind]
    avg_s = ms_tot / launches / 1e3
    # algorithmic matrix-core work, as for the batched path: 32 flop per pair
    # per fused block, on psi (forward) or psi and lambda (backward)
    flop = 0
    for c, wl in zip(circs, items):
        plan = c.plan("c64")
        flop += int((1 << (wl.circuit.n - 1)) * block_ops(plan, kind) * 32 * (2 if kind == 1 else 1))
    tfs = flop / avg_s / 1e12
    name = "k_multi_bwd" if kind == 1 else "k_multi_fwd"
    log(f"{name}: {launches} launches, avg {avg_s * 1e6:.1f} us, {flop / 1e9:.2f} GFLOP per launch "
        f"-> {tfs:.2f} TFLOP/s; eager pass {(e1 - e0) * 1e3 / args.steps:.3f} ms/step; "
        f"persistent fwd {res[0][0] / args.steps:.3f} ms, bwd {res[1][0] / args.steps:.3f} ms per step")
    roof = {"bound": "mfma", "achieved": round(tfs, 3), "peak": MFMA_F32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tfs / MFMA_F32_PEAK_TFLOPS, 4),
            "traffic": recorded_traffic(name, W.WORKLOAD_NAMES["c4"]),
            "kernel": name, "avg_launch_us": round(avg_s * 1e6, 2), "flop_per_launch": int(flop)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        oracle.build(force=False)
        ns = args.cpu_samples or N
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)

        def one(wl):
            oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out, threads=1)

        t0 = time.perf_counter()
        passes = 0
        with ThreadPoolExecutor(threads) as ex:
            # whole passes over the sample until about 10 s of work
            while passes < 20 and (passes == 0 or time.perf_counter() - t0 < 10.0):
                list(ex.map(one, items[:ns]))
                passes += 1
        dt = time.perf_counter() - t0
        cpu = {"value": passes * ns / dt, "unit": "circuit evals/s", "cores": threads, "kind": "oracle",
               "sample": f"{passes} passes over the first {ns} of the {N} circuits, forward + adjoint "
                         f"VJP in complex128, circuits spread over {threads} threads; {dt:.1f} s"}
        log(f"cpu baseline: {cpu['value']:.2f} evals/s")
    out = {
        "metric": "circuit evals/s (fwd+adjoint grad) uneven batch of 1024 circuits",
        "value": round(value, 2), "unit": "circuit evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": W.WORKLOAD_NAMES["c4"], "circuits": N, "precision": "c64",
                   "launch": "persistent kernels in HIP graphs"},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
