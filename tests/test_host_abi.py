"""CPU tests of the C ABI: the library loads, exports every declared symbol,
and its host-side logic (validation, state sizes, options, the fused-path
planner) behaves.  No compute call is made here (no GPU in this suite)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtm.h")


@pytest.fixture(scope="module")
def qtm():
    import paper_2404_06314_amd as q
    q._lib.load()
    return q


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qtm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(qtm):
    lib = qtm._lib.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in qtm._lib.SIGNATURES, f"binding lacks {n}"
    assert lib.qtm_version().decode().startswith("qtm")


def make(qtm, n, gates, n_in=0, n_w=0, masks=(1,)):
    g = np.asarray(gates, dtype=np.int32).reshape(-1, 5)
    return qtm.Circuit(n, g, n_in, n_w, np.asarray(masks, dtype=np.uint64))


@pytest.mark.parametrize("n,gates,n_in,n_w,masks,code", [
    (31, [], 0, 0, [1], -2),                                   # too many qubits
    (0, [], 0, 0, [1], -1),
    (2, [[0, 2, 0, 2, 0]], 0, 1, [1], -1),                     # qubit out of range
    (2, [[3, 1, 1, 0, 0]], 0, 0, [1], -1),                     # control == target
    (2, [[4, 0, 5, 0, 0]], 0, 0, [1], -1),                     # CZ qubit out of range
    (2, [[1, 0, 0, 2, 3]], 0, 3, [1], -1),                     # weight index out of range
    (2, [[0, 0, 0, 1, 1]], 1, 0, [1], -1),                     # input index out of range
    (2, [[0, 0, 0, 0, 0]], 1, 0, [1], -1),                     # rotation without source
    (2, [[1, 0, 2, 3, 0]], 1, 2, [1], -1),                     # scaled: weight slot out of range
    (2, [[1, 0, 0, 3, 1]], 1, 2, [1], -1),                     # scaled: input slot out of range
    (2, [[1, 0, -1, 3, 0]], 1, 2, [1], -1),                    # scaled: negative weight slot
    (2, [[17, 0, 1, 0, 0]], 0, 0, [1], -2),                    # unknown gate type
    (2, [[5, 2, 0, 0, 0]], 0, 0, [1], -1),                     # fixed gate qubit out of range
    (2, [[14, 0, 0, 2, 0]], 0, 1, [1], -1),                    # controlled rotation, control == target
    (2, [[15, 0, 2, 2, 0]], 0, 1, [1], -1),                    # controlled rotation, target out of range
    (2, [[16, 0, 1, 3, 0]], 1, 1, [1], -1),                    # controlled rotation with a scaled input
    (2, [[14, 0, 1, 2, 1]], 0, 1, [1], -1),                    # controlled rotation, weight out of range
    (2, [], 0, 0, [4], -1),                                    # mask bit >= n
    (2, [], 0, 0, [], -1),                                     # no observable
])
def test_validation_errors(qtm, n, gates, n_in, n_w, masks, code):
    with pytest.raises(qtm.QtmError) as ei:
        make(qtm, n, gates, n_in, n_w, masks)
    assert ei.value.code == code
    assert qtm._lib.load().qtm_last_error().decode()


def test_state_bytes_and_options(qtm):
    c = qtm.Circuit.from_workload(W.config_workload("c3").circuit)
    assert c.state_bytes(64, "c64") == 64 * (1 << 20) * 8
    assert c.state_bytes(3, "c128") == 3 * (1 << 20) * 16
    with pytest.raises(qtm.QtmError):
        c.state_bytes(0, "c64")
    with pytest.raises(qtm.QtmError):
        c.set_option(qtm.QTM_OPT_TILE_QUBITS, 13)
    with pytest.raises(qtm.QtmError):
        c.set_option(99, 1)
    c.set_option(qtm.QTM_OPT_TILE_QUBITS, 10)
    c.set_path(qtm.QTM_PATH_PLAIN)
    # renormalisation period: 0 (off) .. 1024
    for bad in (-1, 1025):
        with pytest.raises(qtm.QtmError):
            c.set_option(qtm.QTM_OPT_RENORM, bad)
    c.set_option(qtm.QTM_OPT_RENORM, 3)
    c.set_option(qtm.QTM_OPT_RENORM, 0)


def test_dense_blocks_option_checks_the_circuit_form(qtm):
    """QTM_OPT_DENSE_BLOCKS is accepted for layered RX / RY / RZ / CZ-chain
    circuits of 12, 16, ... qubits only (host check, no device)."""
    qtm.Circuit.from_workload(W.layered_circuit(12, 2, "ladder")).set_option(qtm.QTM_OPT_DENSE_BLOCKS, 1)
    qtm.Circuit.from_workload(W.config_workload("c3").circuit).set_option(qtm.QTM_OPT_DENSE_BLOCKS, 1)
    for circ in (W.layered_circuit(12, 2, "ring"), W.layered_circuit(10, 2, "ladder"),
                 W.layered_circuit(8, 2, "ladder"), W.config_workload("c2").circuit):
        c = qtm.Circuit.from_workload(circ)
        with pytest.raises(qtm.QtmError) as e:
            c.set_option(qtm.QTM_OPT_DENSE_BLOCKS, 1)
        assert e.value.code == -2
        c.set_option(qtm.QTM_OPT_DENSE_BLOCKS, 0)


def test_renormalising_sweeps_compile_without_a_device(qtm):
    """With QTM_OPT_RENORM the specialised kernels are generated per period
    (a kernel-name suffix): the sweeps that rescale read the norm records of
    the sweeps before them, the sweeps before a rescaling one write theirs."""
    c = qtm.Circuit.from_workload(W.layered_circuit(14, 8, "ring"))
    c.set_option(qtm.QTM_OPT_TILE_QUBITS, 10)
    S = len(c.plan("c64")["sweeps"])
    assert S >= 4
    c.set_option(qtm.QTM_OPT_RENORM, 2)
    for s in range(S):
        f = c.jit_source("c64", 0, s)
        assert "qtm_jit_fwd_t10l5_rn" in f
        assert ("a.rn_prev" in f) == (s > 0 and s % 2 == 0), s
        assert ("a.rn_out" in f) == (s + 1 < S and (s + 1) % 2 == 0), s
        bw = c.jit_source("c64", 1, s)
        assert ("rn_bwd_ratio" in bw) == (s > 0 and s % 2 == 0), s
        assert ("a.rn_rec +" in bw) == (s < S - 1), s
    c.jit_compile("c64")
    c.set_option(qtm.QTM_OPT_RENORM, 0)
    assert "rn_" not in c.jit_source("c64", 0, 2)


def test_null_pointer_errors_do_not_touch_the_gpu(qtm):
    c = qtm.Circuit.from_workload(W.config_workload("c1").circuit)
    lib = qtm._lib.load()
    # expvals NULL -> invalid argument before any device call
    rc = lib.qtm_forward(c.handle, 2, 0, None, None, None, None, None)
    assert rc == qtm._lib.QTM_ERR_INVALID_ARG
    rc = lib.qtm_backward(c.handle, 2, 0, None, None, None, None, None, None, None)
    assert rc == qtm._lib.QTM_ERR_INVALID_ARG
    rc = lib.qtm_forward(c.handle, 0, 0, None, None, None, None, None)
    assert rc == qtm._lib.QTM_ERR_INVALID_ARG
    # the no-allocation forward needs expvals and state
    rc = lib.qtm_forward_noalloc(c.handle, 2, 0, None, None, None, None, None)
    assert rc == qtm._lib.QTM_ERR_INVALID_ARG
    # norms: NULL output, then no forward has run on the handle
    assert lib.qtm_forward_norms(c.handle, 2, None, None) == qtm._lib.QTM_ERR_INVALID_ARG
    assert lib.qtm_forward_norms(c.handle, 2, ctypes.c_void_p(8), None) == qtm._lib.QTM_ERR_STATE
    c.set_option(qtm.QTM_OPT_CHECK_ANGLES, 1)
    c.set_option(qtm.QTM_OPT_CHECK_ANGLES, 0)


def _plan_gate_order(plan):
    order = []
    for sw in plan["sweeps"]:
        for st in sw["stages"]:
            order.extend(st["gates"])
    return order


def _check_plan(qtm, circ, precision="c64", tile=None, klo=None, batch=2, seed=0, zero_skip=False):
    c = qtm.Circuit.from_workload(circ)
    if tile:
        c.set_option(qtm.QTM_OPT_TILE_QUBITS, tile)
    if klo:
        c.set_option(qtm.QTM_OPT_LOW_QUBITS, klo)
    if zero_skip:
        # plans for the specialised kernels, which skip all-zero tiles
        c.set_option(qtm.QTM_OPT_JIT, 1)
    plan = c.plan(precision)
    assert "error" not in plan
    order = _plan_gate_order(plan)
    assert sorted(order) == list(range(circ.n_gates))
    for sw in plan["sweeps"]:
        assert len(sw["tile"]) == plan["kt"]
        assert sw["tile"][:plan["klo"]] == list(range(plan["klo"]))
    # executing the gates in plan order gives the same results (oracle)
    rng = np.random.default_rng(seed)
    wl = W.random_workload(rng, circ, batch)
    re = W.Circuit(n=circ.n, gates=circ.gates[order], n_inputs=circ.n_inputs,
                   n_weights=circ.n_weights, masks=circ.masks)
    a = oracle.vjp(circ, wl.inputs, wl.weights, wl.grad_out)
    b = oracle.vjp(re, wl.inputs, wl.weights, wl.grad_out)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, atol=1e-11)
    return plan


@pytest.mark.parametrize("zero_skip", [False, True])
@pytest.mark.parametrize("name", ["c1", "c2"])
def test_plan_reorders_only_commuting_gates(qtm, name, zero_skip):
    _check_plan(qtm, W.config_workload(name).circuit, zero_skip=zero_skip)


@pytest.mark.parametrize("zero_skip", [False, True])
@pytest.mark.parametrize("n,L,ent,tile,klo", [(10, 3, "ring", 6, 3), (9, 2, "ladder", 5, 2),
                                              (11, 2, "ring", 7, 5), (8, 4, "ladder", 4, 4)])
def test_plan_multi_sweep_small(qtm, n, L, ent, tile, klo, zero_skip):
    plan = _check_plan(qtm, W.layered_circuit(n, L, ent), tile=tile, klo=klo, zero_skip=zero_skip)
    assert len(plan["sweeps"]) >= 2


@pytest.mark.parametrize("zero_skip", [False, True])
def test_plan_random_circuits(qtm, zero_skip):
    rng = np.random.default_rng(5)
    for n in (4, 5, 7, 9):
        for _ in range(4):
            circ = W.random_circuit(rng, n, 40)
            _check_plan(qtm, circ, tile=4 if n > 4 else None, klo=2, seed=n, zero_skip=zero_skip)


def _live_blocks(plan, n):
    """Per sweep, the fraction of the tiles the specialised kernels run: those
    whose outer bits are 0 on every outer qubit not excited before the sweep."""
    out, ex = [], 0
    for sw, ex_after in zip(plan["sweeps"], plan["excited"]):
        tile = sum(1 << q for q in sw["tile"])
        outer_ex = bin(ex & ~tile & ((1 << n) - 1)).count("1")
        out.append(2.0 ** (outer_ex - (n - plan["kt"])))
        ex = ex_after
    return out


@pytest.mark.parametrize("klo", [4, 5])
def test_zero_skip_plan_for_the_n20_ladder(qtm, klo):
    """With the specialised kernels on, the n = 20, 8-layer CZ-ladder circuit
    is planned for skipping all-zero tiles: it runs fewer blocks over the
    whole state and fewer tile-weighted blocks than the greedy plan, still
    schedules every gate once in an order the oracle agrees with, and
    QTM_OPT_GREEDY_PLAN restores the greedy plan."""
    import bench
    circ = W.config_workload("c3").circuit
    plans = {}
    for mode in ("greedy", "zero", "forced"):
        c = qtm.Circuit.from_workload(circ)
        c.set_option(qtm.QTM_OPT_TILE_QUBITS, 12)
        c.set_option(qtm.QTM_OPT_LOW_QUBITS, klo)
        if mode != "greedy":
            c.set_option(qtm.QTM_OPT_JIT, 1)
        if mode == "forced":
            c.set_option(qtm.QTM_OPT_GREEDY_PLAN, 1)
        plans[mode] = c.plan("c64")
    g, z = plans["greedy"], plans["zero"]
    assert [s["tile"] for s in plans["forced"]["sweeps"]] == [s["tile"] for s in g["sweeps"]]
    assert [s["tile"] for s in z["sweeps"]] != [s["tile"] for s in g["sweeps"]]
    order = _plan_gate_order(z)
    assert sorted(order) == list(range(circ.n_gates))
    stats = {}
    for name, p in (("greedy", g), ("zero", z)):
        blocks = bench._sweep_block_ops(p, 0, False)
        live = _live_blocks(p, circ.n)
        stats[name] = (sum(b for b, f in zip(blocks, live) if f == 1.0), sum(b * f for b, f in zip(blocks, live)))
    assert stats["zero"][0] < stats["greedy"][0], stats
    assert stats["zero"][1] < stats["greedy"][1], stats
    # the 36 blocks that depend on qubit 19's first gate (its light cone in
    # the ladder) are the least any plan must run over the whole state
    if klo == 4:
        assert stats["zero"][0] <= 36, stats


def test_plan_sizes_for_configs(qtm):
    """The n = 20 and n = 26 configurations plan into few sweeps."""
    for name, max_sweeps in (("c3", 12), ("c5", 36)):
        c = qtm.Circuit.from_workload(W.config_workload(name).circuit)
        plan = c.plan("c64")
        assert 1 <= len(plan["sweeps"]) <= max_sweeps, (name, len(plan["sweeps"]))


def test_specialised_kernels_compile_without_a_device(qtm):
    """The sweep kernels generated for a circuit compile with the runtime
    compiler on a host with no GPU (both precisions, CNOT ring and CZ
    ladder), and the generated source names the circuit's register bits as
    literals."""
    import workloads as W
    for ent in ("ring", "ladder"):
        circ = W.layered_circuit(6, 2, ent)
        c = qtm.Circuit.from_workload(circ)
        for prec in ("c64", "c128"):
            c.jit_compile(prec)
            src = c.jit_source(prec, 1, 0)
            assert "qtm_jit_bwd" in src and "u1_" in src


def test_last_forward_sweep_writes_expectations_only_for_single_tile_samples(qtm):
    """With one tile per sample the last specialised forward sweep divides by
    the norm and writes <Z_m> (and the norm into its partial row, for the
    norm diagnostics); with several it leaves per-workgroup partial rows of
    every sum for the reduction kernel (the n = 20 benchmark circuit)."""
    for n, tile, direct in ((8, 8, True), (12, 12, True), (12, 10, False), (20, 12, False)):
        c = qtm.Circuit.from_workload(W.layered_circuit(n, 2, "ladder"))
        c.set_option(qtm.QTM_OPT_TILE_QUBITS, tile)
        last = len(c.plan("c64")["sweeps"]) - 1
        src = c.jit_source("c64", 0, last)
        assert ("a.out[" in src) == direct, (n, tile)
        assert "a.part_obs[" in src, (n, tile)
        assert ("else a.part_obs[" in src) == direct, (n, tile)
        # earlier sweeps never write observables
        if last > 0:
            assert "a.out[" not in c.jit_source("c64", 0, 0)


def test_paper_ansatz_plans_and_compiles(qtm):
    """The paper's ansatz (weight-scaled inputs) plans like any circuit: the
    plan's gate order gives the oracle's results, and its specialised
    kernels compile without a device."""
    for ent in ("chain", "ring"):
        circ = W.paper_ansatz(9, 2, ent)
        _check_plan(qtm, circ, tile=5, klo=2)
    c = qtm.Circuit.from_workload(W.paper_ansatz(12, 3))
    c.jit_compile("c64")


def test_fixed_gates_fuse_into_blocks_and_controlled_rotations_stay_per_gate(qtm):
    """Fixed one-qubit gates plan like rotations (the plan's gate order gives
    the oracle's results); a circuit with a controlled rotation has no fused
    plan and reports why."""
    rng = np.random.default_rng(3)
    g = W.random_circuit(rng, 6, 50, extended=0.5)
    fixed_only = W.Circuit(n=6, gates=g.gates[[int(t) not in W.CONTROLLED_TYPES for t in g.gates[:, 0]]],
                           n_inputs=g.n_inputs, n_weights=g.n_weights, masks=g.masks)
    assert any(int(t) in W.FIXED_TYPES for t in fixed_only.gates[:, 0])
    _check_plan(qtm, fixed_only, tile=4, klo=2)
    with_cr = W.Circuit(n=6, gates=np.concatenate([fixed_only.gates, [[W.CRY, 1, 4, W.SRC_WEIGHT, 0]]]).astype(np.int32),
                        n_inputs=g.n_inputs, n_weights=g.n_weights, masks=g.masks)
    c = qtm.Circuit.from_workload(with_cr)
    with pytest.raises(qtm.QtmError) as ei:
        c.plan("c64")
    assert ei.value.code == -2 and "per-gate" in str(ei.value)


def test_missing_library_raises_instead_of_falling_back(qtm, monkeypatch, tmp_path):
    # No CPU path exists behind the binding: without the shared library the
    # loader raises, and so does every compute entry point that needs it.
    monkeypatch.setattr(qtm._lib, "_lib", None)
    monkeypatch.setattr(qtm._lib, "LIB_PATH", tmp_path / "libqtm.so")
    with pytest.raises(ImportError, match="no CPU fallback"):
        qtm._lib.load()
    wl = W.config_workload("c1")
    with pytest.raises(ImportError):
        qtm.Circuit.from_workload(wl.circuit)


def test_plan_io_option(qtm):
    """QTM_OPT_PLAN_IO (the weight of a full-state sweep's HBM traffic in the
    zero-skip planner's cost estimate) accepts 1..64; every weight gives a
    plan that schedules each gate once, and at n = 20 a heavier weight gives
    no more sweeps than a lighter one."""
    import ctypes
    circ = W.config_workload("c3").circuit
    sweeps = {}
    for io in (1, 8, 12, 16, 64):
        c = qtm.Circuit.from_workload(circ)
        c.set_option(qtm.QTM_OPT_TILE_QUBITS, 12)
        c.set_option(qtm.QTM_OPT_LOW_QUBITS, 4)
        c.set_option(qtm.QTM_OPT_JIT, 1)
        c.set_option(qtm.QTM_OPT_PLAN_IO, io)
        p = c.plan("c64")
        assert sorted(_plan_gate_order(p)) == list(range(circ.n_gates))
        sweeps[io] = len(p["sweeps"])
    assert sweeps[16] <= sweeps[8] <= sweeps[1], sweeps
    lib = qtm._lib.load()
    c = qtm.Circuit.from_workload(circ)
    for bad in (0, 65, -3):
        assert lib.qtm_set_option(c.handle, qtm.QTM_OPT_PLAN_IO, bad) == qtm._lib.QTM_ERR_INVALID_ARG


def test_jac_chunk_option(qtm):
    """QTM_OPT_JAC_CHUNK (observables per adjoint pass of qtm_jacobian)
    accepts 0 (automatic) to 65535 and refuses anything else."""
    circ = W.config_workload("c1").circuit
    lib = qtm._lib.load()
    c = qtm.Circuit.from_workload(circ)
    for good in (0, 1, 7, 65535):
        assert lib.qtm_set_option(c.handle, qtm.QTM_OPT_JAC_CHUNK, good) == 0
    for bad in (-1, 65536):
        assert lib.qtm_set_option(c.handle, qtm.QTM_OPT_JAC_CHUNK, bad) == qtm._lib.QTM_ERR_INVALID_ARG
