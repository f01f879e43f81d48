"""CPU emulation of the fused kernels' index arithmetic over the encoded
device program: every global address and LDS slot the kernels compute must
be in range and each stage's / load's mapping must be a permutation.  This
runs before any kernel is launched, so a layout bug cannot reach the GPU."""
import numpy as np
import pytest

import workloads as W

KREG = 4
SW_OUTER, SW_TILE, SW_LOADG, SW_LOADL, SW_LOADTB, SW_STAGES = 4, 34, 46, 62, 78, 90
ST_FLAGS, ST_THR, ST_LDS, ST_GLOB, ST_REGPOS, ST_OPS = 1, 2, 4, 20, 36, 40


def swz(i):
    return i ^ ((i >> 5) & 31) ^ ((i >> 10) & 31)


def insert_zeros(t, regpos):
    x = t.copy()
    for r in regpos:
        low = (1 << int(r)) - 1
        x = ((x & ~low) << 1) | (x & low)
    return x


def parity(v):
    return np.array([bin(int(a)).count("1") & 1 for a in np.ravel(v)]).reshape(np.shape(v))


def check_program(plan, n, circ=None):
    code = np.array(plan["code"], dtype=np.int64)
    thr = np.array(plan["thr"], dtype=np.int64)
    kt = plan["kt"]
    nt = 1 << (kt - KREG)
    t = np.arange(nt)
    rng = np.random.default_rng(0)
    for direction, offs in (("fwd", plan["sweep_off_fwd"]), ("bwd", plan["sweep_off_bwd"])):
        assert len(offs) == len(plan["sweeps"])
        for si, off in enumerate(offs):
            H = code[off:]
            nst, nout = int(H[0]), int(H[1])
            assert nout == n - kt
            outer = H[SW_OUTER:SW_OUTER + nout]
            tiles = np.arange(1 << nout)
            tbase = np.zeros_like(tiles)
            for i, pos in enumerate(outer):
                tbase |= ((tiles >> i) & 1) << int(pos)
            gload = np.zeros_like(t)
            for i in range(kt - KREG):
                gload |= ((t >> i) & 1) << int(H[SW_LOADTB + i])
            addrs = (tbase[:, None, None] | gload[None, :, None] |
                     H[SW_LOADG:SW_LOADG + 16][None, None, :])
            assert addrs.max() < (1 << n) and addrs.min() >= 0
            assert len(np.unique(addrs)) == 1 << n, "load addresses are not a permutation"
            lload = swz(t)[:, None] ^ H[SW_LOADL:SW_LOADL + 16][None, :]
            assert lload.max() < (1 << kt)
            assert len(np.unique(lload)) == 1 << kt
            tile_pos = H[SW_TILE:SW_TILE + kt]
            local_of = {}
            for tt in range(nt):
                for j in range(16):
                    local = tt + nt * j
                    g = 0
                    for k in range(kt):
                        if (local >> k) & 1:
                            g |= 1 << int(tile_pos[k])
                    local_of[swz(local)] = g
            sweep = plan["sweeps"][si if direction == "fwd" else len(offs) - 1 - si]
            for s in range(nst):
                S = code[int(H[SW_STAGES + s]):]
                regpos = S[ST_REGPOS:ST_REGPOS + 4]
                assert list(regpos) == sorted(regpos) and len(set(regpos)) == 4
                lt = insert_zeros(t, regpos)
                gt = thr[int(S[ST_THR]):int(S[ST_THR]) + nt]
                lidx = swz(lt)[:, None] ^ S[ST_LDS:ST_LDS + 16][None, :]
                assert lidx.max() < (1 << kt)
                assert len(np.unique(lidx)) == 1 << kt, "stage LDS slots not a permutation"
                gidx = gt[:, None] | S[ST_GLOB:ST_GLOB + 16][None, :]
                assert len(np.unique(gidx)) == 1 << kt
                assert np.all((gt[:, None] & S[ST_GLOB:ST_GLOB + 16][None, :]) == 0)
                for tt in range(nt):
                    for j in range(16):
                        assert local_of[int(lidx[tt, j])] == int(gidx[tt, j])
                nops = int(S[0])
                diag_recs = []
                for o in range(nops):
                    op = S[ST_OPS + 4 * o: ST_OPS + 4 * o + 4]
                    assert op[0] in (1, 2, 3) or op[0] == (4 if direction == "bwd" else 5)
                    if op[0] in (1, 4, 5):
                        assert 0 <= op[1] < 4 and 0 <= op[2] < plan["n_blocks"]
                    elif op[0] == 2:
                        assert 0 <= op[1] < 4 and op[2] in (0, 1)
                        assert (0 <= op[3] < 4 and op[3] != op[1]) if op[2] == 0 else 0 <= op[3] < n
                    else:
                        diag_recs.append(code[int(op[1]):])
                if circ is None or not diag_recs:
                    continue
                # CZ runs of this stage (forward order) -> diag records
                st_gates = sweep["stages"][s if direction == "fwd" else nst - 1 - s]["gates"]
                runs, cur = [], []
                for g in st_gates:
                    if circ.gates[g][0] == 4:
                        cur.append((int(circ.gates[g][1]), int(circ.gates[g][2])))
                    elif cur:
                        runs.append(cur)
                        cur = []
                if cur:
                    runs.append(cur)
                if direction == "bwd":
                    runs = [list(r) for r in reversed(runs)]
                assert len(runs) == len(diag_recs)
                W = S[ST_GLOB:ST_GLOB + 16]
                for pairs, rec in zip(runs, diag_recs):
                    ng = int(rec[0])
                    C = rec[1 + 2 * ng:1 + 2 * ng + 4]
                    qm = int(rec[1 + 2 * ng + 4])
                    for tb in rng.choice(tbase, size=min(3, len(tbase)), replace=False):
                        G = tb | gt
                        qg = np.zeros(nt, dtype=np.int64)
                        for g in range(ng):
                            d, m = int(rec[1 + 2 * g]), int(rec[2 + 2 * g])
                            qg ^= parity(G & (G >> d) & m)
                        for j in range(16):
                            x = G | W[j]
                            direct = np.zeros(nt, dtype=np.int64)
                            for a, b in pairs:
                                direct ^= ((x >> a) & (x >> b)) & 1
                            lin = np.zeros(nt, dtype=np.int64)
                            for b in range(4):
                                if (j >> b) & 1:
                                    lin ^= parity(G & int(C[b]))
                            rec_sign = qg ^ lin ^ ((qm >> j) & 1)
                            assert np.array_equal(direct, rec_sign), "diag sign decomposition"


@pytest.mark.parametrize("name,tile,klo,zero_skip", [("c1", 0, 0, 0), ("c2", 0, 0, 0), ("c3", 0, 0, 0),
                                                     ("c3", 10, 4, 0), ("c5", 0, 0, 0), ("c2", 0, 0, 1),
                                                     ("c3", 12, 4, 1), ("c3", 12, 3, 1)])
def test_program_layout_configs(name, tile, klo, zero_skip):
    import paper_2404_06314_amd as q
    wl = W.config_workload(name)
    c = q.Circuit.from_workload(wl.circuit)
    if tile:
        c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    if klo:
        c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    if zero_skip:
        c.set_option(q.QTM_OPT_JIT, 1)
    if name == "c5":
        pytest.skip("n = 26 emulation is too large for the CPU suite; covered by c3 layouts")
    check_program(c.plan("c64"), wl.circuit.n, wl.circuit)


@pytest.mark.parametrize("n,L,ent,tile,klo", [(6, 2, "ring", 4, 2), (9, 3, "ladder", 5, 3),
                                              (10, 2, "ring", 6, 4), (13, 2, "ring", 12, 5),
                                              (14, 3, "ladder", 8, 5), (11, 4, "ring", 7, 6)])
def test_program_layout_small(n, L, ent, tile, klo):
    import paper_2404_06314_amd as q
    c_w = W.layered_circuit(n, L, ent)
    c = q.Circuit.from_workload(c_w)
    c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    check_program(c.plan("c64"), n, c_w)


def test_program_layout_random():
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(9)
    for n in (4, 5, 6, 8):
        circ = W.random_circuit(rng, n, 60)
        c = q.Circuit.from_workload(circ)
        if n > 4:
            c.set_option(q.QTM_OPT_TILE_QUBITS, 4)
        c.set_option(q.QTM_OPT_LOW_QUBITS, 2)
        check_program(c.plan("c64"), n, circ)


def test_program_layout_empty_circuit():
    """A circuit without gates still gets one sweep with one stage (it must
    write |0...0> and read the observables)."""
    import paper_2404_06314_amd as q
    circ = W.Circuit(n=6, gates=np.zeros((0, 5), np.int32), n_inputs=0, n_weights=0,
                     masks=W.z_masks(6))
    plan = q.Circuit.from_workload(circ).plan("c64")
    assert len(plan["sweeps"]) == 1 and len(plan["sweeps"][0]["stages"]) == 1
    check_program(plan, 6, circ)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_last_op_per_qubit_is_marked_in_the_backward(seed):
    """The backward marks a fused block as T-only (op code 4) exactly when it
    is the first op on its qubit in the plan's execution order (the last the
    backward meets there); the forward marks the same blocks with op code 5
    (the |1> inputs of the gate are still 0)."""
    import paper_2404_06314_amd as qtm
    rng = np.random.default_rng(seed)
    for n in (5, 7, 9):
        circ = W.random_circuit(rng, n, 50, extended=0.2)
        circ = W.Circuit(n=n, gates=circ.gates[[int(t) not in W.CONTROLLED_TYPES for t in circ.gates[:, 0]]],
                         n_inputs=circ.n_inputs, n_weights=circ.n_weights, masks=circ.masks)
        c = qtm.Circuit.from_workload(circ)
        c.set_option(qtm.QTM_OPT_TILE_QUBITS, 4)
        c.set_option(qtm.QTM_OPT_LOW_QUBITS, 2)
        plan = c.plan("c64")
        code = np.array(plan["code"], dtype=np.int64)
        counts = {}
        for direction, offs, mark in (("fwd", plan["sweep_off_fwd"], 5), ("bwd", plan["sweep_off_bwd"], 4)):
            k = 0
            for off in offs:
                H = code[off:]
                for s in range(int(H[0])):
                    S = code[int(H[SW_STAGES + s]):]
                    for o in range(int(S[0])):
                        k += int(S[ST_OPS + 4 * o] == mark)
            counts[direction] = k
        order = [g for sw in plan["sweeps"] for st in sw["stages"] for g in st["gates"]]
        first = {}
        for g in order:
            t, q0, q1 = (int(v) for v in circ.gates[g][:3])
            for q in ((q0,) if t in W.PARAM_TYPES or t in W.FIXED_TYPES else (q0, q1)):
                first.setdefault(q, t)
        want = sum(1 for t in first.values() if t in W.PARAM_TYPES or t in W.FIXED_TYPES)
        assert counts["fwd"] == want and counts["bwd"] == want, (n, counts, want)


DIAGONAL_1Q = (W.RZ, W.Z, W.S, W.SDG, W.T, W.TDG)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_excited_qubits_per_sweep(seed):
    """Per sweep, the qubits excited by its end: those that were the target
    of a non-diagonal one-qubit gate or of a CNOT in it or an earlier sweep
    (a CZ, or a block of diagonal gates, keeps the |1> half of a qubit at 0).
    The masks are monotone, every qubit the circuit rotates off the diagonal
    is in the last one, and a qubit given only RZ and CZ never is."""
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(700 + seed)
    n = 9
    circ = W.random_circuit(rng, n, 60, extended=0.3)
    keep = [int(t) not in W.CONTROLLED_TYPES and not (int(t) not in DIAGONAL_1Q + (W.CZ,) and
                                                       (int(a) == 8 or (int(t) == W.CNOT and int(b) == 8)))
            for t, a, b in circ.gates[:, :3]]
    circ = W.Circuit(n=n, gates=circ.gates[keep], n_inputs=circ.n_inputs, n_weights=circ.n_weights,
                     masks=circ.masks)
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 5)
    c.set_option(q.QTM_OPT_LOW_QUBITS, 2)
    p = c.plan()
    ex = p["excited"]
    assert len(ex) == len(p["sweeps"])
    want, seen = 0, []
    for sw, got in zip(p["sweeps"], ex):
        for st in sw["stages"]:
            for gi in st["gates"]:
                t, a, b = (int(v) for v in circ.gates[gi, :3])
                if t == W.CNOT:
                    want |= 1 << b
                elif t != W.CZ and t not in DIAGONAL_1Q:
                    want |= 1 << a
        seen.append(want)
    # a block's gates are fused, so its qubit is excited if any of them is
    # off the diagonal: the per-gate reading above gives the same mask
    assert ex == seen
    assert all((x & y) == x for x, y in zip(ex, ex[1:]))
    assert not (ex[-1] >> 8) & 1


@pytest.mark.parametrize("name,tile,klo", [("c3", 11, 4), ("c3", 12, 5), ("c5", 12, 4)])
def test_bench_work_model(name, tile, klo):
    """bench.py's count of the work the sweeps do: the compiled kernels read
    and write every state once per sweep (the first forward sweep only
    writes, the last backward one only reads); the specialised kernels never
    move more and apply no more blocks, except the last block of each qubit
    they un-apply in sweeps after the first."""
    import bench
    import paper_2404_06314_amd as q
    wl = W.config_workload(name, batch=1)
    c = q.Circuit.from_workload(wl.circuit)
    c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    p = c.plan()
    S, n = len(p["sweeps"]), wl.circuit.n
    for kind in (0, 1):
        passes, units = bench.live_work(p, n, kind, False)
        assert passes == (1 + 2 * (S - 1) if kind == 0 else 3 + 4 * (S - 2) + 2)
        assert units == bench.block_ops(p, kind)
        lp, lu = bench.live_work(p, n, kind, True)
        assert 0 < lp <= passes
        extra = sum(bench._sweep_block_ops(p, kind, True)) - bench.block_ops(p, kind)
        assert 0 < lu <= units + extra


def test_bench_work_model_n20_tile11():
    """The n = 20 plan at tile 11 / 4 low qubits: qubits 11-19 are unexcited
    after sweep 0, 16-19 after sweeps 1 and 2, none after sweep 3.  So the
    forward writes 1/512, reads 1/512 and writes 1/16, reads and writes 1/16,
    reads 1/16 and writes all, reads and writes all: 3 + 4/16 + 2/512 state
    passes.  The backward reads psi in full and writes psi and lambda
    (sweep 4: 3), reads both in full and writes 2/16 (sweep 3), reads and
    writes 2/16 (sweep 2), reads 2/16 and writes 2/512 (sweep 1), reads
    2/512 (sweep 0): 5 + 8/16 + 4/512."""
    import bench
    import paper_2404_06314_amd as q
    wl = W.config_workload("c3", batch=1)
    c = q.Circuit.from_workload(wl.circuit)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 11)
    c.set_option(q.QTM_OPT_LOW_QUBITS, 4)
    p = c.plan()
    full = (1 << 20) - 1
    assert p["excited"] == [(1 << 11) - 1, (1 << 16) - 1, (1 << 16) - 1, full, full]
    fwd = (1 / 512) + (1 / 512 + 1 / 16) + (1 / 16 + 1 / 16) + (1 / 16 + 1) + (1 + 1)
    bwd = (1 + 2) + (2 + 2 / 16) + (2 / 16 + 2 / 16) + (2 / 16 + 2 / 512) + 2 / 512
    assert bench.live_work(p, 20, 0, True)[0] == pytest.approx(fwd)
    assert bench.live_work(p, 20, 1, True)[0] == pytest.approx(bwd)
