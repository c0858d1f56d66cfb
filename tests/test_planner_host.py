"""CPU checks of the fused planner and its program encoding.

The tile-program emulator (tests/tile_emulator.py) decodes the exact words
the library would upload for the tile kernel; its output must match the CPU
oracle for every circuit family, both precisions and several tile sizes.
Pass counts are checked to be below the gate counts (fusion happens) and
stable for a fixed structure.
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O
from paper_1807_07914_amd import qsv

import tile_emulator as E

TOL = {"c64": 2e-6, "c128": 1e-13}


def families(n, seed):
    rng = np.random.default_rng(seed)
    return {
        "random": qc.random_ops(n, 50, seed, dense_k=(1, 2, 3)),
        "brickwork": qc.random_brickwork(n, 5, seed),
        "rounds": qc.paper_rounds(n, 3, seed),
        "qft": qc.qft(n),
        "hea": qc.hea_circuit(n, rng.uniform(0, 2 * np.pi, (3, n, 2)), layers=3),
        "rotring": qc.rot_ring_ansatz(n, rng.uniform(0, 2 * np.pi, 2 * 3 * n), 2),
        "ghz": qc.ghz(n),
        "cz_mesh": qc.cz_mesh(n, 4, seed),
    }


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,tile", [(5, 0), (7, 6), (9, 7)])
def test_emulated_fused_plans_match_oracle(dtype, n, tile):
    psi0 = qc.random_state(n, 3 + n)
    for name, ops in families(n, 11 + n).items():
        ref = O.run(ops, n, psi=psi0.copy())
        got = E.emulate(n, dtype, ops, psi0, tile)
        assert np.abs(got - ref).max() <= TOL[dtype], name


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 2e-6)])
def test_emulated_deep_circuit_one_pass(dtype, tol):
    # 290 gates in one tile pass (10 qubits, depth 20): every scale factor the
    # planner defers must stay well conditioned over the whole pass
    n = 10
    ops = qc.random_brickwork(n, 20, qc.SEEDS["c1"])
    psi0 = np.zeros(1 << n, dtype=complex)
    psi0[0] = 1.0
    ref = O.run(ops, n)
    got = E.emulate(n, dtype, ops, psi0)
    assert np.abs(got - ref).max() <= tol


def test_pass_counts_fuse_gates():
    ops = qc.random_brickwork(28, 40, qc.SEEDS["c2"])
    a = qsv.plan_info(28, "c64", ops)
    b = qsv.plan_info(28, "c64", ops)
    assert a == b and a["separate_ops"] == 0
    assert a["passes"] <= 40
    assert qsv.plan_info(30, "c64", qc.qft(30))["passes"] <= 8
    # a circuit that fits one tile is a single pass
    assert qsv.plan_info(10, "c128", qc.random_brickwork(10, 20, 1))["passes"] == 1


def test_plan_info_rejects_bad_input():
    with pytest.raises(qsv.QsvError):
        qsv.plan_info(4, "c64", [qc.op("H", 4)])
    with pytest.raises(qsv.QsvError):
        qsv.plan_info(10, "c64", qc.ghz(10), tile_qubits=20)


def _algebra_family(n, seed):
    """Gates that exercise the planner's diagonal bookkeeping: scaled and
    non-unitary 2x2 matrices, projectors, anti-diagonal gates, and general
    2-qubit diagonals with and without zero entries, on every kind of qubit
    (register, free and outside a tile)."""
    rng = np.random.default_rng(seed)
    cplx = lambda *s: rng.normal(size=s) + 1j * rng.normal(size=s)
    ops = []
    for _ in range(60):
        kind = int(rng.integers(0, 11))
        q = [int(x) for x in rng.permutation(n)[:2]]
        if kind == 0:
            ops.append(qc.op("U", q[0], mat=qc.haar_unitary(1, rng) * rng.uniform(0.5, 2.0)))
        elif kind == 1:
            ops.append(qc.op("U", q[0], mat=cplx(2, 2)))
        elif kind == 2:
            ops.append(qc.op("U", q[0], mat=np.diag([1.0, 0.0]).astype(complex)))
        elif kind == 3:
            ops.append(qc.op("U", q[0], mat=np.array([[0, 1], [1, 0]]) * np.exp(1j * rng.uniform(0, 6, (2, 2)))))
        elif kind == 4:
            ops.append(qc.op("U", *q, mat=np.diag(np.exp(1j * rng.uniform(0, 6, 4)))))
        elif kind == 5:
            d = cplx(4)
            d[int(rng.integers(0, 4))] = 0.0
            ops.append(qc.op("U", *q, mat=np.diag(d)))
        elif kind == 6:
            ops.append(qc.op("U", q[0], mat=np.diag(cplx(2))))
        elif kind == 7:
            ops.append(qc.op("CPHASE", *q, params=(float(rng.uniform(-3, 3)),)))
        elif kind == 8:
            ops.append(qc.op(("CZ", "CNOT", "SWAP")[int(rng.integers(0, 3))], *q))
        elif kind == 9:
            ops.append(qc.op(("RZ", "RX", "RY")[int(rng.integers(0, 3))], q[0],
                             params=(float(rng.uniform(-3, 3)),)))
        else:
            ops.append(qc.op(("H", "S", "T", "Z", "X", "Y")[int(rng.integers(0, 6))], q[0]))
    return ops


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,tile,seed", [(6, 5, 1), (7, 6, 2), (9, 7, 3), (9, 6, 4)])
def test_emulated_gate_algebra_edge_cases(dtype, n, tile, seed):
    ops = _algebra_family(n, 100 + seed)
    psi0 = qc.random_state(n, 7 + seed)
    ref = O.run(ops, n, psi=psi0.copy())
    got = E.emulate(n, dtype, ops, psi0, tile)
    scale = max(1.0, float(np.abs(ref).max()))
    assert np.abs(got - ref).max() <= TOL[dtype] * 10 * scale


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,tile,seed", [(8, 6, 1), (11, 7, 2), (12, 12, 3)])
def test_emulated_cnot_store_maps(dtype, n, tile, seed):
    # CNOTs between qubits at every kind of tile position (register bits,
    # free bits, controls outside the tile), full ladders, and phases carried
    # on a target up to its CNOT: the rounds' store maps apply them all
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(5):
        for q in range(n):
            ops.append(qc.op("RZ", q, params=(float(rng.uniform(-3, 3)),)))
            if rng.random() < 0.6:
                ops.append(qc.op("RY", q, params=(float(rng.uniform(-3, 3)),)))
        ops += [qc.op("CNOT", q, q + 1) for q in range(n - 1)]
        for _ in range(n):
            a, b = (int(x) for x in rng.permutation(n)[:2])
            ops.append(qc.op("CNOT", a, b))
        ops.append(qc.op("T", int(rng.integers(n))))
    words, steps = E.program(n, dtype, ops, tile)
    counts = E.op_counts(words, steps, dtype)
    assert counts.get("maps", 0) > 0 and counts.get("separate", 0) == 0, counts
    psi0 = qc.random_state(n, 40 + seed)
    ref = O.run(ops, n, psi=psi0.copy())
    got = E.emulate(n, dtype, ops, psi0, tile)
    assert np.abs(got - ref).max() <= TOL[dtype]


def test_cnot_ladders_take_no_layers():
    # the paper's round family: each round's CNOT ladder is applied by store
    # maps, so the plan has no more layers than rotation levels need
    n = 16
    ops = qc.paper_rounds(n, 4, 5)
    words, steps = E.program(n, "c64", ops, 12)
    counts = E.op_counts(words, steps, "c64")
    ncnot = sum(o.name == "CNOT" for o in ops)
    assert counts.get("maps", 0) > 0 and counts.get("CZR", 0) == 0 and counts.get("CZF", 0) == 0, counts
    assert counts["layers"] < ncnot, (counts, ncnot)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_emulated_sign_steps(dtype):
    # CZs between every kind of qubit position (register, free, outside):
    # pair negations, conditional Zs and group parities all appear and
    # match the oracle
    n, tile = 11, 7
    allcz = [qc.op("CZ", i, j) for i in range(n) for j in range(i + 1, n)]
    ops = allcz + qc.cz_mesh(n, 4, 31) + allcz
    psi0 = qc.random_state(n, 32)
    words, steps = E.program(n, dtype, ops, tile)
    counts = E.op_counts(words, steps, dtype)
    assert counts.get("CZR", 0) > 0 and counts.get("CZF", 0) > 0 and counts.get("SIGN", 0) > 0, counts
    ref = O.run(ops, n, psi=psi0.copy())
    got = E.emulate(n, dtype, ops, psi0, tile)
    assert np.abs(got - ref).max() <= TOL[dtype]


def test_givens_split_counts():
    """Unitary 2x2 gates become real rotations (shears), pure phases are
    carried (no step of their own), and diagonal factors are applied in bulk:
    one table per layer of rotations at most."""
    n = 12
    ops = qc.random_brickwork(n, 8, 5)
    words, steps = E.program(n, "c64", ops)
    counts = E.op_counts(words, steps, "c64")
    n_u1 = sum(1 for o in ops if o.name == "U")
    # consecutive 2x2 gates on one qubit are multiplied first, so there are
    # at most as many rotations as 2x2 gates
    assert n_u1 // 2 < counts.get("ROT", 0) <= n_u1
    assert counts.get("U1", 0) == 0 and counts.get("RAWD", 0) == 0
    assert counts.get("TAB", 0) < n_u1 // 2
    assert counts["layers"] < n_u1 // 2
    rz = [qc.op("RZ", q, params=(0.3 * q + 0.1,)) for q in range(n)]
    words, steps = E.program(n, "c64", rz)
    counts = E.op_counts(words, steps, "c64")
    assert counts.get("ROT", 0) == 0 and counts.get("RAWD", 0) == 0


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_zero_angles_keep_the_plan(dtype):
    # rotations are planned by gate, not by angle value: a batch built at
    # angle 0 (the usual start of a parameter sweep) has the passes of one
    # built at random angles, so an update between them keeps its structure;
    # the zero-angle programs still give the oracle's states
    widths = [6, 11, 14]
    rng = np.random.default_rng(77)
    zero = [qc.hea_circuit(w, np.zeros((3, w, 2)), layers=3) for w in widths]
    rand = [qc.hea_circuit(w, rng.uniform(0, 2 * np.pi, (3, w, 2)), layers=3) for w in widths]
    w0, p0, j0 = E.batch_program(dtype, zero, widths, 0)
    w1, p1, j1 = E.batch_program(dtype, rand, widths, 0)
    assert len(p0) == len(p1) and np.array_equal(j0, j1)
    for i, w in enumerate(widths):
        job = next(j for j in j0 if int(j[0]) == w)
        got = E.emulate_batch_job(dtype, w0, p0, job)
        ref = O.run(zero[i], w)
        assert np.abs(got - ref).max() <= TOL[dtype]


def swap_network(n, layers, seed):
    """RY layers, CZ on neighbours and a random perfect matching of SWAPs per
    layer: the SWAPs cross tile boundaries."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(layers):
        for q in range(n):
            ops.append(qc.op("RY", q, params=(float(rng.uniform(0, 2 * np.pi)),)))
        for q in range(0, n - 1, 2):
            ops.append(qc.op("CZ", q, q + 1))
        perm = rng.permutation(n)
        for k in range(0, n - 1, 2):
            ops.append(qc.op("SWAP", int(perm[k]), int(perm[k + 1])))
    return ops


def plan_kinds(n, dtype, ops, tile=0):
    words, steps = E.program(n, dtype, ops, tile)
    return "".join("P" if E.is_qperm(words, int(s)) else ("T" if s >= 0 else "X") for s in steps)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,tile,seed", [(8, 6, 0), (8, 6, 1), (9, 6, 2), (10, 7, 0), (11, 6, 1), (12, 7, 2)])
def test_emulated_swap_relabeling(dtype, n, tile, seed):
    # plans that relabel SWAPs away and end in one (an involution) or two
    # qubit-permutation passes, against the oracle; a three-qubit matrix
    # after the SWAPs checks that separate ops are relabeled too
    ops = swap_network(n, 3, seed)
    ops.append(qc.op("U", 0, n - 1, 2, mat=qc.haar_unitary(3, np.random.default_rng(seed))))
    ops += swap_network(n, 1, seed + 10)
    kinds = plan_kinds(n, dtype, ops, tile)
    assert "P" in kinds and kinds.endswith("P") and kinds.count("P") <= 2, kinds
    psi0 = qc.random_state(n, 40 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    got = E.emulate(n, dtype, ops, psi0, tile)
    assert np.abs(got - ref).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype,n,tile", [("c64", 9, 6), ("c128", 10, 6), ("c64", 12, 7)])
def test_emulated_qft_one_permutation_pass(dtype, n, tile):
    # the QFT's final SWAPs form an involution (bit reversal): one pass
    ops = qc.qft(n)
    kinds = plan_kinds(n, dtype, ops, tile)
    assert kinds.endswith("P") and kinds.count("P") == 1, kinds
    psi0 = qc.random_state(n, 77 + n)
    got = E.emulate(n, dtype, ops, psi0, tile)
    assert np.abs(got - O.run(ops, n, psi=psi0.copy())).max() <= TOL[dtype]


def test_relabeling_only_when_it_saves_passes():
    # a SWAP inside the register group costs nothing in a pass: no relabeling
    n = 10
    ops = qc.random_brickwork(n, 4, 3) + [qc.op("SWAP", 0, 1)] + qc.random_brickwork(n, 2, 4)
    assert "P" not in plan_kinds(n, "c64", ops)
    # the 30-qubit QFT: three tile passes and the bit reversal
    assert plan_kinds(30, "c64", qc.qft(30)) == "TTTP"
    assert qsv.plan_info(30, "c64", qc.qft(30))["passes"] == 4


@pytest.mark.parametrize("dtype,n", [("c64", 13), ("c128", 12)])
def test_emulated_lane_tables_full_tile(dtype, n):
    # a full tile has 8 free bits, so the per-group phase steps' lane tables
    # use both of their 16-entry halves; the plan must take that form
    ops = qc.qft(n) + qc.random_brickwork(n, 2, 91)
    words, steps = E.program(n, dtype, ops)
    W = [int(x) for x in words]
    nlane = 0
    for s in steps:
        if s >= 0 and not E.is_qperm(words, int(s)):
            blocks = E._round_blocks(W, int(s), W[s], W[s + 2])
            nlane += W[blocks[0] + E.LANE_TAB_N_HDR] if blocks else 0
    assert nlane >= 64
    psi0 = qc.random_state(n, 300 + n)
    got = E.emulate(n, dtype, ops, psi0)
    assert np.abs(got - O.run(ops, n, psi=psi0.copy())).max() <= TOL[dtype]


def test_environment_switches_read_again_after_reload():
    # QSV_SEGMENT_QUBITS is read at first use; the debug export
    # qsv_debug_reload_env makes the library read it again (and drops the
    # schedule cache): the 30-qubit QFT needs 5 passes with 5 segment qubits
    # and 4 with 4 (the planner's own choice)
    import os
    L = qsv.lib()
    ops = qc.qft(30)
    old = os.environ.get("QSV_SEGMENT_QUBITS")
    try:
        got = {}
        for v in ("5", "4", None):
            if v is None:
                os.environ.pop("QSV_SEGMENT_QUBITS", None)
            else:
                os.environ["QSV_SEGMENT_QUBITS"] = v
            assert L.qsv_debug_reload_env() == 0
            got[v] = qsv.plan_info(30, "c64", ops)["passes"]
        assert got["5"] > got["4"] and got[None] == min(got["5"], got["4"])
    finally:
        if old is None:
            os.environ.pop("QSV_SEGMENT_QUBITS", None)
        else:
            os.environ["QSV_SEGMENT_QUBITS"] = old
        L.qsv_debug_reload_env()
