"""Batched persistent launch (through the C ABI) against the CPU oracle."""
import sys
import time

import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def Batch(*a, **k):
    from paper_1807_07914_amd import Batch as B
    return B(*a, **k)


def say(*a):
    print("[%s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def hea_subset(per_width=2, seed=qc.SEEDS["c4"], count=4096):
    b = qc.hea_batch(count, seed)
    picked = {}
    for i, w in enumerate(b.widths):
        picked.setdefault(int(w), [])
        if len(picked[int(w)]) < per_width:
            picked[int(w)].append(i)
    idx = sorted(i for v in picked.values() for i in v)
    return b, idx


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-4), ("c128", 1e-10)])
def test_hea_subset_covering_all_widths(dtype, tol):
    # 2 circuits of every width 8..20 drawn from the 4096-circuit batch
    b, idx = hea_subset()
    assert sorted({int(b.widths[i]) for i in idx}) == list(range(8, 21))
    circs = [b.circuit(i) for i in idx]
    hams = [b.hamiltonian(i) for i in idx]
    widths = [int(b.widths[i]) for i in idx]
    say("creating batch of", len(circs), dtype)
    bt = Batch(circs, widths, hams, dtype=dtype)
    say("created", bt.info())
    e = bt.run()
    e2 = bt.run()  # graph replay gives identical results
    say("ran twice")
    info = bt.info()
    bt.close()
    assert np.array_equal(e, e2)
    ref = np.array([O.expval(O.run(c, w), h) for c, w, h in zip(circs, widths, hams)])
    say("oracle done")
    assert np.abs(e - ref).max() <= tol, (np.abs(e - ref).max(), info)


@pytest.mark.parametrize("tile", [0, 11, 12])
def test_batch_matches_single_state_path(tile):
    from paper_1807_07914_amd import State
    b = qc.hea_batch(96, 1234, wmin=5, wmax=16)
    circs = [b.circuit(i) for i in range(96)]
    hams = [b.hamiltonian(i) for i in range(96)]
    widths = [int(w) for w in b.widths]
    bt = Batch(circs, widths, hams, dtype="c64", tile_qubits=tile)
    e = bt.run()
    bt.close()
    for i in range(0, 96, 7):
        s = State(widths[i], "c64")
        s.apply_circuit(circs[i])
        assert abs(s.expval(hams[i]) - e[i]) < 1e-4
        s.close()


def test_batch_update_and_general_z_strings():
    rng = np.random.default_rng(8)
    widths = [3, 6, 9, 14, 15]
    circs, hams = [], []
    for w in widths:
        circs.append(qc.random_ops(w, 40, 100 + w, dense_k=(1, 2)))
        terms = []
        for t in range(5):
            k = int(rng.integers(1, min(3, w) + 1))
            qs = rng.permutation(w)[:k]
            terms.append((float(rng.uniform(-1, 1)), tuple(("Z", int(q)) for q in qs)))
        hams.append(terms)
    bt = Batch(circs, widths, hams, dtype="c128")
    e = bt.run()
    ref = [O.expval(O.run(c, w), h) for c, w, h in zip(circs, widths, hams)]
    assert np.abs(e - ref).max() < 1e-10
    # same structure, new angles and matrices
    circs2 = []
    for c in circs:
        c2 = []
        for o in c:
            if o.params:
                c2.append(qc.op(o.name, *o.qubits, params=[p + 0.3 for p in o.params]))
            elif o.name == "U":
                c2.append(qc.op("U", *o.qubits, mat=o.mat.conj()))
            else:
                c2.append(o)
        circs2.append(c2)
    bt.update(circs2)
    e2 = bt.run()
    bt.close()
    ref2 = [O.expval(O.run(c, w), h) for c, w, h in zip(circs2, widths, hams)]
    assert np.abs(e2 - ref2).max() < 1e-10


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-4), ("c128", 1e-10)])
def test_batch_update_from_zero_angles(dtype, tol):
    # a sweep starts at angle 0: a batch built there accepts random angles and
    # the way back, each checked against the oracle
    widths = [5, 9, 13, 16]
    hams = [qc.zz_chain(w) for w in widths]
    rng = np.random.default_rng(5)
    zero = [qc.hea_circuit(w, np.zeros((4, w, 2)), layers=4) for w in widths]
    rand = [qc.hea_circuit(w, rng.uniform(0, 2 * np.pi, (4, w, 2)), layers=4) for w in widths]
    bt = Batch(zero, widths, hams, dtype=dtype)
    try:
        for circs in (zero, rand, zero):
            bt.update(circs)
            e = bt.run()
            ref = np.array([O.expval(O.run(c, w), h) for c, w, h in zip(circs, widths, hams)])
            assert np.abs(e - ref).max() <= tol, np.abs(e - ref).max()
    finally:
        bt.close()


def test_batch_rejects_unsupported():
    from paper_1807_07914_amd import QsvError
    with pytest.raises(ValueError):
        Batch([qc.ghz(4)], [4], [[(1.0, (("X", 0),))]])
    U = qc.haar_unitary(3, np.random.default_rng(0))
    with pytest.raises(QsvError):
        Batch([[qc.op("U", 0, 1, 2, mat=U)]], [6], [[(1.0, (("Z", 0),))]])


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-9)])
def test_h2_vqe_sweep_batched(dtype, tol):
    # the paper's VQE sweep (section V.B): 100 values of t0, five terms each,
    # one batched launch; X and Y terms through basis changes
    circs, widths, hams, keys = qc.h2_term_batch(qc.h2_sweep())
    bt = Batch(circs, widths, hams, dtype=dtype)
    e = bt.run()
    bt.close()
    assert len(e) == 500
    for v, (t0, key) in zip(e, keys):
        assert abs(v - qc.h2_closed_forms(t0)[key]) <= tol, (t0, key, v)
    # and against the oracle run of each measured circuit
    ref = np.array([O.expval(O.run(c, w), h) for c, w, h in zip(circs, widths, hams)])
    assert np.abs(e - ref).max() <= (1e-5 if dtype == "c64" else 1e-12)


def test_c4_full_batch_matches_pergate():
    # all 4096 circuits of the batched workload (widths 8..20) in one launch
    # against the per-gate kernels run circuit by circuit (complex64)
    from paper_1807_07914_amd import State
    b = qc.hea_batch(4096, qc.SEEDS["c4"])
    circs = [b.circuit(i) for i in range(4096)]
    hams = [b.hamiltonian(i) for i in range(4096)]
    widths = [int(w) for w in b.widths]
    say("creating the 4096-circuit batch")
    bt = Batch(circs, widths, hams, dtype="c64")
    e = bt.run()
    bt.close()
    say("batch done; per-gate reference")
    states = {w: State(w, "c64") for w in sorted(set(widths))}
    ref = np.empty(4096)
    for i in range(4096):
        s = states[widths[i]]
        s.set_basis(0)
        s.apply_circuit(circs[i], mode="pergate")
        ref[i] = s.expval(hams[i])
    for s in states.values():
        s.close()
    say("reference done")
    assert np.abs(e - ref).max() <= 1e-4


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-11)])
def test_batch_degenerate_circuits(dtype, tol):
    # widths 1..5 and beyond one tile, an empty circuit, a circuit without
    # Hamiltonian terms, and a batch of a single circuit
    rng = np.random.default_rng(77)
    widths = [1, 2, 3, 5, 14, 4, 15]
    circs = []
    for w in widths:
        names = [g for g in ("H", "RX", "RY", "RZ", "S", "CZ", "CNOT") if qc.GATE_ARITY[g] <= w]
        circs.append(qc.random_ops(w, 30, int(rng.integers(1 << 30)), names=names, dense_k=(1, 2) if w >= 2 else (1,)))
    circs[5] = []                                  # the empty circuit
    hams = [qc.zz_chain(w) if w >= 2 else [(0.5, (("Z", 0),))] for w in widths]
    hams[3] = []                                   # no terms: energy 0
    bt = Batch(circs, widths, hams, dtype=dtype)
    e = bt.run()
    bt.close()
    ref = np.array([O.expval(O.run(c, w), h) if h else 0.0 for c, w, h in zip(circs, widths, hams)])
    assert np.abs(e - ref).max() <= tol
    assert e[3] == 0.0 and abs(e[5] - (widths[5] - 1)) <= tol  # |0000>: every ZZ is +1
    bt1 = Batch(circs[4:5], widths[4:5], hams[4:5], dtype=dtype)
    e1 = bt1.run()
    bt1.close()
    assert abs(e1[0] - ref[4]) <= tol
