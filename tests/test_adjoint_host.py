"""CPU checks of the adjoint sweep's program encoding.

The adjoint emulator (tests/adjoint_emulator.py) decodes the exact programs
the library would upload for the sweep kernel (op records, CZ/Z sign runs,
register rounds of one-qubit gates, gradient slot maps, non-tile ops) and
applies them to complex128 vectors.  Its gradients must equal the oracle's
parameter-shift gradients and the sweep must return the state to its start,
for both precisions, including circuits wider than one sweep tile so that
operands outside the tile occur.
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O

import adjoint_emulator as AE

GTOL = {"c64": 2e-6, "c128": 1e-11}


def check(n, dtype, build, params, ham, idx, others_zero=True):
    ops = build(params)
    e, g_ops, back = AE.emulate(n, dtype, ops, ham)
    g = np.zeros(params.size)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    ref = O.param_shift_grad(build, params, ham, n)
    assert abs(e - O.energy(build, params, ham, n)) < 1e-12
    assert np.abs(g - ref).max() <= GTOL[dtype] * max(1, len(ham)), np.abs(g - ref).max()
    if others_zero:  # no other rotations in the circuit
        assert np.all(g_ops[idx < 0] == 0)
    assert abs(back[0] - 1) < 1e-6 and np.abs(back[1:]).max() < 1e-6


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,layers", [(5, 2), (8, 3)])
def test_rotation_ring(dtype, n, layers):
    params, ham = qc.gradient_workload(n, layers, 700 + n)
    idx = qc.rot_ring_param_index(n, layers)
    check(n, dtype, lambda p: qc.rot_ring_ansatz(n, p, layers), params, ham, idx)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_chains_and_sign_runs_beyond_a_tile(dtype):
    # 14 qubits > the sweep tile (12 / 11 qubits): CZ rings reach outside
    # qubits; four one-qubit gates per qubit between entanglers; Z gates; a
    # CZ that cancels one of the ring's
    n, layers = 14, 2
    rng = np.random.default_rng(41)
    theta = rng.uniform(-np.pi, np.pi, n * 2 * layers)

    def build(p):
        ops, k = [], 0
        for l in range(layers):
            for q in range(n):
                ops += [qc.op("H", q), qc.op("RZ", q, params=(p[k],)), qc.op("S", q),
                        qc.op("RX" if q % 2 else "RY", q, params=(p[k + 1],))]
                k += 2
            for q in range(n):
                ops.append(qc.op("CZ", q, (q + 1 + 5 * l) % n))
            ops += [qc.op("Z", q) for q in range(0, n, 3)]
            ops.append(qc.op("CZ", 0, n - 1))
        return ops

    ops = build(theta)
    idx = np.array([-1] * len(ops))
    k = 0
    for i, o in enumerate(ops):
        if o.name in ("RX", "RY", "RZ"):
            idx[i] = k
            k += 1
    check(n, dtype, build, theta, qc.random_hamiltonian(n, 8, 43), idx)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_mixed_gates(dtype):
    # rotations between fixed gates of every kind, including dense blocks
    # on up to 4 qubits
    n = 7
    rng = np.random.default_rng(31)
    fixed = qc.random_ops(n, 40, 32, dense_k=(1, 2, 3, 4))
    nrot = 16
    theta = rng.uniform(-np.pi, np.pi, nrot)
    slots = sorted(rng.choice(len(fixed) + nrot, nrot, replace=False))

    def build(p):
        ops, it_f, k = [], iter(fixed), 0
        for i in range(len(fixed) + nrot):
            if k < nrot and i == slots[k]:
                ops.append(qc.op(("RX", "RY", "RZ")[k % 3], k % n, params=(p[k],)))
                k += 1
            else:
                ops.append(next(it_f))
        return ops

    idx = np.array([-1] * (len(fixed) + nrot))
    for k, sl in enumerate(slots):
        idx[sl] = k
    # the fixed gates include rotations of their own, which get gradients too
    check(n, dtype, build, theta, qc.random_hamiltonian(n, 10, 33), idx, others_zero=False)


def test_program_uses_rounds_and_sign_runs():
    # the 24-qubit gradient workload's programs hold register rounds and
    # sign runs (mostly inside the rounds), not one record per gate (576 gates)
    n, layers = 24, 6
    params, _ = qc.gradient_workload(n, layers, qc.SEEDS["c5"])
    ops = qc.rot_ring_ansatz(n, params, layers)
    words, acts = AE.program(n, "c64", ops)
    kinds = {}
    for off in acts:
        assert off >= 0
        nops, roff = int(words[off + 3]), int(words[off + 5])
        r = off + roff
        for _ in range(nops):
            typ = int(words[r])
            kinds[typ] = kinds.get(typ, 0) + 1
            if typ == 6 and int(words[r + 1]):
                kinds["6+5"] = kinds.get("6+5", 0) + 1
            r += int(words[r + 3]) if typ == 6 else AE.REC_WORDS
    # 2: other diagonal gates (single CZs), 5: sign runs, 6: rounds, 7: phases
    # per tile (RZ on qubits outside a pass's tile, applied by the store);
    # "6+5": rounds that carry the sign run before them, applied at their load
    assert set(kinds) <= {2, 5, 6, 7, "6+5"} and kinds.get(6, 0) > 0, kinds
    assert kinds.get("6+5", 0) > 0 and kinds.get(5, 0) < kinds["6+5"], kinds
    assert kinds.get(7, 0) > 0 and kinds.get(2, 0) < kinds[7], kinds
    assert sum(kinds.values()) < len(ops) // 3, (kinds, len(ops))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_pass_with_more_rotations_than_slots(dtype):
    # 6 qubits fit one tile, so all 360 rotations fall in one pass: the
    # encoder splits it into programs of at most 256 gradient slots
    n, layers = 6, 20
    params, ham = qc.gradient_workload(n, layers, 707)
    idx = qc.rot_ring_param_index(n, layers)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    words, acts = AE.program(n, dtype, build(params))
    assert len(acts) >= 2 and all(int(words[a + 4]) <= 256 for a in acts)
    assert sum(int(words[a + 4]) for a in acts) == params.size
    check(n, dtype, build, params, ham, idx)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_cnot_ladders(dtype):
    # HEA layers (RY, RZ, CNOT ladder): the sweep plans each CNOT as H CZ H and
    # maps the gradient slots back to the listed rotations; 13 qubits so that
    # passes have qubits outside their tile
    n, layers = 13, 2
    theta = np.random.default_rng(61).uniform(0, 2 * np.pi, (layers, n, 2))
    build = lambda p: qc.hea_circuit(n, np.asarray(p).reshape(layers, n, 2), layers)
    ops = build(theta)
    idx = np.array([-1] * len(ops))
    k = 0
    for i, o in enumerate(ops):
        if o.name in ("RY", "RZ"):
            idx[i] = k
            k += 1
    check(n, dtype, build, theta.ravel(), qc.random_hamiltonian(n, 6, 62), idx)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,layers", [(6, 2), (14, 2)])
def test_zero_angles(dtype, n, layers):
    # a rotation at angle 0 is the identity but still has a gradient: the
    # sweep must keep its slot, and must not move a CZ past RX(0) / RY(0)
    # (their generators do not commute with CZ); every third angle is 0, and
    # the all-zero start of a VQE run is checked as well
    params, ham = qc.gradient_workload(n, layers, 900 + n)
    idx = qc.rot_ring_param_index(n, layers)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    some = params.copy()
    some[::3] = 0.0
    check(n, dtype, build, some, ham, idx)
    check(n, dtype, build, np.zeros_like(params), ham, idx)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_zero_angle_between_czs(dtype):
    # RX(0) and RY(0) between two CZs on their qubit: joining the CZs into one
    # sign run would move the second CZ past the rotation's generator
    n = 7
    theta = np.array([0.0, 0.0, 0.4, 0.0, 0.0, 0.0])

    def build(p):
        ops = [qc.op("H", q) for q in range(n)]
        ops += [qc.op("CZ", 0, 1), qc.op("RX", 1, params=(p[0],)), qc.op("CZ", 1, 2),
                qc.op("RY", 2, params=(p[1],)), qc.op("CZ", 2, 0), qc.op("RZ", 0, params=(p[2],)),
                qc.op("CZ", 0, 3), qc.op("RY", 3, params=(p[3],)), qc.op("CZ", 3, 4),
                qc.op("RX", 4, params=(p[4],)), qc.op("CZ", 4, 5), qc.op("RZ", 5, params=(p[5],)),
                qc.op("CZ", 5, 6)]
        return ops

    ops = build(theta)
    idx = np.array([-1] * len(ops))
    k = 0
    for i, o in enumerate(ops):
        if o.name in ("RX", "RY", "RZ"):
            idx[i] = k
            k += 1
    ham = [(1.0, (("X", 1),)), (0.8, (("Y", 2),)), (0.6, (("X", 3), ("Z", 4))), (0.5, (("Y", 4),)),
           (0.3, (("Z", 0), ("Z", 6)))]
    check(n, dtype, build, theta, ham, idx)
