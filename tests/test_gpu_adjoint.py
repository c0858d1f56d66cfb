"""Adjoint gradients (through the C ABI) against the CPU oracle's
parameter-shift rule, which is exact for exp(-i theta P / 2) rotations."""
import json
import os

import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O

pytestmark = pytest.mark.gpu
# Bar on |gradient error| and |energy error| per unit of sum_k |c_k| (the
# Hamiltonian's coefficient 1-norm bounds |lambda| = |H psi|).  Measured
# over these tests: at most 1.8e-7 (complex64, 360 rotations in one pass)
# and 1.2e-15 (complex128); the bars are about ten times that.  (A
# worst-case estimate for complex64, sqrt(#gates) * 3 * 2^-24 relative error
# in each of psi and lambda, gives ~1e-5 at a thousand gates.)
GBAR = {"c128": 1e-14, "c64": 2e-6}
HERE = os.path.dirname(os.path.abspath(__file__))


def record(name, rec):
    """Measured gradient errors go to gpurun_out/ when that folder exists."""
    out = os.path.join(os.path.dirname(HERE), "gpurun_out")
    rec = {k: float(v) for k, v in rec.items()}
    print(name, json.dumps(rec), flush=True)
    if os.path.isdir(out):
        with open(os.path.join(out, "gradient_errors.jsonl"), "a") as f:
            f.write(json.dumps({"case": name, **rec}) + "\n")


def check_grad(name, dtype, ham, e, e_ref, g, g_ref):
    """Records and bounds the energy and gradient errors against the oracle."""
    de, dg = abs(e - e_ref), float(np.abs(np.asarray(g) - np.asarray(g_ref)).max())
    norm1 = sum(abs(c) for c, _ in ham)
    record(name, {"energy_err": de, "max_grad_err": dg, "coeff_l1": norm1,
                  "max_grad_err_per_l1": dg / norm1})
    assert de <= GBAR[dtype] * norm1, (name, de)
    assert dg <= GBAR[dtype] * norm1, (name, dg)


def State(*a, **k):
    from paper_1807_07914_amd import State as S
    return S(*a, **k)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,layers,mode", [(2, 2, "pergate"), (4, 2, "auto"), (7, 3, "fused"),
                                           (12, 2, "auto"), (15, 2, "auto")])
def test_adjoint_matches_parameter_shift(dtype, n, layers, mode):
    params, ham = qc.gradient_workload(n, layers, 900 + n)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    idx = qc.rot_ring_param_index(n, layers)
    s = State(n, dtype)
    e, g_ops = s.adjoint(build(params), ham, mode=mode)
    back = s.to_numpy()
    s.close()
    g = np.zeros(params.size)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    ref = O.param_shift_grad(build, params, ham, n)
    check_grad("ring_n%d_l%d_%s_%s" % (n, layers, mode, dtype), dtype, ham, e,
               O.energy(build, params, ham, n), g, ref)
    assert np.all(g_ops[idx < 0] == 0)
    # the sweep returns the state to its input |0...0>
    assert abs(back[0] - 1) < (1e-10 if dtype == "c128" else 1e-4)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_with_mixed_gates(dtype):
    # rotations interleaved with fixed gates of every other kind
    n = 6
    rng = np.random.default_rng(31)
    fixed = qc.random_ops(n, 30, 32, dense_k=(1, 2, 3, 4))
    nrot = 14
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
    ham = qc.random_hamiltonian(n, 10, 33)
    s = State(n, dtype)
    e, g_ops = s.adjoint(build(theta), ham)
    s.close()
    g = np.zeros(nrot)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    ref = O.param_shift_grad(build, theta, ham, n)
    check_grad("mixed_gates_%s" % dtype, dtype, ham, e, O.energy(build, theta, ham, n), g, ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_chains_and_sign_runs(dtype):
    # four one-qubit gates per qubit between entanglers (merged into one LDS
    # pass per qubit), CZ rings reaching qubits outside a tile, Z gates, and a
    # CZ that cancels one of the ring's
    n, layers = 14, 2
    rng = np.random.default_rng(41)
    nrot = n * 2 * layers
    theta = rng.uniform(-np.pi, np.pi, nrot)

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
    ham = qc.random_hamiltonian(n, 10, 43)
    s = State(n, dtype)
    e, g_ops = s.adjoint(ops, ham)
    back = s.to_numpy()
    s.close()
    g = np.zeros(nrot)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    ref = O.param_shift_grad(build, theta, ham, n)
    check_grad("chains_signs_%s" % dtype, dtype, ham, e, O.energy(build, theta, ham, n), g, ref)
    assert np.all(g_ops[idx < 0] == 0)
    assert abs(back[0] - 1) < (1e-10 if dtype == "c128" else 1e-4)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_energy_paths(dtype):
    # lambda = H psi by tile passes (every X mask fits a tile) or by the
    # gather kernel (an X string over 9 qubits above the tile's low ones):
    # both give the parameter-shift gradient and the oracle energy
    n, layers = 14, 1
    params = np.random.default_rng(51).uniform(0, 2 * np.pi, 3 * n * layers)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    idx = qc.rot_ring_param_index(n, layers)
    fits = qc.zz_chain(n) + [(0.3, (("X", 2), ("Y", 9))), (0.5, (("Y", 0), ("X", 4)))]
    wide = fits + [(0.2, tuple(("X", q) for q in range(4, 13)))]
    for ham in (fits, wide):
        s = State(n, dtype)
        e, g_ops = s.adjoint(build(params), ham)
        s.close()
        g = np.zeros(params.size)
        np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
        ref = O.param_shift_grad(build, params, ham, n)
        check_grad("energy_paths_%d_%s" % (len(ham), dtype), dtype, ham, e, O.energy(build, params, ham, n),
                   g, ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_pass_split_over_programs(dtype):
    # 360 rotations in one tile pass: split into programs of <= 256 slots
    n, layers = 6, 20
    params, ham = qc.gradient_workload(n, layers, 707)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    idx = qc.rot_ring_param_index(n, layers)
    s = State(n, dtype)
    e, g_ops = s.adjoint(build(params), ham)
    s.close()
    g = np.zeros(params.size)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    ref = O.param_shift_grad(build, params, ham, n)
    check_grad("split_programs_%s" % dtype, dtype, ham, e, O.energy(build, params, ham, n), g, ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_cnot_ladders(dtype):
    # HEA layers with CNOT ladders (planned as H CZ H in the sweep), 13 qubits
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
    ham = qc.random_hamiltonian(n, 6, 62)
    s = State(n, dtype)
    e, g_ops = s.adjoint(ops, ham)
    back = s.to_numpy()
    s.close()
    g = np.zeros(theta.size)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    ref = O.param_shift_grad(build, theta.ravel(), ham, n)
    check_grad("cnot_ladders_%s" % dtype, dtype, ham, e, O.energy(build, theta.ravel(), ham, n), g, ref)
    assert np.all(g_ops[idx < 0] == 0)
    assert abs(back[0] - 1) < (1e-10 if dtype == "c128" else 1e-4)


def test_autograd_function():
    import torch
    from paper_1807_07914_amd.autograd import expectation
    n, layers = 5, 2
    params, ham = qc.gradient_workload(n, layers, 77)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    idx = qc.rot_ring_param_index(n, layers)
    th = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    e = expectation(th, build, idx, n, ham, dtype="c128")
    (2.0 * e).backward()
    ref = O.param_shift_grad(build, params, ham, n)
    assert abs(e.item() - O.energy(build, params, ham, n)) < 1e-10
    assert np.abs(th.grad.numpy() - 2.0 * ref).max() < 1e-9


def test_autograd_forward_then_backward_from_the_output_state():
    # the forward pass applies the circuit only; backward sweeps back from
    # the output it left on the GPU.  14 qubits reach past one sweep tile.
    import torch
    from paper_1807_07914_amd.autograd import expectation
    n, layers = 14, 2
    params, ham = qc.gradient_workload(n, layers, 78)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    idx = qc.rot_ring_param_index(n, layers)
    ref = O.param_shift_grad(build, params, ham, n)
    e_ref = O.energy(build, params, ham, n)
    with torch.no_grad():  # a forward pass without a gradient
        e0 = expectation(torch.tensor(params), build, idx, n, ham)
    assert abs(e0.item() - e_ref) <= GBAR["c64"] * sum(abs(c) for c, _ in ham)
    s = State(n, "c64")  # a caller-provided state, reused by two steps
    for step in range(2):
        th = torch.tensor(params, dtype=torch.float64, requires_grad=True)
        e = expectation(th, build, idx, n, ham, dtype="c64", state=s)
        e.backward(retain_graph=True)
        check_grad("autograd_n14_step%d" % step, "c64", ham, e.item(), e_ref, th.grad.numpy(), ref)
        with pytest.raises(RuntimeError):  # a second backward of the same node
            e.backward()
    # the sweep left |0...0> behind
    back = s.to_numpy()
    s.close()
    assert abs(back[0] - 1) < 1e-4


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_adjoint_from_the_output_state(dtype):
    # qsv_adjoint on a state that already holds the circuit's output gives
    # what it gives when it applies the circuit itself
    n, layers = 9, 2
    params, ham = qc.gradient_workload(n, layers, 79)
    ops = qc.rot_ring_ansatz(n, params, layers)
    s = State(n, dtype)
    e1, g1 = s.adjoint(ops, ham)
    s.set_basis(0)  # the sweep's recomputed input is |0...0> only up to rounding
    s.apply_circuit(ops)
    e2, g2 = s.adjoint(ops, ham, state_is_output=True)
    back = s.to_numpy()
    s.close()
    assert abs(e1 - e2) <= 1e-12 and np.abs(g1 - g2).max() <= 1e-12
    assert abs(back[0] - 1) < (1e-10 if dtype == "c128" else 1e-4)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_gradient_workload_24q_against_golden(dtype):
    # 24 qubits, 6 layers of RX/RY/RZ + CZ ring (432 parameters); 16 of the
    # derivatives (every 27th: all layers, all three axes) by the oracle's
    # parameter shift and by its central finite differences
    path = os.path.join(HERE, "golden", "c5_gradients.json")
    gold = json.load(open(path))
    n, layers = gold["n"], gold["layers"]
    params, ham = qc.gradient_workload(n, layers, qc.SEEDS["c5"])
    idx = qc.rot_ring_param_index(n, layers)
    s = State(n, dtype)
    e, g_ops = s.adjoint(qc.rot_ring_ansatz(n, params, layers), ham)
    s.close()
    g = np.zeros(params.size)
    np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
    k = np.asarray(gold["indices"])
    d_ps = np.abs(g[k] - np.asarray(gold["grad"])).max()
    d_fd = np.abs(g[k] - np.asarray(gold["fd"])).max()
    record("c5_24q_golden_%s" % dtype, {"energy_err": abs(e - gold["energy"]), "max_err_vs_param_shift": d_ps,
                                        "max_err_vs_finite_diff": d_fd})
    bar = GBAR[dtype] * sum(abs(c) for c, _ in ham)
    assert len(k) == 16
    assert abs(e - gold["energy"]) <= bar
    assert d_ps <= bar, d_ps
    # finite differences carry their own O(h^2) and rounding error (~1e-10)
    assert d_fd <= bar + 1e-8, d_fd


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [6, 14])
def test_adjoint_at_zero_angles(dtype, n):
    # a rotation at angle 0 is the identity but has a nonzero derivative; the
    # usual VQE start has every angle at 0.  14 qubits reach past one sweep
    # tile, so CZs meet rotations on qubits outside a pass's tile too
    layers = 2
    params, ham = qc.gradient_workload(n, layers, 950 + n)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    idx = qc.rot_ring_param_index(n, layers)
    some = params.copy()
    some[::3] = 0.0
    for theta in (some, np.zeros_like(params)):
        s = State(n, dtype)
        e, g_ops = s.adjoint(build(theta), ham)
        s.close()
        g = np.zeros(theta.size)
        np.add.at(g, idx[idx >= 0], g_ops[idx >= 0])
        ref = O.param_shift_grad(build, theta, ham, n)
        assert np.abs(ref).max() > 0.1  # the zero-angle derivatives are not trivially 0
        check_grad("zero_angles_n%d_%s" % (n, dtype), dtype, ham, e, O.energy(build, theta, ham, n), g, ref)
