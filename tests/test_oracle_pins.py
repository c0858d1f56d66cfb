"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
independent of the oracle's own code paths.

* gate matrices: algebraic identities (unitarity, H^2 = I, R_P(pi) = -iP,
  R_P(2 pi) = -I, dR/dtheta = -(i/2) P R, XY = iZ, CNOT = (I x H) CZ (I x H)
  with the control listed first, SWAP = three CNOTs, CPHASE(pi) = CZ);
* gate application and index conventions: brute-force Kronecker unitaries for
  n <= 6 (a second construction route), basis-state actions;
* closed forms: GHZ amplitudes, the QFT of a basis state, the paper's H2
  ansatz expectation values (section V.B) on its 100-point grid;
* the paper's entanglement claim for its random "rounds" family
  (section V.A): Schmidt rank across every line cut <= 2^rounds (= 4 for two);
* invariants: norm preservation, mirror echo C^dag C |x> = |x>;
* reductions: expectation values against Kronecker Pauli matrices, sampling
  against an independent search over the cumulative distribution;
* gradients: parameter shift against central finite differences.
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import brute
from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")

NAMED1 = ["I", "X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ"]
NAMED2 = ["CNOT", "CZ", "CPHASE", "SWAP"]
X = np.array([[0, 1], [1, 0]], complex)
Y = np.array([[0, -1j], [1j, 0]], complex)
Z = np.array([[1, 0], [0, -1]], complex)
I2 = np.eye(2)


def M(name, *p):
    return O.gate_matrix(name, p)


def matrix_of(o):
    return o.mat if o.name == "U" else O.gate_matrix(o.name, o.params)


# ---------------------------------------------------------------- gate table
@pytest.mark.parametrize("name", NAMED1 + NAMED2)
@pytest.mark.parametrize("theta", [0.0, 0.37, -2.1, 5.9])
def test_gates_unitary(name, theta):
    U = M(name, theta)
    assert np.abs(U.conj().T @ U - np.eye(U.shape[0])).max() < 1e-15


def test_pauli_and_clifford_identities():
    assert np.allclose(M("X"), X, atol=0) and np.allclose(M("Y"), Y, atol=0)
    assert np.allclose(M("Z"), Z, atol=0)
    assert np.abs(M("X") @ M("Y") - 1j * M("Z")).max() < 1e-15
    H = M("H")
    assert np.abs(H @ H - I2).max() < 1e-15
    assert np.abs(H @ M("Z") @ H - M("X")).max() < 1e-15
    assert np.abs(M("S") @ M("S") - M("Z")).max() < 1e-15
    assert np.abs(M("T") @ M("T") - M("S")).max() < 1e-15
    assert np.abs(M("S") @ M("SDG") - I2).max() < 1e-15
    assert np.abs(M("T") @ M("TDG") - I2).max() < 1e-15


@pytest.mark.parametrize("name,P", [("RX", X), ("RY", Y), ("RZ", Z)])
def test_rotation_convention(name, P):
    # R_P(pi) = -i P and R_P(2 pi) = -I fix the half-angle and the sign
    assert np.abs(M(name, np.pi) - (-1j) * P).max() < 1e-15
    assert np.abs(M(name, 2 * np.pi) + I2).max() < 1e-15
    # composition and derivative dR/dtheta = -(i/2) P R(theta)
    a, b = 0.731, -1.93
    assert np.abs(M(name, a) @ M(name, b) - M(name, a + b)).max() < 1e-15
    h = 1e-6
    d = (M(name, a + h) - M(name, a - h)) / (2 * h)
    assert np.abs(d - (-0.5j) * P @ M(name, a)).max() < 1e-9


def test_two_qubit_conventions():
    # control listed first: CNOT(0,1) maps |q1 q0> = |01> (index 1) to |11> (3)
    for c, t in [(0, 1), (1, 0)]:
        psi = O.zero_state(2, 1 << c)
        O.apply(psi, 2, qc.op("CNOT", c, t))
        assert abs(psi[(1 << c) | (1 << t)] - 1) < 1e-15
        psi = O.zero_state(2, 1 << t)          # control clear: no change
        O.apply(psi, 2, qc.op("CNOT", c, t))
        assert abs(psi[1 << t] - 1) < 1e-15
    # CNOT = (I x H_target) CZ (I x H_target)
    F = lambda qs, U: brute.full_operator(3, qs, U)
    for c, t in [(0, 2), (2, 1)]:
        lhs = F((c, t), M("CNOT"))
        rhs = F((t,), M("H")) @ F((c, t), M("CZ")) @ F((t,), M("H"))
        assert np.abs(lhs - rhs).max() < 1e-15
        sw = F((c, t), M("CNOT")) @ F((t, c), M("CNOT")) @ F((c, t), M("CNOT"))
        assert np.abs(F((c, t), M("SWAP")) - sw).max() < 1e-15
    assert np.abs(M("CPHASE", np.pi) - M("CZ")).max() < 1e-15
    # CZ and CPHASE are symmetric in their qubits
    assert np.abs(F((0, 2), M("CPHASE", 0.4)) - F((2, 0), M("CPHASE", 0.4))).max() < 1e-15


# ---------------------------------------------------- brute-force unitaries
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("seed", [11, 12])
def test_brute_force_random_circuits(n, seed):
    ops = qc.random_ops(n, 40, seed, dense_k=(1, 2, 3))
    U = brute.circuit_unitary(n, ops, matrix_of)
    for x0 in (0, (1 << n) - 1, (5 * seed) % (1 << n)):
        psi = O.run(ops, n, x0=x0)
        assert np.abs(psi - U[:, x0]).max() < 1e-13


@pytest.mark.parametrize("k", [4, 5, 6])
def test_brute_force_dense_blocks(k):
    n = 6
    rng = np.random.default_rng(k)
    U = qc.haar_unitary(k, rng)
    qs = tuple(int(q) for q in rng.permutation(n)[:k])
    psi0 = O.run(qc.random_ops(n, 20, 5), n)
    psi = psi0.copy()
    O.apply_matrix(psi, n, qs, U)
    assert np.abs(psi - brute.full_operator(n, qs, U) @ psi0).max() < 1e-13


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("n", [1, 2, 5, 12])
def test_ghz(n):
    psi = O.run(qc.ghz(n), n)
    ref = np.zeros(1 << n, complex)
    ref[0] = ref[-1] = 2 ** -0.5
    assert np.abs(psi - ref).max() < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 7, 10])
def test_qft_closed_form(n):
    N = 1 << n
    y = np.arange(N, dtype=np.int64)
    for x in {0, 1, N - 1, qc.qft_input(n, 1003)}:
        psi = O.run(qc.qft(n), n, x0=x)
        ref = np.exp(2j * np.pi * ((x * y) % N) / N) / np.sqrt(N)
        assert np.abs(psi - ref).max() < 1e-14


def test_h2_listing_closed_forms():
    # paper section V.B: with the listing's literal decimals the per-term
    # values equal the exact-pi closed forms to ~2.5e-10
    for t0 in qc.h2_sweep():
        psi = O.run(qc.h2_ansatz(t0), 2)
        v = {k: O.pauli_expval(psi, t) for k, t in qc.H2_TERMS.items()}
        ref = {"Z0": np.cos(t0), "Z1": -np.cos(t0), "Z0Z1": -1.0,
               "X0X1": -np.sin(t0), "Y0Y1": -np.sin(t0)}
        for key in ref:
            assert abs(v[key].real - ref[key]) < 1e-9, key
            assert abs(v[key].imag) < 1e-15


def test_h2_term_batch_basis_changes():
    # the batched sweep measures X0X1 and Y0Y1 as Z0Z1 after H (X) or S^dag
    # then H (Y) on both qubits: on the oracle every measured circuit gives
    # the closed form of its term
    circs, widths, hams, keys = qc.h2_term_batch(qc.h2_sweep())
    assert len(circs) == 500
    for c, w, h, (t0, key) in zip(circs, widths, hams, keys):
        v = O.expval(O.run(c, w), h)
        assert abs(v - qc.h2_closed_forms(t0)[key]) < 1e-9, (t0, key)


# ------------------------------------------------------ paper's chi claim
def schmidt_ranks(psi, n, tol=1e-10):
    out = []
    for cut in range(1, n):
        # rows: qubits >= cut, cols: qubits < cut
        m = psi.reshape(1 << (n - cut), 1 << cut)
        s = np.linalg.svd(m, compute_uv=False)
        out.append(int((s > tol * s[0]).sum()))
    return out


@pytest.mark.parametrize("rounds", [1, 2, 3, 4])
def test_paper_rounds_schmidt_bound(rounds):
    # section V.A: two rounds give a maximum bond dimension of 4 at any n;
    # each further round can at most double it
    best = 0
    for seed in range(6):
        psi = O.run(qc.paper_rounds(10, rounds, seed), 10)
        r = schmidt_ranks(psi, 10)
        assert max(r) <= 2 ** rounds
        best = max(best, max(r))
    if rounds == 2:
        assert best == 4


# ----------------------------------------------------------- invariants
@pytest.mark.parametrize("n", [3, 8, 11])
def test_norm_and_mirror_echo(n):
    ops = qc.random_ops(n, 60, 100 + n)
    x0 = (37 * n) % (1 << n)
    psi = O.run(ops, n, x0=x0)
    assert abs(O.norm(psi) - 1) < 1e-13
    back = O.run(qc.dagger(ops), n, psi=psi)
    ref = np.zeros(1 << n, complex); ref[x0] = 1
    assert np.abs(back - ref).max() < 1e-13


def test_norm_and_inner_sums():
    rng = np.random.default_rng(3)
    for n in (4, 13):
        a = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        b = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        assert abs(O.norm(a) - np.sum(np.abs(a) ** 2)) < 1e-9 * np.sum(np.abs(a) ** 2)
        assert abs(O.inner(a, b) - np.vdot(a, b)) < 1e-9 * np.abs(a).sum() * np.abs(b).max()


# --------------------------------------------------------- expectation
@pytest.mark.parametrize("n", [1, 3, 5])
def test_expval_against_kron_paulis(n):
    psi = O.run(qc.random_ops(n, 30, 7 + n), n)
    ham = qc.random_hamiltonian(n, 12, 9 + n)
    for (c, term), v in zip(ham, O.expval(psi, ham, per_term=True)):
        ref = np.vdot(psi, brute.pauli_operator(n, term) @ psi)
        assert abs(v - c * ref.real) < 1e-13
        assert abs(O.pauli_expval(psi, term) - ref) < 1e-13
    ref_total = sum(c * np.vdot(psi, brute.pauli_operator(n, t) @ psi).real for c, t in ham)
    assert abs(O.expval(psi, ham) - ref_total) < 1e-12


# ------------------------------------------------------------- sampling
def test_sample_inverse_cdf():
    n = 5
    psi = O.run(qc.random_ops(n, 25, 21), n)
    rng = np.random.default_rng(0)
    u = np.concatenate([[0.0, 1 - 2 ** -53], rng.random(4000)])
    got = O.sample(psi, u)
    C = np.cumsum(np.abs(psi) ** 2)
    ref = np.searchsorted(C, u * C[-1], side="right")
    ref = np.minimum(ref, np.flatnonzero(np.abs(psi) > 0).max())
    assert np.array_equal(got, ref.astype(np.uint64))


def test_sample_zero_probability_entries_never_drawn():
    psi = O.run(qc.ghz(6), 6)
    u = np.linspace(0, 1, 1001, endpoint=False)
    got = O.sample(psi, u)
    assert set(np.unique(got).tolist()) == {0, 63}
    C = np.cumsum(np.abs(psi) ** 2)
    assert (got == 0).sum() == (u * C[-1] < C[0]).sum() == 501


def test_sample_distribution_chi2():
    n = 3
    psi = O.run(qc.random_ops(n, 20, 4), n)
    p = np.abs(psi) ** 2
    u = np.random.default_rng(1).random(200000)
    counts = np.bincount(O.sample(psi, u).astype(np.int64), minlength=1 << n)
    chi2 = ((counts - p * u.size) ** 2 / (p * u.size)).sum()
    assert chi2 < 30  # 7 dof, p ~ 1e-4


def test_sample_rejects_bad_uniforms():
    psi = O.zero_state(2)
    with pytest.raises(ValueError):
        O.sample(psi, np.array([1.0]))
    with pytest.raises(ValueError):
        O.sample(psi, np.array([-0.1]))


# ------------------------------------------------------------ gradients
def test_param_shift_matches_finite_differences():
    n, layers = 4, 2
    params, ham = qc.gradient_workload(n, layers, 77)
    build = lambda p: qc.rot_ring_ansatz(n, p, layers)
    ps = O.param_shift_grad(build, params, ham, n)
    fd = O.finite_diff_grad(build, params, ham, n, h=1e-5)
    assert np.abs(ps - fd).max() < 1e-8
    assert np.abs(ps).max() > 1e-2


def test_c5_golden_parameter_shift_agrees_with_finite_differences():
    # the stored 24-qubit derivatives were written by the oracle by two
    # routes: the exact parameter-shift rule and central differences
    # (h = 1e-5, error O(h^2) plus rounding ~1e-11); they must agree
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_gradients.json")))
    assert len(gold["indices"]) == 16 and len(gold["grad"]) == 16 and len(gold["fd"]) == 16
    assert np.abs(np.asarray(gold["grad"]) - np.asarray(gold["fd"])).max() < 1e-9
    assert np.abs(np.asarray(gold["grad"])).max() > 0.1
