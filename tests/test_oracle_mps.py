"""Pins of the MPS oracle (oracle/mps.py) against what the paper and the
mathematics fix, independent of the oracle's own arithmetic:

- with no truncation the MPS holds the exact state: its contraction equals
  the state-vector oracle's result (itself pinned in test_oracle_pins.py) on
  random circuits with adjacent and distant two-qubit gates in both operand
  orders;
- the bond matrices are the Schmidt coefficients: the singular values of the
  state vector reshaped across each cut (a library SVD of a different matrix),
  and without truncation the bond dimension is that cut's numerical rank;
- GHZ and product states have the bond dimensions and coefficients of their
  closed forms, and the Bell pair its amplitudes;
- the paper's two-round random circuits keep chi <= 4 at any width
  (section V.A);
- a single truncation of a normalised state leaves norm^2 = the kept weight
  and <exact|truncated> = the kept weight (the Schmidt decomposition).
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import mps as M
from oracle import oracle as O


def schmidt_of_state(psi, n, b):
    """Singular values of psi across the cut between qubits < b and >= b."""
    mat = psi.reshape(1 << (n - b), 1 << b)   # row: qubits >= b, column: qubits < b
    s = np.linalg.svd(mat, compute_uv=False)
    return s[s > 1e-10 * s[0]]


def mixed_circuit(n, count, seed):
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(count):
        r = rng.random()
        if r < 0.4:
            g = ("H", "X", "Y", "S", "T", "RX", "RY", "RZ")[int(rng.integers(8))]
            q = int(rng.integers(n))
            ops.append(qc.op(g, q, params=(float(rng.uniform(0, 2 * np.pi)),) if g[0] == "R" else ()))
        else:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            g = ("CNOT", "CZ", "CPHASE", "SWAP", "U")[int(rng.integers(5))]
            if g == "U":
                ops.append(qc.op("U", a, b, mat=qc.haar_unitary(2, rng)))
            else:
                ops.append(qc.op(g, a, b, params=(float(rng.uniform(0, 2 * np.pi)),) if g == "CPHASE" else ()))
    return ops


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (5, 3), (7, 4), (9, 5)])
def test_exact_mps_equals_state_vector(n, seed):
    ops = mixed_circuit(n, 12 * n, seed)
    m = M.run(ops, n, cutoff=0.0)
    psi = O.run(ops, n)
    assert np.abs(m.to_state() - psi).max() < 1e-10
    assert m.discarded < 1e-20
    for x in (0, (1 << n) - 1, (0x5A5A5 % (1 << n))):
        assert abs(m.amplitude(x) - psi[x]) < 1e-10


@pytest.mark.parametrize("n,seed", [(6, 11), (8, 12)])
def test_bond_matrices_are_schmidt_coefficients(n, seed):
    ops = mixed_circuit(n, 10 * n, seed)
    m = M.run(ops, n, cutoff=0.0)
    psi = O.run(ops, n)
    for b in range(1, n):
        ref = schmidt_of_state(psi, n, b)
        assert m.bond_dims()[b] == len(ref), b   # numerical zeros are not kept
        got = np.sort(m.lam[b])[::-1]
        assert np.abs(got - ref).max() < 1e-10, b


def test_ghz_product_and_bell():
    n = 8
    m = M.run(qc.ghz(n), n)
    assert m.bond_dims() == [1] + [2] * (n - 1) + [1]
    for b in range(1, n):
        assert np.allclose(m.lam[b], [2 ** -0.5] * 2)
    p = M.run([qc.op("H", q) for q in range(n)] + [qc.op("RY", q, params=(0.3 * q,)) for q in range(n)], n)
    assert p.bond_dims() == [1] * (n + 1)
    # a Haar gate and its inverse leave rounding-level singular values, which
    # the numerical-zero rule drops even with no cutoff: back to chi = 1
    U = qc.haar_unitary(2, np.random.default_rng(5))
    back = M.run([qc.op("U", 2, 3, mat=U), qc.op("U", 2, 3, mat=U.conj().T)], 5, cutoff=0.0)
    assert back.bond_dims() == [1] * 6
    bell = M.run([qc.op("H", 0), qc.op("CNOT", 0, 1)], 2).to_state()
    assert np.allclose(bell, [2 ** -0.5, 0, 0, 2 ** -0.5])
    # control on the higher qubit, routed past two sites
    far = M.run([qc.op("H", 3), qc.op("CNOT", 3, 0)], 4).to_state()
    ref = np.zeros(16, complex)
    ref[0] = ref[9] = 2 ** -0.5
    assert np.allclose(far, ref)


@pytest.mark.parametrize("n", [5, 10, 15, 20])
def test_two_rounds_keep_chi_four(n):
    # section V.A: for two rounds the largest bond dimension is 4 at any width
    top = 0
    for seed in range(3):
        m = M.run(qc.paper_rounds(n, 2, 100 * n + seed), n)
        top = max(top, max(m.bond_dims()))
    assert 2 <= top <= 4


def test_single_truncation_weight():
    n = 6
    ops = mixed_circuit(n, 60, 21)
    exact = M.run(ops, n, cutoff=0.0)
    psi_before = exact.to_state()
    G = qc.haar_unitary(2, np.random.default_rng(22))
    ref = M.run([qc.op("U", 2, 3, mat=G)], n, cutoff=0.0, mps=exact).to_state()
    trunc = M.run(ops, n, cutoff=0.0)
    trunc.cutoff = 0.25
    M.run([qc.op("U", 2, 3, mat=G)], n, mps=trunc)
    assert np.allclose(np.linalg.norm(psi_before), 1.0)
    kept = float(np.sum(trunc.lam[3] ** 2))
    assert 0 < trunc.discarded and kept < 1
    got = trunc.to_state()
    assert abs(np.vdot(got, got).real - kept) < 1e-12
    assert abs(np.vdot(ref, got) - kept) < 1e-12
    assert abs(kept + trunc.discarded - 1.0) < 1e-12
