"""MPS gate application on the GPU (through the C ABI) against the MPS oracle
and the state-vector oracle.

The site tensors are fixed only up to gauge (phases and rotations inside
degenerate singular subspaces), so the comparisons are on what is unique:
amplitudes, bond dimensions and Schmidt coefficients.
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import mps as M
from oracle import oracle as O
from test_oracle_mps import mixed_circuit

pytestmark = pytest.mark.gpu


def gpu_mps(ops, n, chi, cutoff):
    from paper_1807_07914_amd import MPS
    m = MPS(n, chi, cutoff)
    m.apply_circuit(ops)
    return m


def haar_brickwork(n, layers, seed, far=True):
    """Haar two-qubit gates on a brickwork (generic singular values, so a
    truncation has one answer), plus a distant pair per layer."""
    rng = np.random.default_rng(seed)
    ops = []
    for l in range(layers):
        for q in range(l % 2, n - 1, 2):
            ops.append(qc.op("U", q, q + 1, mat=qc.haar_unitary(2, rng)))
        if far and n >= 4:
            a, b = sorted(int(x) for x in rng.choice(n, 2, replace=False))
            ops.append(qc.op("U", b, a, mat=qc.haar_unitary(2, rng)))
    return ops


def compare(m, ref, n, tol):
    dims, lam = m.bonds()
    assert dims == ref.bond_dims()
    for b in range(n + 1):
        assert np.abs(lam[b] - ref.lam[b]).max() <= tol, b
    psi = m.to_numpy()
    assert np.abs(psi - ref.to_state()).max() <= tol
    return psi


@pytest.mark.parametrize("n,seed,chi", [(2, 1, 32), (3, 2, 32), (5, 3, 32), (8, 4, 32), (10, 5, 32),
                                        (12, 6, 64), (13, 7, 64)])
def test_exact_matches_oracles(n, seed, chi):
    # n = 12 reaches bond 64 in the middle (the workspace path), n = 13 keeps
    # it there for two bonds; every smaller bond still runs in LDS
    ops = mixed_circuit(n, 12 * n, seed)
    ref = M.run(ops, n, cutoff=0.0)
    assert max(ref.bond_dims()) <= chi
    m = gpu_mps(ops, n, chi, 0.0)
    psi = compare(m, ref, n, 1e-12)
    m.close()
    assert np.abs(psi - O.run(ops, n)).max() < 1e-12


@pytest.mark.parametrize("n,chi,cutoff", [(10, 8, 1e-2), (10, 4, 0.0), (12, 32, 1e-4), (14, 48, 0.0),
                                          (14, 64, 1e-4)])
def test_truncated_matches_oracle(n, chi, cutoff):
    ops = haar_brickwork(n, 12, 100 + n + chi)
    ref = M.run(ops, n, chi_max=chi, cutoff=cutoff)
    assert ref.discarded > 0 and max(ref.bond_dims()) == chi
    m = gpu_mps(ops, n, chi, cutoff)
    compare(m, ref, n, 1e-9)
    info = m.info()
    m.close()
    assert info["bond_updates"] > 0


@pytest.mark.parametrize("n", [5, 8, 10])
@pytest.mark.parametrize("rounds", [2, 4, 6])
def test_paper_rounds_fidelity(n, rounds):
    # the random-round family of section V.A at the paper's cutoff 1e-4
    ops = qc.paper_rounds(n, rounds, 7000 + 10 * n + rounds)
    m = gpu_mps(ops, n, 32, 1e-4)
    psi = m.to_numpy()
    dims, _ = m.bonds()
    m.close()
    exact = O.run(ops, n)
    fid = abs(np.vdot(exact, psi)) ** 2 / np.vdot(psi, psi).real
    assert fid >= 1 - 1e-6
    if rounds == 2:
        assert max(dims) <= 4
    ref = M.run(ops, n, chi_max=32, cutoff=1e-4)
    assert dims == ref.bond_dims()
    assert np.abs(psi - ref.to_state()).max() <= 1e-9


@pytest.mark.parametrize("n", [60, 85])
def test_wide_registers_two_rounds(n):
    # beyond any state vector: chi <= 4 at two rounds, unit Schmidt weight on
    # every bond, and sampled amplitudes against the oracle's site-by-site ones
    ops = qc.paper_rounds(n, 2, 9100 + n)
    ref = M.run(ops, n)
    m = gpu_mps(ops, n, 32, 1e-4)
    dims, lam = m.bonds()
    assert dims == ref.bond_dims() and max(dims) <= 4
    for b in range(n + 1):
        assert abs(np.sum(lam[b] ** 2) - 1.0) < 1e-10
        assert np.abs(lam[b] - ref.lam[b]).max() < 1e-10
    if n <= 63:
        rng = np.random.default_rng(n)
        idx = [int(x) for x in rng.integers(0, 1 << n, 64)] + [0, (1 << n) - 1]
        got = m.amplitudes(np.array(idx, dtype=np.uint64))
        want = np.array([ref.amplitude(x) for x in idx])
        assert np.abs(got - want).max() < 1e-12
    m.close()


def test_edge_cases_and_errors():
    from paper_1807_07914_amd import MPS, QsvError
    # one qubit: only one-site updates
    ops = [qc.op("H", 0), qc.op("RZ", 0, params=(0.3,)), qc.op("RY", 0, params=(1.1,))]
    m = gpu_mps(ops, 1, 4, 1e-4)
    assert np.abs(m.to_numpy() - O.run(ops, 1)).max() < 1e-14
    m.close()
    # empty circuit, then two calls in a row ending in pending one-qubit gates
    n = 6
    m = MPS(n, 16, 0.0)
    m.apply_circuit([])
    a = mixed_circuit(n, 30, 91) + [qc.op("T", q) for q in range(n)]
    b = mixed_circuit(n, 30, 92) + [qc.op("RX", 2, params=(0.7,))]
    m.apply_circuit(a)
    m.apply_circuit(b)
    assert np.abs(m.to_numpy() - O.run(a + b, n)).max() < 1e-12
    with pytest.raises(QsvError):
        m.apply_circuit([qc.op("U", 0, 1, 2, mat=qc.haar_unitary(3, np.random.default_rng(0)))])
    with pytest.raises(QsvError):
        m.apply_circuit([qc.op("H", n)])
    with pytest.raises(QsvError):
        m.amplitudes(np.array([1 << n], dtype=np.uint64))
    m.close()
    # a Haar gate and its inverse: rounding-level singular values are dropped
    U = qc.haar_unitary(2, np.random.default_rng(5))
    m = gpu_mps([qc.op("U", 2, 3, mat=U), qc.op("U", 2, 3, mat=U.conj().T)], 5, 4, 0.0)
    dims, lam = m.bonds()
    m.close()
    assert dims == [1] * 6 and abs(lam[3][0] - 1.0) < 1e-12
    for bad in ((0, 4, 0.0), (4, 0, 0.0), (4, 65, 0.0), (4, 4, -1.0)):
        with pytest.raises(QsvError):
            MPS(*bad)
