"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: complex128 max|d| <= 1e-12, complex64 max|d| <= 1e-5 (absolute,
per amplitude).  For complex64 the oracle starts from the complex64-rounded
input so that only the path's own error is measured.
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
NAMED1 = ["I", "X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ"]
NAMED2 = ["CNOT", "CZ", "CPHASE", "SWAP"]


def State(*a, **k):
    from paper_1807_07914_amd import State as S
    return S(*a, **k)


def start(n, dtype, seed):
    psi = qc.random_state(n, seed)
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    return psi


def gpu_run(n, dtype, psi0, ops, mode="pergate", **kw):
    s = State(n, dtype)
    s.from_numpy(psi0)
    s.apply_circuit(ops, mode=mode, **kw)
    out = s.to_numpy().astype(np.complex128)
    s.close()
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_every_named_gate_every_qubit(dtype, n):
    psi0 = start(n, dtype, 100 + n)
    for g in NAMED1 + (NAMED2 if n >= 2 else []):
        k = qc.GATE_ARITY[g]
        targets = [(q,) for q in range(n)] if k == 1 else \
            [(a, b) for a in range(n) for b in range(n) if a != b]
        for qs in targets:
            o = qc.op(g, *qs, params=(0.7312,) if g in qc.GATE_NPARAMS else ())
            ref = O.run([o], n, psi=psi0.copy())
            s = State(n, dtype)
            s.from_numpy(psi0)
            s.apply_gate(g, list(qs), list(o.params))
            got = s.to_numpy()
            s.close()
            err = np.abs(got - ref).max()
            assert err <= TOL[dtype], (g, qs, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 6, 11, 14])
def test_random_circuits_pergate(dtype, n):
    ops = qc.random_ops(n, 80, 200 + n, dense_k=(1, 2, 3))
    psi0 = start(n, dtype, 300 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    got = gpu_run(n, dtype, psi0, ops, "pergate")
    assert np.abs(got - ref).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_apply_fused_dense(dtype, k):
    n = 12
    rng = np.random.default_rng(40 + k)
    for trial in range(3):
        qs = [int(q) for q in rng.permutation(n)[:k]]
        if trial == 0:
            qs = list(range(k))            # lowest qubits
        elif trial == 1:
            qs = list(range(n - 1, n - 1 - k, -1))  # highest, reversed
        U = qc.haar_unitary(k, rng)
        psi0 = start(n, dtype, 500 + k + trial)
        ref = psi0.copy()
        O.apply_matrix(ref, n, qs, U)
        s = State(n, dtype)
        s.from_numpy(psi0)
        s.apply_fused(qs, U)
        got = s.to_numpy()
        s.close()
        assert np.abs(got - ref).max() <= TOL[dtype], (k, qs)


@pytest.mark.parametrize("mode", ["pergate", "auto"])
def test_c1_random_circuit_c128(mode):
    # 10-qubit random brickwork circuit, depth 20, complex128, from |0..0>
    n = 10
    ops = qc.random_brickwork(n, 20, qc.SEEDS["c1"])
    assert len(ops) == 290
    ref = O.run(ops, n)
    s = State(n, "c128")
    s.apply_circuit(ops, mode=mode)
    got = s.to_numpy()
    s.close()
    assert np.abs(got - ref).max() <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 4, 7, 10, 13])
def test_expval_and_norm(dtype, n):
    psi0 = start(n, dtype, 600 + n)
    ops = qc.random_ops(n, 30, 700 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    ham = qc.random_hamiltonian(n, 24, 800 + n, max_weight=4)
    s = State(n, dtype)
    s.from_numpy(psi0)
    s.apply_circuit(ops, mode="pergate")
    terms = s.expval(ham, per_term=True)
    ref_terms = O.expval(ref, ham, per_term=True)
    assert np.abs(np.asarray(terms) - ref_terms).max() <= 10 * TOL[dtype]
    assert abs(s.expval(ham) - O.expval(ref, ham)) <= 10 * TOL[dtype] * len(ham)
    assert abs(s.norm() - O.norm(ref)) <= 10 * TOL[dtype]
    s.close()


@pytest.mark.parametrize("dtype,n", [("c64", 11), ("c64", 19), ("c128", 10), ("c128", 18)])
def test_expval_z_register_sums(dtype, n):
    """Z-only terms are summed 32 to a read from per-thread register groups
    (index bits 0, 7..10 complex64 / 6..9 complex128): masks on those bits,
    on the others and on both, one-qubit and long strings, 45 terms (two
    launches), at the smallest supported width and a wider one."""
    psi0 = start(n, dtype, 1300 + n)
    rng = np.random.default_rng(1400 + n)
    ham = [(1.0, (("Z", q),)) for q in range(n)]
    ham += [(0.5, (("Z", q), ("Z", (q + 1) % n))) for q in range(n)]
    while len(ham) < 45:
        qs = sorted(set(int(q) for q in rng.integers(0, n, int(rng.integers(2, 7)))))
        ham.append((float(rng.uniform(-1, 1)), tuple(("Z", q) for q in qs)))
    s = State(n, dtype)
    s.from_numpy(psi0)
    terms = s.expval(ham, per_term=True)
    ref_terms = O.expval(psi0.astype(np.complex128), ham, per_term=True)
    assert np.abs(np.asarray(terms) - ref_terms).max() <= 10 * TOL[dtype]
    s.close()


@pytest.mark.parametrize("dtype,n", [("c64", 5), ("c64", 17), ("c128", 4), ("c128", 16)])
def test_expval_one_qubit_x_y_terms(dtype, n):
    """One-qubit X / Y terms with Z strings are evaluated on register rounds:
    every qubit, X and Y, Z on other tile qubits and on qubits outside the
    tile, two terms on one qubit (separate tiles), against the oracle."""
    psi0 = start(n, dtype, 1500 + n)
    rng = np.random.default_rng(1600 + n)
    ham = [(0.3 + 0.01 * q, (("X", q),)) for q in range(n)]
    ham += [(-0.4, (("Y", q),)) for q in range(0, n, 2)]
    for q in range(n):
        others = [int(p) for p in rng.choice([p for p in range(n) if p != q], size=min(3, n - 1), replace=False)]
        ham.append((float(rng.uniform(-1, 1)), (("X" if q % 3 else "Y", q),) + tuple(("Z", p) for p in others)))
    s = State(n, dtype)
    s.from_numpy(psi0)
    terms = s.expval(ham, per_term=True)
    ref_terms = O.expval(psi0.astype(np.complex128), ham, per_term=True)
    assert np.abs(np.asarray(terms) - ref_terms).max() <= 10 * TOL[dtype]
    s.close()


@pytest.mark.parametrize("dtype,n", [("c64", 17), ("c128", 16)])
def test_expval_tiled_x_terms(dtype, n):
    """Terms with X masks are reduced tile by tile when their masks fit a
    tile (more than 16 of them here, so several tiles), the rest one pass per
    mask; per-term values against the oracle, with Y terms, X masks on high
    qubits, masks too wide for a tile, and Z-only terms mixed in."""
    psi0 = start(n, dtype, 900 + n)
    ham = [(0.3 + 0.01 * q, (("X", q),)) for q in range(n)]
    ham += [(-0.2, (("X", q), ("Y", q + 1))) for q in range(0, n - 1, 2)]
    ham += [(0.15, (("Y", q), ("Z", (q + 3) % n))) for q in range(1, n, 3)]
    ham += [(0.5, tuple(("X", q) for q in range(5, 15)))]                       # 10 high qubits
    ham += [(0.25, (("Y", 0), ("X", n - 1), ("Z", n // 2)))]
    ham += [(0.7, (("Z", q), ("Z", q + 1))) for q in range(n - 1)]
    s = State(n, dtype)
    s.from_numpy(psi0)
    terms = s.expval(ham, per_term=True)
    ref_terms = O.expval(psi0.astype(np.complex128), ham, per_term=True)
    assert np.abs(np.asarray(terms) - ref_terms).max() <= 10 * TOL[dtype]
    assert abs(s.expval(ham) - O.expval(psi0.astype(np.complex128), ham)) <= 10 * TOL[dtype] * len(ham)
    s.close()


def test_h2_listing_on_gpu():
    for t0 in qc.h2_sweep()[::7]:
        ops = qc.h2_ansatz(t0)
        ref = O.run(ops, 2)
        s = State(2, "c128")
        s.apply_circuit(ops)
        v = s.expval([(1.0, t) for t in qc.H2_TERMS.values()], per_term=True)
        r = [O.pauli_expval(ref, t).real for t in qc.H2_TERMS.values()]
        assert np.abs(np.asarray(v) - r).max() < 1e-12
        assert abs(v[2] + 1.0) < 1e-9 and abs(v[0] - np.cos(t0)) < 1e-9
        s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 10, 16])
def test_sample_parity(dtype, n):
    psi0 = start(n, dtype, 900 + n)
    ops = qc.random_ops(n, 20, 910 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    u = np.random.default_rng(n).random(3000)
    u[:2] = [0.0, 1 - 2 ** -53]
    s = State(n, dtype)
    s.from_numpy(psi0)
    s.apply_circuit(ops, mode="pergate")
    got = s.sample(u)
    s.close()
    want = O.sample(ref, u)
    C = O.cdf(ref)
    t = u * C[-1]
    near = np.min(np.abs(C[None, :] - t[:, None]), axis=1) if n <= 10 else None
    bad = np.flatnonzero(got != want)
    tol = 1e-12 if dtype == "c128" else 2e-5
    for i in bad:
        # a mismatch is allowed only where u * total lies within rounding of a
        # CDF boundary, and the result must then be an adjacent valid index
        g, w = int(got[i]), int(want[i])
        lo, hi = min(g, w), max(g, w)
        assert abs(C[lo] - t[i]) <= tol or abs(C[hi - 1] - t[i]) <= tol, (i, g, w)
    assert len(bad) <= max(1, len(u) // 1000)
    assert got.max() < (1 << n)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [4, 20])
def test_sample_distribution_chi2(dtype, n):
    # shots drawn on the GPU from a fused state follow |psi|^2 of the
    # oracle's state: Pearson chi^2 over 16 bins (all outcomes at n = 4, the
    # top four qubits' marginal at n = 20), 15 degrees of freedom; 40 is
    # exceeded with probability ~4e-4
    ops = qc.random_brickwork(n, 8, 930 + n)
    p = np.abs(O.run(ops, n)) ** 2
    shift = n - 4
    pb = p.reshape(16, 1 << shift).sum(axis=1)
    u = np.random.default_rng(940 + n).random(400000)
    s = State(n, dtype)
    s.apply_circuit(ops)
    got = s.sample(u)
    s.close()
    counts = np.bincount((got.astype(np.int64) >> shift), minlength=16)
    assert counts.sum() == u.size
    chi2 = float(((counts - pb * u.size) ** 2 / (pb * u.size)).sum())
    assert chi2 < 40, chi2


def test_ghz_and_qft_closed_forms_medium():
    n = 18
    s = State(n, "c64")
    s.apply_circuit(qc.ghz(n))
    psi = s.to_numpy()
    assert abs(psi[0] - 2 ** -0.5) < 1e-6 and abs(psi[-1] - 2 ** -0.5) < 1e-6
    assert np.abs(psi[1:-1]).max() == 0
    s.close()
    n = 16
    x = qc.qft_input(n, qc.SEEDS["c3"])
    for dtype, tol in (("c128", 1e-12), ("c64", 1e-5)):
        s = State(n, dtype)
        s.set_basis(x)
        s.apply_circuit(qc.qft(n))
        psi = s.to_numpy()
        s.close()
        y = np.arange(1 << n, dtype=np.int64)
        ref = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / 2 ** (n / 2)
        assert np.abs(psi - ref).max() <= tol


def test_error_paths_on_device():
    from paper_1807_07914_amd import QsvError
    s = State(4, "c64")
    with pytest.raises(QsvError):
        s.apply_gate("H", [4])
    with pytest.raises(QsvError):
        s.apply_gate("CNOT", [1, 1])
    with pytest.raises(QsvError):
        s.apply_gate("RX", [0], [float("nan")])
    with pytest.raises(QsvError):
        s.apply_gate("RX", [0], [])
    with pytest.raises(QsvError):
        s.sample(np.array([1.0]))
    with pytest.raises(QsvError):
        s.expval([(1.0, (("Z", 5),))])
    with pytest.raises(QsvError):
        s.apply_fused([0, 1, 2, 3, 0], np.eye(32))
    with pytest.raises(QsvError):
        s.set_basis(16)
    s.close()
    with pytest.raises(QsvError):
        s.norm()


# ------------------------------------------------------------ fused passes
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,tile", [(5, 0), (8, 0), (13, 0), (14, 0), (16, 0), (16, 9), (18, 7),
                                    (17, 12)])
def test_fused_random_circuits(dtype, n, tile):
    if dtype == "c128" and tile > 12:
        tile = 12
    ops = qc.random_ops(n, 150, 1000 + n + tile, dense_k=(1, 2, 3))
    psi0 = start(n, dtype, 1100 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    got = gpu_run(n, dtype, psi0, ops, "fused", tile_qubits=tile)
    assert np.abs(got - ref).max() <= TOL[dtype]


@pytest.mark.parametrize("small_tile", [False, True])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("family", ["brickwork", "rounds", "qft", "hea", "rotring", "ghz", "cz_mesh"])
def test_fused_families(dtype, family, small_tile):
    # small_tile: 2^12 (complex64) / 2^11 (complex128) tiles, which run on the
    # half-size LDS kernels (lean or full by the pass's steps)
    n = 16
    rng = np.random.default_rng(5)
    x0 = 0
    if family == "brickwork":
        ops = qc.random_brickwork(n, 12, 77)
    elif family == "rounds":
        ops = qc.paper_rounds(n, 6, 78)
    elif family == "qft":
        ops = qc.qft(n)
        x0 = qc.qft_input(n, 79)
    elif family == "hea":
        ops = qc.hea_circuit(n, rng.uniform(0, 2 * np.pi, (10, n, 2)))
    elif family == "rotring":
        ops = qc.rot_ring_ansatz(n, rng.uniform(0, 2 * np.pi, 3 * 3 * n), 3)
    elif family == "cz_mesh":
        allcz = [qc.op("CZ", i, j) for i in range(n) for j in range(i + 1, n)]
        ops = allcz + qc.cz_mesh(n, 10, 80) + allcz
    else:
        ops = qc.ghz(n)
    ref = O.run(ops, n, x0=x0)
    s = State(n, dtype)
    s.set_basis(x0)
    tile = (12 if dtype == "c64" else 11) if small_tile else 0
    info = s.plan_info(ops, tile_qubits=tile)
    s.apply_circuit(ops, mode="fused", tile_qubits=tile)
    got = s.to_numpy()
    s.close()
    assert info["passes"] < len(ops)
    assert np.abs(got - ref).max() <= TOL[dtype], info


def _swap_network(n, layers, seed):
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


def _plan_kinds(n, dtype, ops, tile=0):
    import tile_emulator as E
    words, steps = E.program(n, dtype, ops, tile)
    return "".join("P" if E.is_qperm(words, int(s)) else ("T" if s >= 0 else "X") for s in steps)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,tile,seed,layers", [(8, 6, 1, 3), (10, 6, 0, 3), (12, 7, 2, 3), (18, 0, 2, 4),
                                                (20, 9, 3, 4)])
def test_fused_swap_relabeling(dtype, n, tile, seed, layers):
    # SWAPs relabeled away and the state put back in order by one or two
    # qubit-permutation passes (the plan is checked to take that route)
    ops = _swap_network(n, layers, seed)
    kinds = _plan_kinds(n, dtype, ops, tile)
    if "P" not in kinds:
        pytest.skip("the planner keeps the SWAPs for this case and dtype: " + kinds)
    assert kinds.endswith("P") and kinds.count("P") <= 2
    psi0 = start(n, dtype, 1300 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    got = gpu_run(n, dtype, psi0, ops, "fused", tile_qubits=tile)
    assert np.abs(got - ref).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [14, 22])
def test_tuned_mode_matches_oracle(dtype, n):
    # mode "tuned": the autotuner picks the tile shape on the first call of
    # the structure (timing on a copy of the state), later calls reuse it
    ops = qc.random_brickwork(n, 12, 1500 + n) + [qc.op("SWAP", 0, n - 1)] + qc.qft(n)
    psi0 = start(n, dtype, 1510 + n)
    ref = O.run(ops, n, psi=psi0.copy())
    first = gpu_run(n, dtype, psi0, ops, "tuned")
    assert np.abs(first - ref).max() <= TOL[dtype]
    assert np.array_equal(gpu_run(n, dtype, psi0, ops, "tuned"), first)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fused_qft_bit_reversal_pass(dtype):
    # 22 qubits: the QFT's swaps become one bit-reversal pass (complex64),
    # against the oracle element by element from a random state
    n = 22
    ops = qc.qft(n)
    psi0 = start(n, dtype, 1401)
    ref = O.run(ops, n, psi=psi0.copy())
    got = gpu_run(n, dtype, psi0, ops, "fused")
    assert np.abs(got - ref).max() <= TOL[dtype]
    if dtype == "c64":
        assert _plan_kinds(n, dtype, ops) == "TTP"


def test_fused_plan_is_reused_with_new_matrices():
    # same structure, different angles: the cached schedule must take the new values
    n = 15
    for seed in (1, 2, 3):
        ops = qc.random_brickwork(n, 6, seed)
        ref = O.run(ops, n)
        s = State(n, "c128")
        s.apply_circuit(ops, mode="fused")
        got = s.to_numpy()
        s.close()
        assert np.abs(got - ref).max() <= 1e-12


# ------------------------------------------------------- dense blocks, MFMA
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [4, 5, 6])
@pytest.mark.parametrize("n", [6, 9, 17])
def test_dense_blocks_on_matrix_cores(dtype, k, n):
    if k > n:
        pytest.skip("block wider than register")
    rng = np.random.default_rng(100 * k + n)
    layouts = [list(range(k)), list(range(n - 1, n - 1 - k, -1)),
               [int(q) for q in rng.permutation(n)[:k]]]
    for qs in layouts:
        U = qc.haar_unitary(k, rng)
        psi0 = start(n, dtype, 7 * k + n)
        ref = psi0.copy()
        O.apply_matrix(ref, n, qs, U)
        s = State(n, dtype)
        s.from_numpy(psi0)
        s.apply_fused(qs, U)
        got = s.to_numpy()
        s.close()
        assert np.abs(got - ref).max() <= TOL[dtype], (qs, np.abs(got - ref).max())


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode", ["pergate", "fused"])
def test_circuits_with_wide_blocks(dtype, mode):
    n = 14
    ops = qc.random_ops(n, 60, 4242, dense_k=(3, 4, 5, 6), p_dense=0.3)
    psi0 = start(n, dtype, 4243)
    ref = O.run(ops, n, psi=psi0.copy())
    got = gpu_run(n, dtype, psi0, ops, mode)
    assert np.abs(got - ref).max() <= TOL[dtype]


@pytest.mark.parametrize("rounds", [2, 6, 10])
@pytest.mark.parametrize("n", [5, 10, 15])
def test_paper_rounds_grid(n, rounds):
    # the paper's random-round family on its n / rounds grid, fused passes
    # against the oracle, complex64
    ops = qc.paper_rounds(n, rounds, 2000 + 100 * n + 10 * rounds)
    ref = O.run(ops, n)
    s = State(n, "c64")
    s.apply_circuit(ops, mode="fused")
    got = s.to_numpy()
    s.close()
    assert np.abs(got - ref).max() <= TOL["c64"]


@pytest.mark.parametrize("n,rounds", [(16, 2), (16, 4), (20, 2), (20, 4), (20, 6)])
def test_paper_rounds_schmidt_bound_on_gpu(n, rounds):
    # one CNOT per round crosses the middle cut, so the state computed on the
    # GPU has Schmidt rank <= 2^rounds there (host SVD of the result)
    ops = qc.paper_rounds(n, rounds, 3000 + n + rounds)
    s = State(n, "c64")
    s.apply_circuit(ops, mode="fused")
    psi = s.to_numpy()
    s.close()
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-4
    sv = np.linalg.svd(psi.reshape(1 << (n - n // 2), 1 << (n // 2)), compute_uv=False)
    assert int(np.sum(sv > 1e-4 * sv[0])) <= 2 ** rounds
    # and the bound is not vacuous: the rank reaches it for these seeds
    assert int(np.sum(sv > 1e-4 * sv[0])) >= 2


# ------------------------------------------------------------ degenerate inputs
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_degenerate_sizes_and_empty_inputs(dtype, n):
    # states smaller than a register group, in every apply mode; the empty
    # circuit, an empty Hamiltonian and zero shots leave or return nothing
    ops = qc.random_ops(n, 25, 500 + n, dense_k=tuple(k for k in (1, 2, 3) if k <= n))
    ref = O.run(ops, n)
    for mode in ("fused", "pergate", "auto"):
        s = State(n, dtype)
        s.apply_circuit(ops, mode=mode)
        got = s.to_numpy().astype(np.complex128)
        assert np.abs(got - ref).max() <= TOL[dtype], mode
        s.apply_circuit([], mode=mode)
        assert np.array_equal(s.to_numpy().astype(np.complex128), got)
        assert s.expval([]) == 0.0
        assert s.sample(np.zeros(0)).size == 0
        s.close()
    # an adjoint sweep over no ops: the energy of the current state, no gradients
    ham = qc.random_hamiltonian(n, 3, 600 + n, max_weight=min(n, 2))
    s = State(n, dtype)
    s.from_numpy(ref)
    e, g = s.adjoint([], ham)
    back = s.to_numpy().astype(np.complex128)
    s.close()
    assert g.size == 0
    assert abs(e - O.expval(ref, ham)) <= 10 * TOL[dtype] * len(ham)
    assert np.abs(back - ref).max() <= TOL[dtype]
