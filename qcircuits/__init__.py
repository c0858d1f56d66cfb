"""Seeded synthetic circuit generators.

This module is *input data only*: it emits gate records (name, qubits,
parameters and, for explicitly given unitaries, the matrix itself) and
Pauli-sum Hamiltonians as (coefficient, ((pauli, qubit), ...)) tuples.  It
contains none of the simulation arithmetic: gate matrices for named gates,
state updates, expectation values and sampling are implemented separately by
the GPU library and by the CPU oracle, and both consume these records.

Circuit families follow the workloads of the paper (random "rounds" circuits,
section V.A; the H2 VQE ansatz listing, section V.B) and the synthetic
benchmark families built on them: random brickwork circuits with Haar SU(2)
single-qubit layers and CZ entanglers, the quantum Fourier transform,
hardware-efficient ansatz batches and a rotation/CZ-ring ansatz for gradients.

Conventions (shared vocabulary, not arithmetic):
  * qubit q is bit q of the amplitude index (little-endian);
  * for multi-qubit gates the first listed qubit is the least-significant bit
    of the gate's local matrix index; CNOT and CPHASE list (control, target);
  * rotations are R_P(theta) = exp(-i theta P / 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

GATE_ARITY = {
    "I": 1, "X": 1, "Y": 1, "Z": 1, "H": 1, "S": 1, "SDG": 1, "T": 1, "TDG": 1,
    "RX": 1, "RY": 1, "RZ": 1,
    "CNOT": 2, "CZ": 2, "CPHASE": 2, "SWAP": 2,
}
GATE_NPARAMS = {"RX": 1, "RY": 1, "RZ": 1, "CPHASE": 1}
ROTATIONS = ("RX", "RY", "RZ")

SEEDS = {"c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "c5": 1005}


@dataclass(frozen=True)
class Op:
    """One gate record.  ``name == "U"`` carries an explicit complex128
    matrix of shape (2^k, 2^k) acting on ``qubits`` (first listed = LSB)."""
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    mat: Optional[np.ndarray] = field(default=None, compare=False)

    @property
    def k(self) -> int:
        return len(self.qubits)


def op(name: str, *qubits: int, params: Sequence[float] = (), mat=None) -> Op:
    return Op(name, tuple(int(q) for q in qubits), tuple(float(p) for p in params),
              None if mat is None else np.ascontiguousarray(mat, dtype=np.complex128))


# --------------------------------------------------------------------------
# random unitaries (input data: drawn here, passed explicitly to both sides)
# --------------------------------------------------------------------------

def haar_su2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(2): (Re a, Im a, Re b, Im b) = g/|g| with g ~ N(0, I4),
    matrix [[a, -conj(b)], [b, conj(a)]]."""
    g = rng.standard_normal(4)
    g = g / np.linalg.norm(g)
    a = complex(g[0], g[1])
    b = complex(g[2], g[3])
    return np.array([[a, -np.conj(b)], [b, np.conj(a)]], dtype=np.complex128)


def haar_unitary(k: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random U(2^k) via QR of a complex Gaussian matrix with the phases
    of R's diagonal moved into Q (Mezzadri's recipe)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return np.ascontiguousarray(q * ph[None, :], dtype=np.complex128)


# --------------------------------------------------------------------------
# circuit families
# --------------------------------------------------------------------------

def random_brickwork(n: int, depth: int, seed: int) -> list:
    """Random circuit family of the benchmark configs: each layer applies a
    Haar SU(2) to every qubit 0..n-1 (drawn in qubit order), then CZ on
    nearest-neighbour line pairs (0,1),(2,3),... on even layers and
    (1,2),(3,4),... on odd layers."""
    rng = np.random.default_rng(seed)
    ops = []
    for layer in range(depth):
        for q in range(n):
            ops.append(op("U", q, mat=haar_su2(rng)))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            ops.append(op("CZ", a, a + 1))
    return ops


def cz_mesh(n: int, depth: int, seed: int) -> list:
    """Haar SU(2) on every qubit, then CZ on a random pairing of all qubits
    (any distance), per layer: entanglers between every kind of qubit
    position a tile pass distinguishes."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(depth):
        for q in range(n):
            ops.append(op("U", q, mat=haar_su2(rng)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            ops.append(op("CZ", int(perm[i]), int(perm[i + 1])))
    return ops


def qft(n: int) -> list:
    """Quantum Fourier transform with the + phase convention: for j = n-1
    down to 0, H(j) then CPHASE(pi / 2^(j-m)) on (m, j) for m = j-1 .. 0;
    finally SWAP(q, n-1-q) for q < n/2 (bit reversal).  No angle is dropped."""
    ops = []
    for j in range(n - 1, -1, -1):
        ops.append(op("H", j))
        for m in range(j - 1, -1, -1):
            ops.append(op("CPHASE", m, j, params=(np.pi / float(1 << (j - m)),)))
    for q in range(n // 2):
        ops.append(op("SWAP", q, n - 1 - q))
    return ops


def qft_input(n: int, seed: int) -> int:
    """Seeded basis state |x> for the QFT workload."""
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 1 << n))


def ghz(n: int) -> list:
    ops = [op("H", 0)]
    for q in range(n - 1):
        ops.append(op("CNOT", q, q + 1))
    return ops


def hea_circuit(width: int, thetas: np.ndarray, layers: int = 10) -> list:
    """Hardware-efficient ansatz: per layer RY(theta[l,q,0]) then
    RZ(theta[l,q,1]) on every qubit, then the ascending CNOT ladder
    CNOT(q, q+1), q = 0..w-2."""
    thetas = np.asarray(thetas, dtype=np.float64).reshape(layers, width, 2)
    ops = []
    for l in range(layers):
        for q in range(width):
            ops.append(op("RY", q, params=(thetas[l, q, 0],)))
            ops.append(op("RZ", q, params=(thetas[l, q, 1],)))
        for q in range(width - 1):
            ops.append(op("CNOT", q, q + 1))
    return ops


@dataclass
class HeaBatch:
    widths: np.ndarray          # int, (count,)
    thetas: list                # list of (layers, w, 2) float64 arrays
    layers: int

    def circuit(self, i: int) -> list:
        return hea_circuit(int(self.widths[i]), self.thetas[i], self.layers)

    def hamiltonian(self, i: int) -> list:
        return zz_chain(int(self.widths[i]))


def hea_batch(count: int, seed: int, wmin: int = 8, wmax: int = 20, layers: int = 10) -> HeaBatch:
    """Batch of hardware-efficient-ansatz circuits: widths uniform on
    {wmin..wmax} (all drawn first), then per circuit its (layers, w, 2)
    angles uniform on [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    widths = rng.integers(wmin, wmax + 1, size=count)
    thetas = [rng.uniform(0.0, 2.0 * np.pi, size=(layers, int(w), 2)) for w in widths]
    return HeaBatch(widths=widths, thetas=thetas, layers=layers)


def zz_chain(n: int, coeff: float = 1.0, ring: bool = False) -> list:
    """sum_i Z_i Z_{i+1} over the open chain i = 0..n-2 (or the ring)."""
    terms = [(coeff, (("Z", i), ("Z", i + 1))) for i in range(n - 1)]
    if ring and n > 2:
        terms.append((coeff, (("Z", n - 1), ("Z", 0))))
    return terms


def rot_ring_ansatz(n: int, params: np.ndarray, layers: int) -> list:
    """Gradient workload ansatz: per layer RX, RY, RZ on every qubit with
    parameter index layer*3n + 3q + r, then CZ(q, (q+1) mod n) for all q."""
    params = np.asarray(params, dtype=np.float64)
    assert params.size == layers * 3 * n
    ops = []
    for l in range(layers):
        for q in range(n):
            base = l * 3 * n + 3 * q
            ops.append(op("RX", q, params=(params[base + 0],)))
            ops.append(op("RY", q, params=(params[base + 1],)))
            ops.append(op("RZ", q, params=(params[base + 2],)))
        for q in range(n):
            b = (q + 1) % n
            if b != q and not (n == 2 and q == 1):
                ops.append(op("CZ", q, b))
    return ops


def rot_ring_param_index(n: int, layers: int) -> np.ndarray:
    """For each op of ``rot_ring_ansatz`` the parameter index it reads, or -1."""
    idx = []
    for l in range(layers):
        for q in range(n):
            base = l * 3 * n + 3 * q
            idx += [base, base + 1, base + 2]
        for q in range(n):
            b = (q + 1) % n
            if b != q and not (n == 2 and q == 1):
                idx.append(-1)
    return np.asarray(idx, dtype=np.int64)


def gradient_workload(n: int, layers: int, seed: int):
    """(params, hamiltonian) of the gradient workload: params uniform on
    [0, 2 pi); H = sum_i Z_i Z_{i+1} (open chain) + 0.7 sum_i X_i."""
    rng = np.random.default_rng(seed)
    params = rng.uniform(0.0, 2.0 * np.pi, size=layers * 3 * n)
    ham = zz_chain(n) + [(0.7, (("X", i),)) for i in range(n)]
    return params, ham


def paper_rounds(n: int, rounds: int, seed: int) -> list:
    """Random "rounds" family of the paper's memory-profiling experiment
    (section V.A): a Hadamard layer in the first round only, then per round
    a layer of random single-qubit gates drawn from {X, Y, Z, RX, RY, RZ}
    (angles uniform on [0, 2 pi)) and a nearest-neighbour CNOT ladder."""
    rng = np.random.default_rng(seed)
    choices = ("X", "Y", "Z", "RX", "RY", "RZ")
    ops = [op("H", q) for q in range(n)]
    for _ in range(rounds):
        for q in range(n):
            g = choices[int(rng.integers(0, len(choices)))]
            if g in ROTATIONS:
                ops.append(op(g, q, params=(rng.uniform(0.0, 2.0 * np.pi),)))
            else:
                ops.append(op(g, q))
        for q in range(n - 1):
            ops.append(op("CNOT", q, q + 1))
    return ops


# The H2 ansatz of the paper's VQE listing (section V.B), with its decimal
# constants kept literally and "CNOT 1 0" read as control 1, target 0.
H2_CONSTANTS = (3.1415926, 1.57079, 7.85397, 7.8539752, 1.57079)


def h2_ansatz(t0: float) -> list:
    c = H2_CONSTANTS
    return [
        op("RX", 0, params=(c[0],)),
        op("RY", 1, params=(c[1],)),
        op("RX", 0, params=(c[2],)),
        op("CNOT", 1, 0),
        op("RZ", 0, params=(t0,)),
        op("CNOT", 1, 0),
        op("RY", 1, params=(c[3],)),
        op("RX", 0, params=(c[4],)),
    ]


H2_TERMS = {
    "Z0": ((("Z", 0),)),
    "Z1": ((("Z", 1),)),
    "Z0Z1": (("Z", 0), ("Z", 1)),
    "X0X1": (("X", 0), ("X", 1)),
    "Y0Y1": (("Y", 0), ("Y", 1)),
}


def h2_sweep(points: int = 100) -> np.ndarray:
    """The listing's parameter grid: linspace(-pi, pi, 100)."""
    return np.linspace(-np.pi, np.pi, points)


def h2_term_batch(t0s):
    """One circuit per (t0, term) of the H2 sweep, for a batch that measures
    Z-strings only: the ansatz, then the basis change that turns the term
    into a Z-string (H for X; S^dag then H for Y), and that Z-string as the
    circuit's one-term Hamiltonian.  Returns (circuits, widths, hamiltonians,
    keys) with keys[i] = (t0, term name)."""
    circuits, widths, hams, keys = [], [], [], []
    for t0 in t0s:
        for key, term in H2_TERMS.items():
            ops = h2_ansatz(float(t0))
            zterm = []
            for p, q in term:
                if p == "X":
                    ops.append(op("H", q))
                elif p == "Y":
                    ops += [op("SDG", q), op("H", q)]
                zterm.append(("Z", q))
            circuits.append(ops)
            widths.append(2)
            hams.append([(1.0, tuple(zterm))])
            keys.append((float(t0), key))
    return circuits, widths, hams, keys


def h2_closed_forms(t0: float) -> dict:
    """Per-term values of the listing's ansatz with exact pi constants."""
    return {"Z0": np.cos(t0), "Z1": -np.cos(t0), "Z0Z1": -1.0,
            "X0X1": -np.sin(t0), "Y0Y1": -np.sin(t0)}


# --------------------------------------------------------------------------
# fuzz circuits for parity tests
# --------------------------------------------------------------------------

ALL_NAMED = ("I", "X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ",
             "CNOT", "CZ", "CPHASE", "SWAP")


def random_ops(n: int, count: int, seed: int, names: Sequence[str] = ALL_NAMED,
               dense_k: Sequence[int] = (1, 2, 3), p_dense: float = 0.15) -> list:
    """Random op list over every named gate kind on random (ordered) qubit
    sets, mixed with explicit Haar unitaries on k qubits."""
    rng = np.random.default_rng(seed)
    ops = []
    names = [g for g in names if GATE_ARITY[g] <= n]
    dense_k = [k for k in dense_k if k <= n]
    for _ in range(count):
        if dense_k and rng.random() < p_dense:
            k = int(dense_k[int(rng.integers(0, len(dense_k)))])
            qs = rng.permutation(n)[:k]
            ops.append(op("U", *qs, mat=haar_unitary(k, rng)))
            continue
        g = names[int(rng.integers(0, len(names)))]
        qs = rng.permutation(n)[:GATE_ARITY[g]]
        ps = tuple(rng.uniform(-2.0 * np.pi, 2.0 * np.pi, size=GATE_NPARAMS.get(g, 0)))
        ops.append(op(g, *qs, params=ps))
    return ops


def random_hamiltonian(n: int, terms: int, seed: int, max_weight: int = 3) -> list:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(terms):
        w = int(rng.integers(1, min(max_weight, n) + 1))
        qs = rng.permutation(n)[:w]
        ps = [("X", "Y", "Z")[int(rng.integers(0, 3))] for _ in qs]
        out.append((float(rng.uniform(-1, 1)), tuple(zip(ps, (int(q) for q in qs)))))
    return out


def dagger(ops: Sequence[Op]) -> list:
    """Inverse circuit as gate records: reversed order, each gate replaced by
    its inverse *name* (rotations negate their angle, S <-> SDG, T <-> TDG);
    explicit matrices are conjugate-transposed (input data)."""
    inv = {"S": "SDG", "SDG": "S", "T": "TDG", "TDG": "T"}
    out = []
    for o in reversed(list(ops)):
        if o.name == "U":
            out.append(Op("U", o.qubits, (), np.ascontiguousarray(o.mat.conj().T)))
        elif o.name in ROTATIONS or o.name == "CPHASE":
            out.append(Op(o.name, o.qubits, tuple(-p for p in o.params)))
        else:
            out.append(Op(inv.get(o.name, o.name), o.qubits, o.params))
    return out


def random_state(n: int, seed: int) -> np.ndarray:
    """Seeded random complex128 input state (Gaussian entries scaled to unit norm)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)
