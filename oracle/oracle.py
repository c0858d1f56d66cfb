"""CPU oracle: plain complex128 state-vector simulation (test infrastructure).

Only the tests, the smoke check and the benchmark's ``cpu_baseline`` leg use
this module.  It wraps ``oracle.c`` (built with gcc, never hipcc) through
ctypes and shares no code with the GPU library: gate matrices, the gather /
scatter update, expectation values, norms and sampling are the oracle's own.

Each routine restates a definition (see ``oracle.c`` for O1..O6):
  * ``run``               O1-O3, program-order execution of the gate list
                          (paper section IV.A: pre-order traversal of the
                          instruction tree, one gate at a time, no fusion).
  * ``expval``            O4, sum_k c_k Re <psi|P_k|psi> (paper section V.B:
                          one expectation value per Hamiltonian term).
  * ``norm``              O5.
  * ``sample``            O6 (paper section V.B, MEASURE), uniforms supplied.
  * ``param_shift_grad``  exact gradient of <H> for R_P(theta) =
                          exp(-i theta P/2): [E(theta+pi/2) - E(theta-pi/2)]/2.
  * ``finite_diff_grad``  central differences, as a second route.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GATE_IDS = {
    "I": 0, "X": 1, "Y": 2, "Z": 3, "H": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8,
    "RX": 9, "RY": 10, "RZ": 11, "CNOT": 12, "CZ": 13, "CPHASE": 14, "SWAP": 15, "U": 16,
}
PAULI_IDS = {"X": 1, "Y": 2, "Z": 3}

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP).  Rebuilds when the source is newer."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    c_int, c_double, c_u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    vp = ctypes.c_void_p
    lib.orc_gate_matrix.argtypes = [c_int, P(c_double), vp]
    lib.orc_gate_matrix.restype = c_int
    lib.orc_init_basis.argtypes = [vp, c_int, c_u64]
    lib.orc_init_basis.restype = None
    lib.orc_apply_matrix.argtypes = [vp, c_int, c_int, P(c_int), vp]
    lib.orc_apply_matrix.restype = c_int
    lib.orc_apply_op.argtypes = [vp, c_int, c_int, c_int, P(c_int), P(c_double), vp]
    lib.orc_apply_op.restype = c_int
    lib.orc_norm.argtypes = [vp, c_int]
    lib.orc_norm.restype = c_double
    lib.orc_inner.argtypes = [vp, vp, c_int, P(c_double)]
    lib.orc_inner.restype = None
    lib.orc_pauli_expval.argtypes = [vp, c_int, c_int, P(c_int), P(c_int), vp, P(c_double)]
    lib.orc_pauli_expval.restype = c_int
    lib.orc_sample.argtypes = [vp, c_int, P(c_double), c_int, P(c_u64)]
    lib.orc_sample.restype = c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = c_int
    lib.orc_set_threads.argtypes = [c_int]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ints(xs: Sequence[int]):
    arr = (ctypes.c_int * max(1, len(xs)))(*[int(x) for x in xs])
    return arr


def _dbls(xs: Sequence[float], size: int = 3):
    vals = list(xs) + [0.0] * (size - len(xs))
    return (ctypes.c_double * size)(*vals)


def gate_matrix(name: str, params: Sequence[float] = ()) -> np.ndarray:
    """O2: the oracle's FP64 matrix for a named gate."""
    out = np.zeros(16, dtype=np.complex128)
    k = _load().orc_gate_matrix(GATE_IDS[name], _dbls(params), _ptr(out))
    if k < 0:
        raise ValueError("unknown gate %s" % name)
    d = 1 << k
    return out[: d * d].reshape(d, d).copy()


def zero_state(n: int, x: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    _load().orc_init_basis(_ptr(psi), n, int(x))
    return psi


def apply(psi: np.ndarray, n: int, o) -> None:
    """O3 for one gate record (in place)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == (1 << n)
    lib = _load()
    if o.name == "U":
        mat = np.ascontiguousarray(o.mat, dtype=np.complex128)
        assert mat.shape == (1 << o.k, 1 << o.k)
        rc = lib.orc_apply_op(_ptr(psi), n, GATE_IDS["U"], o.k, _ints(o.qubits),
                              _dbls(()), _ptr(mat))
    else:
        rc = lib.orc_apply_op(_ptr(psi), n, GATE_IDS[o.name], o.k, _ints(o.qubits),
                              _dbls(o.params), None)
    if rc != 0:
        raise ValueError("oracle rejected op %r" % (o,))


def apply_matrix(psi: np.ndarray, n: int, qubits: Sequence[int], mat: np.ndarray) -> None:
    mat = np.ascontiguousarray(mat, dtype=np.complex128)
    rc = _load().orc_apply_matrix(_ptr(psi), n, len(qubits), _ints(qubits), _ptr(mat))
    if rc != 0:
        raise ValueError("bad qubits")


def run(ops: Iterable, n: int, x0: int = 0, psi: Optional[np.ndarray] = None) -> np.ndarray:
    """O1-O3: psi_out = U_L ... U_1 e_{x0}, gate by gate, in program order."""
    if psi is None:
        psi = zero_state(n, x0)
    for o in ops:
        apply(psi, n, o)
    return psi


def norm(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return float(_load().orc_norm(_ptr(psi), n))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = int(a.size).bit_length() - 1
    out = (ctypes.c_double * 2)()
    _load().orc_inner(_ptr(a), _ptr(b), n, out)
    return complex(out[0], out[1])


def pauli_expval(psi: np.ndarray, term: Sequence, work: Optional[np.ndarray] = None) -> complex:
    """O4 for one Pauli string ((P, q), ...): <psi| P psi>, complex (imaginary
    part ~0 for a Hermitian string; returned as a check)."""
    n = int(psi.size).bit_length() - 1
    if work is None:
        work = np.empty_like(psi)
    paulis = [PAULI_IDS[p] for p, _ in term]
    qubits = [int(q) for _, q in term]
    out = (ctypes.c_double * 2)()
    rc = _load().orc_pauli_expval(_ptr(psi), n, len(term), _ints(paulis), _ints(qubits),
                                  _ptr(work), out)
    if rc != 0:
        raise ValueError("bad Pauli term %r" % (term,))
    return complex(out[0], out[1])


def expval(psi: np.ndarray, hamiltonian: Sequence, per_term: bool = False):
    """sum_k c_k Re <psi|P_k|psi> (or the list of per-term values)."""
    work = np.empty_like(psi)
    vals = [c * pauli_expval(psi, term, work).real for c, term in hamiltonian]
    if per_term:
        return vals
    # fixed-order pairwise combination of the per-term values
    while len(vals) > 1:
        vals = [vals[i] + vals[i + 1] if i + 1 < len(vals) else vals[i]
                for i in range(0, len(vals), 2)]
    return float(vals[0]) if vals else 0.0


def sample(psi: np.ndarray, uniforms: np.ndarray) -> np.ndarray:
    """O6: indices for the given uniforms in [0, 1)."""
    n = int(psi.size).bit_length() - 1
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    out = np.zeros(u.size, dtype=np.uint64)
    rc = _load().orc_sample(_ptr(psi), n, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            int(u.size), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("uniforms must lie in [0, 1)")
    return out


def cdf(psi: np.ndarray) -> np.ndarray:
    """Sequential inclusive prefix of |psi_i|^2 (for boundary checks in tests)."""
    return np.cumsum(psi.real ** 2 + psi.imag ** 2)


# ---------------------------------------------------------------------------
# gradients of E(theta) = <0| U(theta)^dag H U(theta) |0>
# ---------------------------------------------------------------------------

def energy(build_ops, params: np.ndarray, hamiltonian, n: int) -> float:
    return expval(run(build_ops(params), n), hamiltonian)


def param_shift_grad(build_ops, params: np.ndarray, hamiltonian, n: int,
                     indices: Optional[Sequence[int]] = None) -> np.ndarray:
    """Parameter-shift rule, exact for gates exp(-i theta P/2) whose angle is
    a single parameter: dE/dtheta_k = [E(theta + pi/2 e_k) - E(theta - pi/2 e_k)] / 2."""
    params = np.asarray(params, dtype=np.float64)
    idx = range(params.size) if indices is None else indices
    g = np.zeros(len(list(idx)))
    for j, k in enumerate(idx):
        p = params.copy(); p[k] += np.pi / 2
        ep = energy(build_ops, p, hamiltonian, n)
        p[k] -= np.pi
        em = energy(build_ops, p, hamiltonian, n)
        g[j] = 0.5 * (ep - em)
    return g


def finite_diff_grad(build_ops, params: np.ndarray, hamiltonian, n: int,
                     indices: Optional[Sequence[int]] = None, h: float = 1e-5) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    idx = range(params.size) if indices is None else indices
    g = np.zeros(len(list(idx)))
    for j, k in enumerate(idx):
        p = params.copy(); p[k] += h
        ep = energy(build_ops, p, hamiltonian, n)
        p[k] -= 2 * h
        em = energy(build_ops, p, hamiltonian, n)
        g[j] = (ep - em) / (2 * h)
    return g
