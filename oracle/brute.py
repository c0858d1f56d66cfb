"""Brute-force full-unitary construction for small registers (n <= 6).

TEST INFRASTRUCTURE ONLY.  A second, independent construction route used to
pin the oracle's index conventions: every gate becomes an explicit
2^n x 2^n matrix assembled from Kronecker products, with qubit n-1 the
leftmost factor (so qubit q is bit q of the index), and the circuit is the
ordinary matrix product U_L ... U_1.

A k-qubit gate U on qubits (q_0..q_{k-1}) (q_0 = least significant bit of the
local index) is  sum_{r,c} U[r,c] * kron_{q=n-1..0} F_q(r,c),  where
F_q = |r_j><c_j| if q = q_j and the 2x2 identity otherwise.
"""
from __future__ import annotations

from functools import reduce
from typing import Sequence

import numpy as np

_E = [[np.array([[1, 0], [0, 0]], complex), np.array([[0, 1], [0, 0]], complex)],
      [np.array([[0, 0], [1, 0]], complex), np.array([[0, 0], [0, 1]], complex)]]
_I2 = np.eye(2, dtype=complex)


def full_operator(n: int, qubits: Sequence[int], U: np.ndarray) -> np.ndarray:
    k = len(qubits)
    d = 1 << k
    assert U.shape == (d, d) and n <= 8
    pos = {int(q): j for j, q in enumerate(qubits)}
    F = np.zeros((1 << n, 1 << n), dtype=complex)
    for r in range(d):
        for c in range(d):
            if U[r, c] == 0:
                continue
            factors = []
            for q in range(n - 1, -1, -1):
                if q in pos:
                    j = pos[q]
                    factors.append(_E[(r >> j) & 1][(c >> j) & 1])
                else:
                    factors.append(_I2)
            F += U[r, c] * reduce(np.kron, factors)
    return F


def pauli_operator(n: int, term) -> np.ndarray:
    """Full matrix of a Pauli string ((P, q), ...) by Kronecker products."""
    P = {"X": np.array([[0, 1], [1, 0]], complex),
         "Y": np.array([[0, -1j], [1j, 0]], complex),
         "Z": np.array([[1, 0], [0, -1]], complex)}
    mats = {int(q): P[p] for p, q in term}
    return reduce(np.kron, [mats.get(q, _I2) for q in range(n - 1, -1, -1)])


def circuit_unitary(n: int, ops, matrix_of) -> np.ndarray:
    """U_L ... U_1 with each gate's matrix supplied by ``matrix_of(op)``."""
    U = np.eye(1 << n, dtype=complex)
    for o in ops:
        U = full_operator(n, o.qubits, matrix_of(o)) @ U
    return U
