"""Matrix-product-state oracle (test infrastructure only).

Imported only by the tests, the smoke check and the benchmark's CPU baseline;
the library never calls it.  Plain NumPy in complex128, written from the
paper's description of its MPS visitor (section III, the figure on gate
application by SVD; section IV.B, the ITensor MPS instruction visitor):

- the state is held in the canonical form the paper names: n rank-3 site
  tensors Gamma[l] of shape (chi_l, 2, chi_{l+1}) and n - 1 diagonal bond
  matrices Lambda[b] (b = 1 .. n-1, between sites b-1 and b), with
  Lambda[0] = Lambda[n] = [1];
- a one-qubit gate contracts with its site tensor and leaves the form as it is;
- a two-qubit gate on adjacent sites l, l+1 contracts with the two site
  tensors and the three bond matrices around them into a rank-4 tensor, which
  is reshaped to a (2 chi_l) x (2 chi_{l+2}) matrix and split by an SVD; the
  singular values below the cutoff epsilon are dropped (the paper's default
  is 1e-4) and the kept ones become the new bond matrix; the new site tensors
  are the singular vectors with the outer bond matrices divided back out;
- a two-qubit gate on qubits further apart is routed with SWAP gates on
  adjacent sites: the higher qubit is swapped down next to the lower one,
  the gate applied, and the chain swapped back, so qubit q always lives at
  site q between instructions.

Readings (the paper is silent on these): the cutoff is absolute on the
singular values, which are the Schmidt coefficients of a normalised state in
this form; values not above 1e-12 of the largest are numerical zeros and are
dropped as well; at most ``chi_max`` values are kept and at least one; the
state is not renormalised after truncation.

Pinned by tests/test_oracle_mps.py against the state-vector oracle (exact
runs), the SVD of the state vector across every cut (Schmidt values), the
GHZ and product states, the paper's chi = 4 at two rounds, and the norm and
overlap of a single truncation.
"""
from __future__ import annotations

from typing import Iterable, Optional

import numpy as np

from oracle import oracle as O

ZERO_REL = 1e-12   # relative numerical-zero rule for singular values
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


class MPS:
    """|0...0> on n qubits in Gamma/Lambda form; qubit q at site q."""

    def __init__(self, n: int, chi_max: int = 1 << 30, cutoff: float = 1e-4):
        self.n, self.chi_max, self.cutoff = n, chi_max, cutoff
        self.gam = []
        for _ in range(n):
            g = np.zeros((1, 2, 1), dtype=np.complex128)
            g[0, 0, 0] = 1.0
            self.gam.append(g)
        self.lam = [np.ones(1) for _ in range(n + 1)]
        self.discarded = 0.0   # sum of squared dropped singular values

    # section III: a one-body gate touches one site tensor only
    def apply1(self, q: int, U: np.ndarray) -> None:
        self.gam[q] = np.einsum("ts,asb->atb", U, self.gam[q])

    # section III figure / IV.B: contract, SVD, truncate, split
    def bond_update(self, l: int, G: np.ndarray) -> None:
        """G: 4x4 with local index (bit of site l) + 2 (bit of site l+1)."""
        L0, L1, L2 = self.lam[l], self.lam[l + 1], self.lam[l + 2]
        A, B = self.gam[l], self.gam[l + 1]
        theta = np.einsum("a,asm,m,mtc,c->astc", L0, A, L1, B, L2)
        Gr = G.reshape(2, 2, 2, 2)          # axes (t', s', t, s): row index = s' + 2 t'
        theta2 = np.einsum("TSts,astc->aSTc", Gr, theta)
        cl, cr = theta2.shape[0], theta2.shape[3]
        U, S, Vh = np.linalg.svd(theta2.reshape(2 * cl, 2 * cr), full_matrices=False)
        keep = (S > self.cutoff) & (S > ZERO_REL * S[0])
        k = int(min(max(1, keep.sum()), self.chi_max))
        self.discarded += float(np.sum(S[k:] ** 2))
        self.lam[l + 1] = S[:k].copy()
        self.gam[l] = U[:, :k].reshape(cl, 2, k) / L0[:, None, None]
        self.gam[l + 1] = Vh[:k].reshape(k, 2, cr) / L2[None, None, :]

    def apply2(self, q0: int, q1: int, G: np.ndarray) -> None:
        """G: 4x4 with local index bit(q0) + 2 bit(q1) (q0 the first listed qubit)."""
        lo, hi = min(q0, q1), max(q0, q1)
        if q0 != lo:   # re-index so that the lower site's bit is the low bit
            P = SWAP
            G = P @ G @ P
        for b in range(hi - 1, lo, -1):     # bring qubit hi to site lo + 1
            self.bond_update(b, SWAP)
        self.bond_update(lo, G)
        for b in range(lo + 1, hi):         # and back
            self.bond_update(b, SWAP)

    def to_state(self) -> np.ndarray:
        """Amplitudes psi[i], bit q of i = qubit q (the state-vector convention)."""
        v = np.ones((1, 1), dtype=np.complex128)     # (2^l, chi_l)
        for l in range(self.n):
            w = np.einsum("xb,b,bsc->sxc", v, self.lam[l], self.gam[l])
            v = w.reshape(-1, w.shape[2])
        return v[:, 0] * self.lam[self.n][0]

    def amplitude(self, x: int) -> complex:
        """One amplitude <x|psi>, site by site (for registers too wide to expand)."""
        v = np.ones(1, dtype=np.complex128)
        for l in range(self.n):
            v = (v * self.lam[l]) @ self.gam[l][:, (x >> l) & 1, :]
        return complex(v[0] * self.lam[self.n][0])

    def bond_dims(self) -> list:
        return [len(x) for x in self.lam]

    def memory_bytes(self) -> int:
        """Bytes of the site tensors and bond matrices (complex128 / float64)."""
        return sum(g.size * 16 for g in self.gam) + sum(x.size * 8 for x in self.lam)


def op_matrix(o) -> np.ndarray:
    if getattr(o, "mat", None) is not None:
        return np.asarray(o.mat, dtype=np.complex128)
    return O.gate_matrix(o.name, o.params)


def run(ops: Iterable, n: int, chi_max: int = 1 << 30, cutoff: float = 1e-4,
        mps: Optional[MPS] = None) -> MPS:
    """Apply an instruction list in program order."""
    m = mps if mps is not None else MPS(n, chi_max, cutoff)
    for o in ops:
        U = op_matrix(o)
        if len(o.qubits) == 1:
            m.apply1(o.qubits[0], U)
        elif len(o.qubits) == 2:
            m.apply2(o.qubits[0], o.qubits[1], U)
        else:
            raise ValueError("the MPS path takes one- and two-qubit instructions")
    return m
