"""CPU checks of the MPS host encoder (one-qubit folding, SWAP routing,
operand re-indexing, ASAP launch levels).

The library's encoder output (site, gate) per update and the launch sizes
come from a host-only debug export; this test replays them with NumPy
(two-site updates split by numpy.linalg.svd in the right-canonical form the
kernels keep, no truncation) and compares the state with the state-vector
oracle.  It also checks that the updates of one launch touch disjoint sites.
"""
import ctypes

import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O
from paper_1807_07914_amd import qsv
from test_oracle_mps import mixed_circuit


def program(n, ops):
    L = qsv.lib()
    f = L.qsv_debug_mps_program
    f.restype = ctypes.c_int
    i64 = ctypes.c_int64
    ol = qsv.OpList(ops)
    nj, nl = i64(), i64()
    qsv.check(f(n, ol.arr, ol.n, None, None, 0, ctypes.byref(nj), None, 0, ctypes.byref(nl)))
    sites = np.zeros(max(1, nj.value), np.int32)
    gates = np.zeros(32 * max(1, nj.value), np.float64)
    counts = np.zeros(max(1, nl.value), np.int32)
    qsv.check(f(n, ol.arr, ol.n, sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                gates.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nj.value, ctypes.byref(nj),
                counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nl.value, ctypes.byref(nl)))
    g = gates.view(np.complex128).reshape(-1, 16)
    return sites[: nj.value], g[: nj.value], counts[: nl.value]


def replay(n, sites, gates, counts):
    B = [np.zeros((1, 2, 1), complex) for _ in range(n)]
    for b in B:
        b[0, 0, 0] = 1
    lam = [np.ones(1) for _ in range(n + 1)]
    j = 0
    for c in counts:
        if c > 0:
            used = set()
            for l, G in zip(sites[j:j + c], gates[j:j + c]):
                assert not ({l, l + 1} & used), "one launch, overlapping sites"
                used |= {l, l + 1}
                cl, cr = B[l].shape[0], B[l + 1].shape[2]
                th = np.einsum("asm,mtc->astc", B[l], B[l + 1])
                Tp = np.einsum("TSts,astc->aSTc", G.reshape(2, 2, 2, 2), th).reshape(2 * cl, 2 * cr)
                _, S, Vh = np.linalg.svd(lam[l].repeat(2)[:, None] * Tp, full_matrices=False)
                k = int(max(1, np.sum(S > 1e-12 * S[0])))
                B[l + 1] = Vh[:k].reshape(k, 2, cr)
                B[l] = (Tp @ Vh[:k].conj().T).reshape(cl, 2, k)
                lam[l + 1] = S[:k]
            j += c
        else:
            for l, G in zip(sites[j:j - c], gates[j:j - c]):
                B[l] = np.einsum("ts,asb->atb", G[:4].reshape(2, 2), B[l])
            j -= c
    assert j == len(sites)
    v = np.ones((1, 1), complex)
    for l in range(n):
        w = np.einsum("xb,bsc->sxc", v, B[l])
        v = w.reshape(-1, w.shape[2])
    return v[:, 0]


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (4, 2), (6, 3), (9, 4)])
def test_encoder_replays_to_the_state_vector(n, seed):
    ops = mixed_circuit(n, 12 * n, seed) if n > 1 else [qc.op("H", 0), qc.op("T", 0), qc.op("RY", 0, params=(0.4,))]
    sites, gates, counts = program(n, ops)
    assert np.abs(replay(n, sites, gates, counts) - O.run(ops, n)).max() < 1e-12


def test_rounds_ladders_share_launches():
    # successive rounds' CNOT ladders overlap diagonally: fewer launches than updates
    n, rounds = 9, 4
    ops = qc.paper_rounds(n, rounds, 77)
    sites, gates, counts = program(n, ops)
    nb = int(np.sum(counts[counts > 0]))
    assert nb == rounds * (n - 1) and len(counts) < nb
    assert max(counts) >= 2
    assert np.abs(replay(n, sites, gates, counts) - O.run(ops, n)).max() < 1e-12
