"""CPU emulation of the adjoint sweep's tile programs (test infrastructure).

The library's host encoder turns the reversed gate list into tile programs
(op records, sign runs, register rounds, gradient slots) for the sweep
kernel.  This module decodes those programs from the debug export and
applies every record to full complex128 state vectors with the oracle's
gate application, so that the encoder (grouping, reordering past commuting
ops, record layouts, slot maps, program splits) can be checked against the
oracle's parameter-shift gradients without a GPU.  A record that acts on
the local bits of each tile acts on the whole state the same way, with
local bit j standing for qubit S[j].
"""
import ctypes

import numpy as np

from oracle import oracle as O
from paper_1807_07914_amd import qsv
from tile_emulator import expand_cnots

REC_WORDS, GATE_WORDS = 72, 20
ROUND_BITS = {"c64": 4, "c128": 3}
PAULI = {"X": O.gate_matrix("X"), "Y": O.gate_matrix("Y"), "Z": O.gate_matrix("Z")}


def program(n, dtype, ops):
    """(words, actions): actions[i] >= 0 is a program offset, -(op + 1) an op
    applied as its inverse by the per-gate kernels."""
    ol = ops if isinstance(ops, qsv.OpList) else qsv.OpList(ops)
    fn = qsv.lib().qsv_debug_adjoint_program
    fn.restype = ctypes.c_int
    i64p = ctypes.POINTER(ctypes.c_int64)
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsv.QsvOp), ctypes.c_int,
                   ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, i64p, i64p, ctypes.c_int64, i64p]
    dt = qsv.QSV_C64 if dtype == "c64" else qsv.QSV_C128
    nw, ns = ctypes.c_int64(), ctypes.c_int64()
    qsv.check(fn(n, dt, ol.arr, ol.n, None, 0, ctypes.byref(nw), None, 0, ctypes.byref(ns)))
    words = np.zeros(max(1, nw.value), dtype=np.int32)
    acts = np.zeros(max(1, ns.value), dtype=np.int64)
    qsv.check(fn(n, dt, ol.arr, ol.n, words.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nw.value,
                 ctypes.byref(nw), acts.ctypes.data_as(i64p), ns.value, ctypes.byref(ns)))
    return words[: nw.value], [int(a) for a in acts[: ns.value]]


def _f64(words, k):
    return float(np.array(words[k:k + 2], dtype=np.int32).view(np.float64)[0])


def _cd(words, k):
    return complex(_f64(words, k), _f64(words, k + 2))


def _gen_term(lam, psi, n, q, gen):
    """Im <lambda| G_q |psi> for G = X, Y, Z (0, 1, 2) on qubit q."""
    v = psi.copy()
    O.apply_matrix(v, n, [q], PAULI["XYZ"[gen]])
    return float(np.vdot(lam, v).imag)


def _apply(psi, lam, n, qubits, U):
    O.apply_matrix(psi, n, list(qubits), U)
    O.apply_matrix(lam, n, list(qubits), U)


def _sign_run(rec, n, psi, lam, loc, base, idx):
    """A sign-run block (type-5 layout) applied to both states."""
    assert int(rec[0]) == 5
    nd, nlo, noo = int(rec[1]), int(rec[2]), int(rec[3])
    w = [int(x) for x in rec[8:8 + 2 * (nd + nlo + noo)]]
    assert len(w) == 2 * (nd + nlo + noo)
    par = np.zeros(1 << n, dtype=np.int64)
    for i in range(nd):
        dist, M = w[2 * i], w[2 * i + 1]
        par += np.vectorize(lambda v: bin(v).count("1"))(loc & (loc >> dist) & M)
    for i in range(nlo):
        lb, oq = w[2 * (nd + i)], w[2 * (nd + i) + 1]
        on = np.ones_like(idx) if oq < 0 else (base >> oq) & 1
        par += on * ((loc >> lb) & 1)
    for i in range(noo):
        qa, qb = w[2 * (nd + nlo + i)], w[2 * (nd + nlo + i) + 1]
        par += (base >> qa) & (base >> qb) & 1
    sg = np.where(par & 1, -1.0, 1.0)
    psi *= sg
    lam *= sg


def run_program(words, off, n, dtype, psi, lam, grads):
    t, c, nns, nops, ngrad, roff, moff, ntph = (int(x) for x in words[off:off + 8])
    seen_tph = 0
    S = [int(x) for x in words[off + 8:off + 8 + t]]
    assert S[:c] == list(range(c)) and len(set(S)) == t and 0 < t <= n and nns == n - t
    slot_g = np.zeros(max(ngrad, 1))
    used = set()
    idx = np.arange(1 << n, dtype=np.int64)
    loc = np.zeros(1 << n, dtype=np.int64)
    for j, q in enumerate(S):
        loc |= ((idx >> q) & 1) << j
    base = idx.copy()
    for q in S:
        base &= ~(1 << q)
    r = off + roff
    for _ in range(nops):
        typ = int(words[r])
        if typ == 6:
            K = ROUND_BITS[dtype]
            counts, length = int(words[r + 2]), int(words[r + 3])
            bits = [int(x) for x in words[r + 4:r + 4 + K]]
            assert bits == sorted(bits) and len(set(bits)) == K and max(bits) < t
            ngate = sum((counts >> (8 * j)) & 255 for j in range(K))
            soff = int(words[r + 1])
            if soff:  # a sign run that precedes the round, applied at its load
                assert soff == 8 + GATE_WORDS * ngate and length > soff and (length - soff) % 8 == 0
                _sign_run(words[r + soff:r + length], n, psi, lam, loc, base, idx)
            else:
                assert length == 8 + GATE_WORDS * ngate
            last_j = -1
            for e in range(ngate):
                gw = r + 8 + GATE_WORDS * e
                info, slot = int(words[gw]), int(words[gw + 1])
                j, gen = info & 15, (info >> 8) & 3
                assert j >= last_j, "round gates grouped by register bit"
                last_j = j
                ft = np.float32 if dtype == "c64" else np.float64
                nb = 8 * (4 if dtype == "c64" else 8)
                m = np.frombuffer(np.array(words[gw + 4:gw + 4 + nb // 4], dtype=np.int32).tobytes(), dtype=ft)
                U = (m[0::2].astype(np.float64) + 1j * m[1::2].astype(np.float64)).reshape(2, 2)
                q = S[bits[j]]
                if slot >= 0:
                    slot_g[slot] += _gen_term(lam, psi, n, q, gen)
                    used.add(slot)
                _apply(psi, lam, n, [q], U)
            for j in range(K):  # the counts match the gates' bits
                assert (counts >> (8 * j)) & 255 == sum(
                    1 for e in range(ngate) if int(words[r + 8 + GATE_WORDS * e]) & 15 == j)
            r += length
            continue
        rec = words[r:r + REC_WORDS]
        a, b, slot, gen = int(rec[1]), int(rec[2]), int(rec[3]), int(rec[4])
        if typ == 1:
            U = np.array([_cd(rec, 8 + 4 * e) for e in range(4)]).reshape(2, 2)
            if slot >= 0:
                slot_g[slot] += _gen_term(lam, psi, n, S[a], gen)
                used.add(slot)
            _apply(psi, lam, n, [S[a]], U)
        elif typ == 7:
            # a phase per tile: diag(d0, d1) on a qubit outside the tile; the
            # kernel applies it at the tile's store, which gives the same
            # states and the same gradient term as applying it here
            q = a
            assert q not in S and 0 <= q < n and b == -1
            d0, d1 = _cd(rec, 8), _cd(rec, 12)
            assert abs(abs(d0) - 1) < 1e-12 and abs(abs(d1) - 1) < 1e-12
            bit = (idx >> q) & 1
            if slot >= 0:
                slot_g[slot] += float(np.sum(np.where(bit == 1, -1.0, 1.0) * (np.conj(lam) * psi).imag))
                used.add(slot)
            fac = np.where(bit == 1, d1, d0)
            psi *= fac
            lam *= fac
            seen_tph += 1
        elif typ == 2:
            d = [_cd(rec, 8 + 4 * e) for e in range(4)]

            def qubit(opnd):
                return S[opnd & 255] if (opnd >> 8) == 0 else opnd & 255
            bA = (idx >> qubit(a)) & 1
            bB = (idx >> qubit(b)) & 1 if b >= 0 else np.zeros_like(idx)
            fac = np.array(d)[bA + 2 * bB]
            if slot >= 0:  # generator Z on operand a
                slot_g[slot] += float(np.sum(np.where(bA == 1, -1.0, 1.0) * (np.conj(lam) * psi).imag))
                used.add(slot)
            psi *= fac
            lam *= fac
        elif typ == 3:
            U = np.array([_cd(rec, 8 + 4 * e) for e in range(16)]).reshape(4, 4)
            assert a < b and slot < 0
            _apply(psi, lam, n, [S[a], S[b]], U)
        elif typ == 5:
            _sign_run(rec, n, psi, lam, loc, base, idx)
        else:
            raise AssertionError("unknown record type %d" % typ)
        r += REC_WORDS
    assert seen_tph == ntph, "header word 7 counts the tile-phase records"
    assert sorted(used) == list(range(ngrad)), "every gradient slot taken once"
    omap = [int(x) for x in words[off + moff:off + moff + ngrad]]
    for sl, op in enumerate(omap):
        grads[op] += slot_g[sl]


def hamiltonian_apply(psi, n, ham):
    lam = np.zeros_like(psi)
    for coeff, term in ham:
        v = psi.copy()
        for p, q in term:
            O.apply_matrix(v, n, [q], PAULI[p])
        lam += coeff * v
    return lam


def emulate(n, dtype, ops, ham, x0=0):
    """(energy, gradient per op, state after the sweep) from the emulated programs."""
    psi = O.run(ops, n, x0=x0)
    lam = hamiltonian_apply(psi, n, ham)
    energy = float(np.vdot(psi, lam).real)
    words, acts = program(n, dtype, ops)
    grads = np.zeros(len(ops))
    xops = expand_cnots(list(ops))  # per-gate steps index the list with CNOT as H CZ H
    for a in acts:
        if a >= 0:
            run_program(words, a, n, dtype, psi, lam, grads)
        else:
            o = xops[-a - 1]
            M = o.mat if o.mat is not None else O.gate_matrix(o.name, o.params)
            _apply(psi, lam, n, o.qubits, np.conj(np.asarray(M)).T)
    return energy, grads, psi
