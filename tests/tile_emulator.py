"""Host-side emulator of the fused tile-pass program (test infrastructure).

Executes the int32 program image that the library's planner emits (exported
by the debug call ``qsv_debug_plan_program``) on a complex128 NumPy state,
decoding every word the way the tile kernel does: pass header, 256-word
round blocks, the XOR-swizzled LDS layout, register groups and the U1 / U2 /
SIGN / PHASE1 / DIAG2 ops.  Comparing its output with the CPU oracle checks
the planner and the encoder on machines without a GPU; it also asserts the
block layout rules the kernel relies on (no op straddles a 64-word line
unless it is longer than one, block bounds).
"""
from __future__ import annotations

import ctypes

import numpy as np

from paper_1807_07914_amd import qsv

ROUND_WORDS = 256
TOP_U1, TOP_U2, TOP_SIGN, TOP_PHASE1, TOP_DIAG2, TOP_PERM2 = 1, 2, 3, 4, 5, 6
TK_REG, TK_FREE, TK_OUT = 0, 1, 2
CFG = {"c64": dict(RB=5, SB=5, WT=1), "c128": dict(RB=4, SB=4, WT=2)}


def program(n, dtype, ops, tile=0):
    ol = ops if isinstance(ops, qsv.OpList) else qsv.OpList(ops)
    L = qsv.lib()
    fn = L.qsv_debug_plan_program
    fn.restype = ctypes.c_int
    i64p = ctypes.POINTER(ctypes.c_int64)
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsv.QsvOp), ctypes.c_int,
                   ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, i64p, i64p,
                   ctypes.c_int64, i64p]
    nw, ns = ctypes.c_int64(), ctypes.c_int64()
    dt = qsv.QSV_C64 if dtype == "c64" else qsv.QSV_C128
    qsv.check(fn(n, dt, ol.arr, ol.n, tile, None, 0, ctypes.byref(nw), None, 0, ctypes.byref(ns)))
    words = np.zeros(max(1, nw.value), dtype=np.int32)
    steps = np.zeros(max(1, ns.value), dtype=np.int64)
    qsv.check(fn(n, dt, ol.arr, ol.n, tile, words.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 nw.value, ctypes.byref(nw), steps.ctypes.data_as(i64p), ns.value,
                 ctypes.byref(ns)))
    return words[: nw.value], steps[: ns.value]


def swizzle(l, B):
    M = (1 << B) - 1
    return l ^ ((l >> B) & M) ^ ((l >> (2 * B)) & M)


def deposit(x, positions):
    out = 0
    for j, p in enumerate(positions):
        if (x >> j) & 1:
            out |= 1 << p
    return out


def pdep_mask(x, mask):
    out, b = 0, 0
    while mask:
        low = mask & -mask
        if (x >> b) & 1:
            out |= low
        mask ^= low
        b += 1
    return out


def _real(blk, k, WT):
    if WT == 1:
        return float(np.int32(blk[k]).view(np.float32))
    lo = np.uint32(np.int32(blk[k]).view(np.uint32))
    hi = np.uint32(np.int32(blk[k + 1]).view(np.uint32))
    return float((np.uint64(hi) << np.uint64(32) | np.uint64(lo)).view(np.float64))


def _cplx(blk, k, WT, count):
    return [complex(_real(blk, k + 2 * e * WT, WT), _real(blk, k + (2 * e + 1) * WT, WT))
            for e in range(count)]


def _apply_dense(psi, n, qubits, U):
    k = len(qubits)
    mask = sum(1 << q for q in qubits)
    for b in range(1 << n):
        if b & mask:
            continue
        idx = [b | deposit(m, qubits) for m in range(1 << k)]
        psi[idx] = U @ psi[idx]


def run_pass(psi, n, words, off, cfg):
    RB, SB, WT = cfg["RB"], cfg["SB"], cfg["WT"]
    NR = 1 << RB
    t, c, nns, nblocks = (int(x) for x in words[off:off + 4])
    S = [int(x) for x in words[off + 4:off + 4 + t]]
    nonS = [int(x) for x in words[off + 4 + t:off + 4 + t + nns]]
    assert S == sorted(S) and S[:c] == list(range(c))
    b0 = off + ((4 + t + nns + 63) & ~63)
    for tid in range(1 << (n - t)):
        base = deposit(tid, nonS)
        lds = np.zeros(1 << t, dtype=np.complex128)
        gidx = [base | deposit(l, S) for l in range(1 << t)]
        for l in range(1 << t):
            lds[swizzle(l, SB)] = psi[gidx[l]]
        for r in range(nblocks):
            blk = [int(x) for x in words[b0 + r * ROUND_WORDS: b0 + (r + 1) * ROUND_WORDS]]
            nops, free_mask = blk[0], blk[1] & 0xffffffff
            lmsw = [blk[2 + m] & 0xffffffff for m in range(NR)]
            for gi in range(1 << (t - RB)):
                lg = pdep_mask(gi, free_mask)
                sg = swizzle(lg, SB)
                a = [lds[sg ^ lmsw[m]] for m in range(NR)]
                k = 2 + NR
                for _ in range(nops):
                    typ, ln = blk[k], blk[k + 1]
                    assert ln >= 2 and k + ln <= ROUND_WORDS
                    if typ in (TOP_U1, TOP_PHASE1) or ln <= 64:
                        assert (k & 63) + min(ln, 64) <= 64 or ln > 64, (typ, k, ln)
                    else:
                        assert k & 63 == 0
                    if typ == TOP_U1:
                        j = blk[k + 2]
                        U = np.array(_cplx(blk, k + 3, WT, 4)).reshape(2, 2)
                        for m in range(NR):
                            if not (m >> j) & 1:
                                m2 = m | (1 << j)
                                a[m], a[m2] = (U[0, 0] * a[m] + U[0, 1] * a[m2],
                                               U[1, 0] * a[m] + U[1, 1] * a[m2])
                    elif typ == TOP_U2:
                        j0, j1 = blk[k + 2], blk[k + 3]
                        assert j0 < j1
                        U = np.array(_cplx(blk, k + 4, WT, 16)).reshape(4, 4)
                        for m in range(NR):
                            if (m >> j0) & 1 or (m >> j1) & 1:
                                continue
                            ii = [m, m | (1 << j0), m | (1 << j1), m | (1 << j0) | (1 << j1)]
                            y = U @ np.array([a[x] for x in ii])
                            for x, v in zip(ii, y):
                                a[x] = v
                    elif typ == TOP_PERM2:
                        j0, j1, code = blk[k + 2:k + 5]
                        assert j0 < j1 and code in (0, 1, 2)
                        sw = {0: (1, 3), 1: (2, 3), 2: (1, 2)}[code]
                        for m in range(NR):
                            if (m >> j0) & 1 or (m >> j1) & 1:
                                continue
                            ii = [m, m | (1 << j0), m | (1 << j1), m | (1 << j0) | (1 << j1)]
                            x, y = ii[sw[0]], ii[sw[1]]
                            a[x], a[y] = a[y], a[x]
                    elif typ == TOP_SIGN:
                        p = k + 2
                        neg = blk[p] & 0xffffffff; p += 1
                        nf = blk[p]; p += 1
                        for _ in range(nf):
                            if (lg >> blk[p]) & 1:
                                neg ^= blk[p + 1] & 0xffffffff
                            p += 2
                        nd = blk[p]; p += 1
                        par = 0
                        for _ in range(nd):
                            par ^= bin(lg & (lg >> blk[p]) & (blk[p + 1] & 0xffffffff)).count("1")
                            p += 2
                        par ^= bin(lg & (blk[p] & 0xffffffff)).count("1"); p += 1
                        nrc = blk[p]; p += 1
                        for _ in range(nrc):
                            if (base >> blk[p]) & 1:
                                neg ^= blk[p + 1] & 0xffffffff
                            p += 2
                        nfc = blk[p]; p += 1
                        for _ in range(nfc):
                            par ^= ((base >> blk[p]) & 1) & ((lg >> blk[p + 1]) & 1)
                            p += 2
                        ncc = blk[p]; p += 1
                        for _ in range(ncc):
                            par ^= (base >> blk[p]) & (base >> blk[p + 1]) & 1
                            p += 2
                        assert p <= k + ln
                        if par & 1:
                            neg = ~neg & 0xffffffff
                        for m in range(NR):
                            if (neg >> m) & 1:
                                a[m] = -a[m]
                    elif typ == TOP_PHASE1:
                        kind, val = blk[k + 2], blk[k + 3]
                        d0, d1 = _cplx(blk, k + 4, WT, 2)
                        for m in range(NR):
                            if kind == TK_REG:
                                bit = (val >> m) & 1
                            elif kind == TK_FREE:
                                bit = (lg >> val) & 1
                            else:
                                bit = (base >> val) & 1
                            a[m] *= d1 if bit else d0
                    elif typ == TOP_DIAG2:
                        ka, va, kb, vb = blk[k + 2:k + 6]
                        d = _cplx(blk, k + 6, WT, 4)

                        def bit(kind, val, m):
                            if kind == TK_REG:
                                return (val >> m) & 1
                            if kind == TK_FREE:
                                return (lg >> val) & 1
                            return (base >> val) & 1
                        for m in range(NR):
                            a[m] *= d[bit(ka, va, m) + 2 * bit(kb, vb, m)]
                    else:
                        assert typ == 0, typ
                    k += ln
                for m in range(NR):
                    lds[sg ^ lmsw[m]] = a[m]
        for l in range(1 << t):
            psi[gidx[l]] = lds[swizzle(l, SB)]


def emulate(n, dtype, ops, psi0, tile=0, matrix_of=None):
    """Run the fused plan of ``ops`` on psi0 (complex128, copied)."""
    words, steps = program(n, dtype, ops, tile)
    psi = np.array(psi0, dtype=np.complex128)
    cfg = CFG[dtype]
    for st in steps:
        if st < 0:
            o = ops[int(-st - 1)]
            _apply_dense(psi, n, list(o.qubits), np.asarray(o.mat, dtype=np.complex128))
        else:
            run_pass(psi, n, words, int(st), cfg)
    return psi


def batch_program(dtype, circuits, widths, tile):
    flat = [o for c in circuits for o in c]
    offs = np.zeros(len(circuits) + 1, dtype=np.int32)
    for i, c in enumerate(circuits):
        offs[i + 1] = offs[i] + len(c)
    toff = np.zeros(len(circuits) + 1, dtype=np.int32)
    w = np.asarray(widths, dtype=np.int32)
    ol = qsv.OpList(flat)
    fn = qsv.lib().qsv_debug_batch_program
    fn.restype = ctypes.c_int
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    fn.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.POINTER(qsv.QsvOp), i32p,
                   ctypes.c_int, i32p, ctypes.c_int64, i64p, i64p, ctypes.c_int64, i64p, i64p]
    dt = qsv.QSV_C64 if dtype == "c64" else qsv.QSV_C128
    nw, npz = ctypes.c_int64(), ctypes.c_int64()
    args = (dt, len(circuits), w.ctypes.data_as(i32p), offs.ctypes.data_as(i32p), ol.arr,
            toff.ctypes.data_as(i32p), tile)
    qsv.check(fn(*args, None, 0, ctypes.byref(nw), None, 0, ctypes.byref(npz), None))
    words = np.zeros(max(1, nw.value), dtype=np.int32)
    passoff = np.zeros(max(1, npz.value), dtype=np.int64)
    jobs = np.zeros(8 * len(circuits), dtype=np.int64)
    qsv.check(fn(*args, words.ctypes.data_as(i32p), nw.value, ctypes.byref(nw),
                 passoff.ctypes.data_as(i64p), npz.value, ctypes.byref(npz),
                 jobs.ctypes.data_as(i64p)))
    return words, passoff, jobs.reshape(-1, 8)


def emulate_batch_job(dtype, words, passoff, job):
    """Final state of one batch job (init from |0...0> in the first pass)."""
    w, np_, p0 = int(job[0]), int(job[1]), int(job[2])
    psi = np.zeros(1 << w, dtype=np.complex128)
    psi[0] = 1.0
    for p in range(np_):
        off = int(passoff[p0 + p])
        t = int(words[off])
        assert 1 <= t <= w, (t, w)
        run_pass(psi, w, words, off, CFG[dtype])
    return psi
