"""Host-side emulator of the fused tile-pass program (test infrastructure).

Executes the int32 program image that the library's planner emits (exported
by the debug call ``qsv_debug_plan_program``) on a complex128 NumPy state,
decoding every word the way the tile kernel does: pass header and round
offsets, round blocks (header, fixed-layout layer records, aux words,
tables), the XOR-swizzled LDS layout, register groups and every step.
Comparing its output with the CPU oracle checks the planner and the encoder
on machines without a GPU; it also asserts the layout rules the kernel
relies on (record fields in range, aux words consumed exactly, tables inside
the program).
"""
from __future__ import annotations

import ctypes

import numpy as np

import qcircuits as qc
from paper_1807_07914_amd import qsv

ROUND_HEADER = 32   # words of a round block header
REC_ROT = 4         # first rotation word of a layer record
TABLE_WORDS = 64
LT_TAB, LT_CZR, LT_SIGN, LT_PHASEL, LT_RAWD, LT_CZF = 1, 2, 4, 8, 16, 32
LT_ROT0, LT_SHEAR3 = 1 << 8, 1 << 16
LT_PERM2, LT_U2, LT_U1 = 1 << 24, 1 << 25, 1 << 26
RAW_PHASE1, RAW_DIAG2 = 4, 5
TK_REG, TK_FREE, TK_OUT = 0, 1, 2
CFG = {"c64": dict(RB=5, SB=5, WT=1, LR=16), "c128": dict(RB=4, SB=4, WT=2, LR=24)}
TILE_FAC_HDR, MAX_TILE_FACTORS = 8, 128  # round-header word of the tile-factor list; slot cap
STORE_HDR = 10  # round-header words of the store's register-bit offsets
MAP_HDR = 16    # round-header word of the store map's offset (0: none)
LANE_TAB_HDR, LANE_TAB_N_HDR = 7, 15  # first round's header: lane-table offset, entries
LANE_TAB_BYTES = 8192


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


def _shear3(x, p, q):
    """exp(i phi) x as three shears of (re, im), as the kernel does."""
    re, im = x.real, x.imag
    re = re + p * im
    im = im + q * re
    re = re + p * im
    return complex(re, im)


def _round_blocks(words, off, t, nns):
    """(start, n_layers, free mask, bit offsets) of each round block."""
    nrounds = int(words[off + 3])
    roff = [int(x) for x in words[off + 4 + t + nns: off + 4 + t + nns + nrounds]]
    out = []
    for r in range(nrounds):
        rb = off + roff[r]
        assert roff[r] > 0 and rb + ROUND_HEADER <= len(words)
        out.append(rb)
    return out


def _record_offsets(blk, nlay, LR):
    """Offsets of the layer records of a round block (each record is followed
    by its table if it has one), plus the end of the last one."""
    out = [ROUND_HEADER]
    for _ in range(nlay):
        k = out[-1]
        out.append(k + LR + (TABLE_WORDS if blk[k] & LT_TAB else 0))
    return out


def run_pass(psi, n, words, off, cfg):
    RB, SB, WT, LR = cfg["RB"], cfg["SB"], cfg["WT"], cfg["LR"]
    NR = 1 << RB
    words = [int(x) for x in words]
    t, c, nns = (int(x) for x in words[off:off + 3])
    S = [int(x) for x in words[off + 4:off + 4 + t]]
    nonS = [int(x) for x in words[off + 4 + t:off + 4 + t + nns]]
    assert S == sorted(S) and S[:c] == list(range(c))
    blocks = _round_blocks(words, off, t, nns)
    esz = 8 * WT  # bytes per amplitude: the header holds LDS byte offsets
    # the pass's tile-factor list (pointed to by the first round's header)
    lane = []  # the pass's lane table (complex entries)
    if blocks:
        lo, ne = words[blocks[0] + LANE_TAB_HDR], words[blocks[0] + LANE_TAB_N_HDR]
        assert 0 <= ne <= LANE_TAB_BYTES // (8 * WT) and (ne == 0 or lo > 0)
        if ne:
            lane = _cplx(words, off + lo, WT, ne)
    tfl = []
    if blocks:
        lo, nk = words[blocks[0] + TILE_FAC_HDR], words[blocks[0] + TILE_FAC_HDR + 1]
        assert 0 <= nk <= MAX_TILE_FACTORS and (nk == 0 or lo > 0)
        for k in range(nk):
            e = off + lo + words[off + lo + k]
            terms = []
            for q in range(words[e]):
                tm = e + 1 + q * (2 + 2 * WT)
                om = (words[tm] & 0xffffffff) | ((words[tm + 1] & 0xffffffff) << 32)
                terms.append((om, _cplx(words, tm + 2, WT, 1)[0]))
            tfl.append(terms)
    for tid in range(1 << (n - t)):
        base = deposit(tid, nonS)
        tfac = []
        for terms in tfl:
            f = 1.0 + 0j
            for om, r_ in terms:
                if (base & om) == om:
                    f *= r_
            tfac.append(f)
        lds = np.zeros(1 << t, dtype=np.complex128)
        gidx = [base | deposit(l, S) for l in range(1 << t)]
        for l in range(1 << t):
            lds[swizzle(l, SB)] = psi[gidx[l]]
        for rb in blocks:
            blk = words[rb:]  # offsets in a round block count from its start
            nlay, free_mask = blk[0], blk[1] & 0xffffffff
            assert all((blk[2 + j] & 0xffffffff) % esz == 0 for j in range(RB))
            bsw = [(blk[2 + j] & 0xffffffff) // esz for j in range(RB)]
            lmsw = []
            for m in range(NR):
                o_ = 0
                for j in range(RB):
                    if (m >> j) & 1:
                        o_ ^= bsw[j]
                lmsw.append(o_)
            recs_at = _record_offsets(blk, nlay, LR)
            rec_end = recs_at[-1] if recs_at else ROUND_HEADER
            moff = blk[MAP_HDR]
            if moff:
                # store map: one offset per free bit, then the outside
                # controls; the kernel loads every group before any store
                assert moff >= rec_end
                nf = bin(free_mask).count("1")
                fcol = [(blk[moff + i] & 0xffffffff) for i in range(nf)]
                no = blk[moff + nf]
                ocol = [(blk[moff + nf + 1 + 2 * k], blk[moff + nf + 2 + 2 * k] & 0xffffffff) for k in range(no)]
                assert all(v % esz == 0 for v in fcol) and all(0 <= q < n and v % esz == 0 for q, v in ocol)
                assert all(q not in S for q, _ in ocol)
                obase = 0
                for q, v in ocol:
                    if (base >> q) & 1:
                        obase ^= v // esz
            stores = []
            for gi in range(1 << (t - RB)):
                lg = pdep_mask(gi, free_mask)
                sg = swizzle(lg, SB)
                a = [lds[sg ^ lmsw[m]] for m in range(NR)]
                for li in range(nlay):
                    rec = blk[recs_at[li]: recs_at[li] + LR]
                    flags = rec[0]
                    p = rec[3]  # aux words
                    if flags & (LT_CZF | LT_SIGN | LT_PHASEL | LT_RAWD | LT_PERM2 | LT_U2 | LT_U1):
                        assert p >= rec_end
                    if flags & LT_TAB:
                        tl = recs_at[li] + LR  # the table follows its record
                        assert tl + TABLE_WORDS <= len(blk)
                        for m in range(NR):
                            zr = _real(blk, tl + 2 * m * WT, WT)
                            zi = _real(blk, tl + (2 * m + 1) * WT, WT)
                            a[m] = a[m] * complex(zr, zi)
                    if flags & LT_CZR:
                        pairs = rec[2] & 0xffffffff
                        for kk in range(1, RB):
                            for jj in range(kk):
                                if (pairs >> (kk * (kk - 1) // 2 + jj)) & 1:
                                    for m in range(NR):
                                        if (m >> jj) & 1 and (m >> kk) & 1:
                                            a[m] = -a[m]
                        assert pairs >> (RB * (RB - 1) // 2) == 0
                    if flags & LT_CZF:
                        ne = blk[p]; p += 1
                        for _ in range(ne):
                            w_ = blk[p]; p += 1
                            jj, kind, val = w_ & 15, (w_ >> 4) & 15, w_ >> 8
                            assert jj < RB and kind in (TK_FREE, TK_OUT)
                            on = (lg >> val) & 1 if kind == TK_FREE else (base >> val) & 1
                            if on:
                                for m in range(NR):
                                    if (m >> jj) & 1:
                                        a[m] = -a[m]
                    if flags & LT_SIGN:
                        par = 0
                        nd = blk[p]; p += 1
                        for _ in range(nd):
                            par ^= bin(lg & (lg >> blk[p]) & (blk[p + 1] & 0xffffffff)).count("1")
                            p += 2
                        nfc = blk[p]; p += 1
                        for _ in range(nfc):
                            par ^= ((base >> blk[p]) & 1) & ((lg >> blk[p + 1]) & 1)
                            p += 2
                        ncc = blk[p]; p += 1
                        for _ in range(ncc):
                            par ^= (base >> blk[p]) & (base >> blk[p + 1]) & 1
                            p += 2
                        if par & 1:
                            a = [-x for x in a]
                    if flags & LT_PHASEL:
                        j, slot, unit, nt = blk[p], blk[p + 1], blk[p + 2], blk[p + 3]
                        p += 4
                        assert -1 <= j < RB and -1 <= slot < len(tfl) and unit in (0, 1)
                        w = tfac[slot] if slot >= 0 else 1.0 + 0j
                        if nt == -1:  # lane-table form
                            e0 = blk[p]
                            p += 1
                            assert 0 <= e0 and e0 + 32 <= len(lane)
                            w *= lane[e0 + (gi & 15)] * lane[e0 + 16 + ((gi >> 4) & 15)]
                            nt = 0
                        for _ in range(nt):
                            lgm = blk[p] & 0xffffffff
                            om = (blk[p + 1] & 0xffffffff) | ((blk[p + 2] & 0xffffffff) << 32)
                            r_ = _cplx(blk, p + 3, WT, 1)[0]
                            if (lg & lgm) == lgm and (base & om) == om:
                                w *= r_
                            p += 3 + 2 * WT
                        if unit:
                            assert abs(abs(w) - 1.0) < 1e-6  # factors stored in the state precision
                        for m in range(NR):
                            if j < 0 or (m >> j) & 1:
                                a[m] *= w
                    if flags & LT_RAWD:
                        typ = blk[p]
                        assert typ in (RAW_PHASE1, RAW_DIAG2)
                        ops_ = blk[p + 1:p + (5 if typ == RAW_DIAG2 else 3)]
                        p += 5 if typ == RAW_DIAG2 else 3
                        nfac = 4 if typ == RAW_DIAG2 else 2
                        fac = []
                        for f in range(nfac):
                            fp_, fq_, fc_ = (_real(blk, p + (3 * f + e) * WT, WT) for e in range(3))
                            fac.append((fp_, fq_, fc_))
                        p += 3 * nfac * WT

                        def bit(kind, val, m):
                            if kind == TK_REG:
                                return (val >> m) & 1
                            if kind == TK_FREE:
                                return (lg >> val) & 1
                            return (base >> val) & 1
                        for m in range(NR):
                            sel = bit(ops_[0], ops_[1], m)
                            if typ == RAW_DIAG2:
                                sel += 2 * bit(ops_[2], ops_[3], m)
                            fp_, fq_, fc_ = fac[sel]
                            a[m] = _shear3(a[m], fp_, fq_) * (1.0 + fc_)
                    for j in range(RB):
                        if flags & (LT_ROT0 << j):
                            p_ = _real(rec, REC_ROT + 2 * j * WT, WT)
                            q_ = _real(rec, REC_ROT + (2 * j + 1) * WT, WT)
                            three = bool(flags & (LT_SHEAR3 << j))
                            # three shears: |tan(theta/2)|, |sin(theta)| <= 1;
                            # two: |tan(theta)| <= 3.2 (cos >= 0.3), |sin cos| <= 1/2
                            if three:
                                assert abs(p_) <= 1.0 + 1e-6 and abs(q_) <= 1.0 + 1e-6, (p_, q_, flags)
                            else:
                                assert abs(p_) <= 3.2 and abs(q_) <= 0.5 + 1e-6
                            for m in range(NR):
                                if not (m >> j) & 1:
                                    m2 = m | (1 << j)
                                    a[m] += p_ * a[m2]
                                    a[m2] += q_ * a[m]
                                    if three:
                                        a[m] += p_ * a[m2]
                    if flags & LT_PERM2:
                        j0, j1, code = blk[p:p + 3]
                        p += 3
                        assert j0 < j1 and code in (0, 1, 2)
                        sw = {0: (1, 3), 1: (2, 3), 2: (1, 2)}[code]
                        for m in range(NR):
                            if (m >> j0) & 1 or (m >> j1) & 1:
                                continue
                            ii = [m, m | (1 << j0), m | (1 << j1), m | (1 << j0) | (1 << j1)]
                            x, y = ii[sw[0]], ii[sw[1]]
                            a[x], a[y] = a[y], a[x]
                    if flags & LT_U2:
                        j0, j1 = blk[p], blk[p + 1]
                        assert j0 < j1
                        U = np.array(_cplx(blk, p + 2, WT, 16)).reshape(4, 4)
                        p += 2 + 32 * WT
                        for m in range(NR):
                            if (m >> j0) & 1 or (m >> j1) & 1:
                                continue
                            ii = [m, m | (1 << j0), m | (1 << j1), m | (1 << j0) | (1 << j1)]
                            y = U @ np.array([a[x] for x in ii])
                            for x, v in zip(ii, y):
                                a[x] = v
                    if flags & LT_U1:
                        j = blk[p]
                        U = np.array(_cplx(blk, p + 1, WT, 4)).reshape(2, 2)
                        p += 1 + 8 * WT
                        for m in range(NR):
                            if not (m >> j) & 1:
                                m2 = m | (1 << j)
                                a[m], a[m2] = (U[0, 0] * a[m] + U[0, 1] * a[m2],
                                               U[1, 0] * a[m] + U[1, 1] * a[m2])
                    # the next record's aux words (if any) start where these end
                    if li + 1 < nlay:
                        nxt = blk[recs_at[li + 1] + 3]
                        if nxt and flags & (LT_CZF | LT_SIGN | LT_PHASEL | LT_RAWD | LT_PERM2 | LT_U2 | LT_U1):
                            assert p == nxt, (hex(flags), p, nxt)
                # the store walks its own register-bit offsets (a permutation
                # that ends the round is folded into them)
                ssw = [(blk[STORE_HDR + j] & 0xffffffff) // esz for j in range(RB)]
                sgs = sg
                if moff:
                    sgs = obase
                    for i in range(nf):
                        if (gi >> i) & 1:
                            sgs ^= fcol[i] // esz
                for m in range(NR):
                    o_ = 0
                    for j in range(RB):
                        if (m >> j) & 1:
                            o_ ^= ssw[j]
                    stores.append((sgs ^ o_, a[m]))
            # every group has loaded before the first store
            dst = [k for k, _ in stores]
            assert len(set(dst)) == len(dst) == 1 << t, "the store must be a bijection of the tile"
            for k, v in stores:
                lds[k] = v
        for l in range(1 << t):
            psi[gidx[l]] = lds[swizzle(l, SB)]


def expand_cnots(ops):
    """The op list the library's adjoint plan indexes: each CNOT(c, t) taken
    as H(t), CZ(c, t), H(t)."""
    out = []
    for o in ops:
        if o.name == "CNOT":
            c, t = o.qubits
            out += [qc.op("H", t), qc.op("CZ", c, t), qc.op("H", t)]
        else:
            out.append(o)
    return out


QPERM = -1   # n_rounds word of a qubit-permutation pass


def is_qperm(words, off):
    return off >= 0 and int(words[off + 3]) == QPERM


def relabel_swaps(ops, n):
    """The op list with its SWAPs relabeled away (a SWAP exchanges which bit
    holds which qubit; later ops act on the bits of their qubits)."""
    lab = list(range(n))
    out = []
    for o in ops:
        if o.name == "SWAP":
            a, b = o.qubits
            lab[a], lab[b] = lab[b], lab[a]
            continue
        out.append(qc.op(o.name, *[lab[q] for q in o.qubits], params=o.params, mat=o.mat))
    return out


def qperm_sigma(words, off, n):
    """The involution of a qubit-permutation pass, checked for the layout
    rules: S holds the low c qubits, S and its complement are closed."""
    t, c, nns = (int(x) for x in words[off:off + 3])
    assert t + nns == n
    k = off + 4
    S = [int(x) for x in words[k:k + t]]
    nonS = [int(x) for x in words[k + t:k + t + nns]]
    pi = [int(x) for x in words[k + t + nns:k + 2 * t + nns]]
    pin = [int(x) for x in words[k + 2 * t + nns:k + 2 * t + 2 * nns]]
    assert S == sorted(S) and sorted(S + nonS) == list(range(n))
    assert S[:c] == list(range(c))
    sigma = [0] * n
    for j, q in enumerate(S):
        sigma[q] = S[pi[j]]
    for i, q in enumerate(nonS):
        sigma[q] = nonS[pin[i]]
    assert sorted(sigma) == list(range(n)) and all(sigma[sigma[q]] == q for q in range(n))
    return sigma


def run_qperm(psi, n, words, off):
    """out[y] = in[sigma(y)], sigma(y) moving bit q of y to bit sigma(q)."""
    sigma = qperm_sigma(words, off, n)
    idx = np.arange(1 << n, dtype=np.int64)
    src = np.zeros_like(idx)
    for q in range(n):
        src |= ((idx >> q) & 1) << sigma[q]
    psi[:] = psi[src]


def emulate(n, dtype, ops, psi0, tile=0, matrix_of=None):
    """Run the fused plan of ``ops`` on psi0 (complex128, copied)."""
    words, steps = program(n, dtype, ops, tile)
    ops = list(ops)
    if any(is_qperm(words, int(st)) for st in steps):
        ops = relabel_swaps(ops, n)
    psi = np.array(psi0, dtype=np.complex128)
    cfg = CFG[dtype]
    for st in steps:
        if st < 0:
            o = ops[int(-st - 1)]
            _apply_dense(psi, n, list(o.qubits), np.asarray(o.mat, dtype=np.complex128))
        elif is_qperm(words, int(st)):
            run_qperm(psi, n, words, int(st))
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


STEP_NAMES = [(LT_TAB, "TAB"), (LT_CZR, "CZR"), (LT_CZF, "CZF"), (LT_SIGN, "SIGN"), (LT_PHASEL, "PHASEL"),
              (LT_RAWD, "RAWD"), (LT_PERM2, "PERM2"), (LT_U2, "U2"), (LT_U1, "U1")]


def op_counts(words, steps, dtype):
    """Number of layers, blocks and steps of each kind in a plan's tile
    programs ('ROT' counts rotations, 'ROT3' those made of three shears,
    'maps' the rounds whose store applies CNOTs)."""
    RB = CFG[dtype]["RB"]
    out = {}

    def add(key, v=1):
        out[key] = out.get(key, 0) + v
    for st in steps:
        if st < 0:
            add("separate")
            continue
        off = int(st)
        if is_qperm(words, off):
            add("qperm")
            continue
        t, c, nns = (int(x) for x in words[off:off + 3])
        LR = CFG[dtype]["LR"]
        blocks = _round_blocks(words, off, t, nns)
        add("blocks", len(blocks))
        for rb in blocks:
            if int(words[rb + MAP_HDR]):
                add("maps")
            k = rb + ROUND_HEADER
            for li in range(int(words[rb])):
                flags = int(words[k])
                k += LR + (TABLE_WORDS if flags & LT_TAB else 0)
                add("layers")
                for bitv, name in STEP_NAMES:
                    if flags & bitv:
                        add(name)
                add("ROT", bin((flags >> 8) & ((1 << RB) - 1)).count("1"))
                add("ROT3", bin((flags >> 16) & ((1 << RB) - 1)).count("1"))
    return out
