"""Fused states at the headline sizes against the complex128 CPU oracle,
element by element.

At 24 qubits the fused planner's tiles (2^13 amplitudes in complex64, 2^12
in complex128) outnumber the resident workgroups of the persistent tile
kernel, so its prefetch of the next tile and its rotated load / store loop
run; every amplitude is compared.  At 28 qubits (the headline circuit:
depth-40 brickwork of Haar SU(2) and CZ, 1660 gates) the oracle computes the
whole 2^28 complex128 state on the host and the complex64 and complex128
fused states and the complex64 per-gate state are compared with it in full.

Each comparison reports max|d|, the normalised max|d| * 2^(n/2) (amplitudes
are ~2^(-n/2) in magnitude), the relative 2-norm ||d|| / ||psi|| and the
FP64 norm drift |sum |psi|^2 - 1| of the GPU state (paper section I: the
brute-force result is exact; the complex64 path's error is stated per
result).  The bars: max|d| <= 1e-5 (complex64) and 1e-12 (complex128), and
on the normalised error 1e-4 and 1e-10.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
BARS = {"c64": (1e-5, 1e-4), "c128": (1e-12, 1e-10)}


def State(*a, **k):
    from paper_1807_07914_amd import State as S
    return S(*a, **k)


def say(*a):
    print("[%s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def errors(gpu, ref, n, chunk=1 << 24):
    """max|d|, normalised max|d|, ||d|| / ||ref||, norm drift; chunked so that
    no full-size complex128 difference array is formed."""
    mx, d2, r2, g2 = 0.0, 0.0, 0.0, 0.0
    for a in range(0, ref.size, chunk):
        g = gpu[a:a + chunk].astype(np.complex128)
        r = ref[a:a + chunk]
        d = g - r
        ad = np.abs(d)
        mx = max(mx, float(ad.max()))
        d2 += float(np.sum(ad * ad))
        r2 += float(np.sum(r.real * r.real + r.imag * r.imag))
        g2 += float(np.sum(g.real * g.real + g.imag * g.imag))
    return {"max_abs": mx, "max_abs_x2^(n/2)": mx * 2.0 ** (n / 2), "rel_l2": (d2 / r2) ** 0.5,
            "norm_drift": abs(g2 - 1.0)}


def record(name, rec):
    """Measured errors go to gpurun_out/ when that folder exists (GPU runs)."""
    out = os.path.join(os.path.dirname(HERE), "gpurun_out")
    say(name, json.dumps(rec))
    if os.path.isdir(out):
        with open(os.path.join(out, "fullsize_errors.jsonl"), "a") as f:
            f.write(json.dumps({"case": name, **rec}) + "\n")


def check(name, dtype, err):
    record(name, err)
    amax, nmax = BARS[dtype]
    assert err["max_abs"] <= amax, (name, err)
    assert err["max_abs_x2^(n/2)"] <= nmax, (name, err)


def run_gpu(n, dtype, ops, mode="fused", x0=0):
    s = State(n, dtype)
    s.set_basis(x0)
    s.apply_circuit(ops, mode=mode)
    psi = s.to_numpy()
    s.close()
    return psi


def fam24():
    n = 24
    rng = np.random.default_rng(2424)
    return n, {
        "brickwork_d40": qc.random_brickwork(n, 40, 2401),
        # explicit 4x4 blocks, SWAPs, CNOTs and every named gate (full-body
        # passes, which complex64 runs on the persistent pipelined kernel
        # too), and 8x8 blocks (their own kernel between fused passes)
        "random_ops": qc.random_ops(n, 400, 2402, dense_k=(1, 2, 3)),
        "qft": qc.qft(n),
        "hea": qc.hea_circuit(n, rng.uniform(0, 2 * np.pi, (6, n, 2)), layers=6),
        # CNOT ladders and CNOTs between any two qubits (controls outside
        # the tile, targets at register and free bits): the rounds' store maps
        "rounds": qc.paper_rounds(n, 6, 2404),
        "cnot_mesh": cnot_mesh(n, 6, 2405),
    }


def cnot_mesh(n, depth, seed):
    """Per layer RY and RZ on every qubit, then CNOTs on a random pairing of
    all qubits (either direction, any distance)."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(depth):
        for q in range(n):
            ops.append(qc.op("RY", q, params=(float(rng.uniform(0, 2 * np.pi)),)))
            ops.append(qc.op("RZ", q, params=(float(rng.uniform(0, 2 * np.pi)),)))
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            ops.append(qc.op("CNOT", int(perm[i]), int(perm[i + 1])))
    return ops


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fused_24_qubits_every_amplitude(dtype):
    n, fams = fam24()
    for name, ops in fams.items():
        x0 = qc.qft_input(n, 2403) if name == "qft" else 0
        say("24q", name, dtype, "gates", len(ops))
        got = run_gpu(n, dtype, ops, x0=x0)
        ref = O.run(ops, n, x0=x0)
        check("n24_%s_%s_fused" % (name, dtype), dtype, errors(got, ref, n))


@pytest.mark.timeout(900)
def test_headline_28_qubits_against_the_oracle():
    # the whole 2^28 complex128 state by the oracle (about two minutes on 16
    # host threads), then the fused complex64 / complex128 and per-gate
    # complex64 GPU states against it
    n = 28
    ops = qc.random_brickwork(n, 40, qc.SEEDS["c2"])
    say("28q oracle run: %d gates on %d threads" % (len(ops), O.num_threads()))
    t0 = time.time()
    ref = O.zero_state(n)
    for a in range(0, len(ops), 200):  # progress lines while the oracle runs
        O.run(ops[a:a + 200], n, psi=ref)
        say("28q oracle: %d gates, %.1f s" % (min(a + 200, len(ops)), time.time() - t0))
    for dtype, mode in (("c64", "fused"), ("c128", "fused"), ("c64", "pergate")):
        say("28q", dtype, mode)
        got = run_gpu(n, dtype, ops, mode=mode)
        check("n28_headline_%s_%s" % (dtype, mode), dtype, errors(got, ref, n))
        del got
