#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Step = one pass of the whole hot path over the headline workload: a 28-qubit
random circuit of depth 40 (Haar SU(2) on every qubit, then CZ on alternating
nearest-neighbour pairs; 1660 gates; seed 1002) in complex64, applied in
place with the fused tile-pass planner, followed by the FP64 reductions
(sum_i Z_i Z_{i+1} + 0.7 sum_i X_i, the norm) and 1024 measurement samples.
State initialisation is inside the step.  The value is gates per second.

Prints ONE JSON line (see the field list in ``result``).  Beside the headline
it measures, on the same GPU: the headline circuit's per-gate and complex128
forms and the complex64 state's deviation from the complex128 one
(``c2_forms``); the 30-qubit QFT, the 4096-circuit batched launch
(circuits/s) and the 24-qubit adjoint gradient (gradients/s), each with its
plain per-gate form and its own roofline fraction (``legs``).  With --extras
it adds the paper's random-round grid, the H2 sweep and the MPS grid.  The
CPU oracle is timed on a bounded sample of the headline circuit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gates/s + achieved HBM GB/s at 28-30 qubits; batched circuits/s; adjoint grads/s"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
TILE_SOURCES = ["paper_1807_07914_amd/csrc/tile.hip", "paper_1807_07914_amd/csrc/tile.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tile_pass_c2_traffic.json")


def kernel_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def op_flops(o):
    """Algorithmic real flops per amplitude of one gate record."""
    if o.name in ("CZ", "Z", "I"):
        return 0.0
    if o.name in ("CNOT", "SWAP", "X"):
        return 0.0
    if o.name in ("RZ", "S", "SDG", "T", "TDG"):
        return 6.0          # one complex multiply per amplitude
    if o.name == "CPHASE":
        return 6.0 / 4.0    # a quarter of the amplitudes
    if o.name == "U":
        d = 1 << o.k
        return 8.0 * d - 2.0  # row of a dense complex mat-vec
    return 14.0             # general 2x2: two complex multiplies and one add


COUNTER_FILE = os.path.join(ROOT, "profiles", "tile_pass_c2_counters.json")


def load_counters(n):
    """Executed-instruction counters of the tile pass (rocprofv3 --pmc),
    when they were taken from the current tile sources at this size."""
    if not os.path.exists(COUNTER_FILE):
        return None
    with open(COUNTER_FILE) as f:
        c = json.load(f)
    if c.get("kernel_hash") != kernel_hash(TILE_SOURCES) or c.get("n") != n:
        return None
    return c.get("summary")


def circuit_flops(ops, n):
    """Algorithmic real flops of applying a gate list to 2^n amplitudes."""
    return sum(op_flops(o) for o in ops) * float(1 << n)


def adjoint_flops(ops, n, n_terms):
    """Algorithmic real flops of one gradient vector by the adjoint method:
    the forward pass, lambda = H psi (one complex multiply-add per amplitude
    and term), the inverse of every gate on psi and on lambda, and one
    Im<lambda|P|psi> (a complex multiply-add per amplitude) per rotation."""
    nrot = sum(o.name in ("RX", "RY", "RZ") for o in ops)
    fwd = circuit_flops(ops, n)
    return 3.0 * fwd + (8.0 * n_terms + 8.0 * nrot) * float(1 << n)


class Timer:
    """HIP events on the state's stream around a region."""

    def __init__(self, stream):
        import torch
        self.stream = stream
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.e0.record(self.stream)
        return self

    def __exit__(self, *a):
        self.e1.record(self.stream)

    def ms(self):
        self.e1.synchronize()
        return self.e0.elapsed_time(self.e1)


def cpu_baseline(ops, n, budget_s=15.0, min_gates=3):
    """The CPU oracle (complex128, as it stands) on the first gates of the
    same circuit at the same size, until the time budget is used."""
    from oracle import oracle as O
    psi = O.zero_state(n)
    t0 = time.perf_counter()
    done = 0
    for o in ops:
        O.apply(psi, n, o)
        done += 1
        if done >= min_gates and time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "gates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": "first %d of %d gates of the %d-qubit depth-40 random circuit, complex128, "
                      "%.1f s" % (done, len(ops), n, dt)}


def bench_batched(np, torch, qc, qsv, count=4096, reps=5, sample=128):
    """4096 hardware-efficient-ansatz circuits (widths 8..20, 10 layers of
    RY, RZ + CNOT ladder, seed 1004), <sum Z_i Z_{i+1}> each, complex64, one
    graph-replayed persistent launch per run.  The per-circuit forms (plain
    per-gate kernels, and fused tile passes) are timed on a sample of
    circuits drawn uniformly from the batch and scaled to circuits/s."""
    b = qc.hea_batch(count, qc.SEEDS["c4"])
    circs = [b.circuit(i) for i in range(count)]
    hams = [b.hamiltonian(i) for i in range(count)]
    widths = [int(w) for w in b.widths]
    t0 = time.perf_counter()
    bt = qsv.Batch(circs, widths, hams, dtype="c64")
    t_create = time.perf_counter() - t0
    bt.run()
    t0 = time.perf_counter()
    for _ in range(reps):
        e = bt.run()
    t_run = (time.perf_counter() - t0) / reps
    info = bt.info()
    bt.close()
    rng = np.random.default_rng(0)
    pick = rng.choice(count, sample, replace=False)
    forms = {}
    for mode in ("pergate", "fused"):
        st = {}
        for i in pick:
            w = widths[i]
            if w not in st:
                st[w] = qsv.State(w, "c64")
        for s in st.values():          # warm-up (code objects, plans)
            s.set_basis(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in pick:
            s = st[widths[i]]
            s.set_basis(0)
            s.apply_circuit(circs[i], mode=mode)
            s.expval(hams[i])
        dt = time.perf_counter() - t0
        for s in st.values():
            s.close()
        forms[mode] = sample / dt
    flops = sum(circuit_flops(c, w) for c, w in zip(circs, widths))
    return {"circuits_per_s": count / t_run, "ms_per_batch": t_run * 1e3,
            "roofline": {"bound": "alu", "achieved": flops / t_run / 1e12,
                         "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / t_run / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                         "algorithmic_flops": flops},
            "create_and_autotune_s": t_create, "tile_qubits": info["tile_qubits"],
            "tile_passes": info["passes"], "scratch_gb": info["scratch_bytes"] / 1e9,
            "energy_checksum": float(np.sum(e)),
            "pergate_circuits_per_s": forms["pergate"], "fused_circuits_per_s": forms["fused"],
            "speedup_vs_pergate": count / t_run / forms["pergate"]}


def bench_rounds(np, torch, qc, qsv, circuits=10):
    """The paper's random-round family on its grid: n = 5..30 step 5, rounds
    2..10 step 2, ten seeded circuits each (complex64, fused passes, plan
    built per circuit and included in the time).  For n <= 20 the first
    circuit's state is checked for Schmidt rank <= 2^rounds across the middle
    cut (host SVD of the GPU state)."""
    out = {}
    for n in range(5, 31, 5):
        s = qsv.State(n, "c64")
        s.apply_circuit(qsv.OpList(qc.paper_rounds(n, 2, 1999)), mode="fused")  # warm-up, untimed
        torch.cuda.synchronize()
        row = {}
        for rounds in range(2, 11, 2):
            gates, t_tot, chi = 0, 0.0, None
            for c in range(circuits):
                lst = qc.paper_rounds(n, rounds, 2000 + 100 * n + 10 * rounds + c)
                ops = qsv.OpList(lst)
                s.set_basis(0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.apply_circuit(ops, mode="fused")
                torch.cuda.synchronize()
                t_tot += time.perf_counter() - t0
                gates += len(lst)
                if c == 0 and n <= 20:
                    psi = s.to_numpy().reshape(1 << (n - n // 2), 1 << (n // 2))
                    sv = np.linalg.svd(psi, compute_uv=False)
                    chi = int(np.sum(sv > 1e-4 * sv[0]))
            row[rounds] = {"gates_per_s": gates / t_tot, "ms_per_circuit": t_tot / circuits * 1e3}
            if chi is not None:
                row[rounds]["schmidt_rank"] = chi
                row[rounds]["schmidt_bound_ok"] = chi <= min(2 ** rounds, 1 << (n // 2))
        out[n] = row
        s.close()
        torch.cuda.empty_cache()
    return out


def bench_h2_sweep(np, torch, qc, qsv, reps=20):
    """The paper's VQE sweep: 100 values of t0 times five terms = 500
    two-qubit circuits (basis changes for X0X1 and Y0Y1) in one batched
    launch, complex64; deviation from the closed forms."""
    circs, widths, hams, keys = qc.h2_term_batch(qc.h2_sweep())
    t0 = time.perf_counter()
    bt = qsv.Batch(circs, widths, hams, dtype="c64")
    t_create = time.perf_counter() - t0
    e = bt.run()
    t0 = time.perf_counter()
    for _ in range(reps):
        e = bt.run()
    t_run = (time.perf_counter() - t0) / reps
    info = bt.info()
    bt.close()
    cf = np.array([qc.h2_closed_forms(t)[k] for t, k in keys])
    return {"circuits": len(circs), "points": 100, "ms_per_sweep": t_run * 1e3,
            "points_per_s": 100 / t_run, "circuits_per_s": len(circs) / t_run,
            "create_and_autotune_s": t_create, "tile_qubits": info["tile_qubits"],
            "max_abs_dev_closed_form": float(np.abs(e - cf).max())}


def bench_mps(np, torch, qc, qsv, circuits=10, chi_max=32, cutoff=1e-4):
    """The paper's MPS experiment (section V.A) on the GPU MPS path: the
    random-round family for n = 5..85 step 5 and rounds 2..10 step 2, ten
    seeded circuits each, bond cap chi_max and the paper's cutoff 1e-4.
    Reports time per circuit, the largest bond dimension and the MPS memory
    (mean and standard deviation over the circuits, the paper's measure), and
    for n <= 20 the fidelity of the first circuit against the complex128
    state-vector path."""
    out = {}
    m = qsv.MPS(10, chi_max, cutoff)    # warm-up (code objects, buffers)
    m.apply_circuit(qc.paper_rounds(10, 2, 1))
    m.bonds()
    m.close()
    for n in range(5, 86, 5):
        row = {}
        for rounds in range(2, 11, 2):
            ts, chis, mems, upd = [], [], [], 0
            fid = None
            for c in range(circuits):
                lst = qc.paper_rounds(n, rounds, 5000 + 100 * n + 10 * rounds + c)
                ops = qsv.OpList(lst)
                m = qsv.MPS(n, chi_max, cutoff)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                m.apply_circuit(ops)
                dims, _ = m.bonds()          # synchronises
                ts.append(time.perf_counter() - t0)
                chis.append(max(dims))
                mems.append(m.memory_bytes())
                upd += m.info()["bond_updates"]
                if c == 0 and n <= 20:
                    amp = m.amplitudes(np.arange(1 << n, dtype=np.uint64))
                    s = qsv.State(n, "c128")
                    s.apply_circuit(ops)
                    psi = s.to_numpy()
                    s.close()
                    fid = float(abs(np.vdot(psi, amp)) ** 2 / np.vdot(amp, amp).real)
                m.close()
            t = float(np.sum(ts))
            row[rounds] = {"ms_per_circuit": t / circuits * 1e3, "gates_per_s": len(lst) * circuits / t,
                           "us_per_bond_update": t / upd * 1e6,
                           "max_chi_mean": float(np.mean(chis)), "max_chi_std": float(np.std(chis)),
                           "memory_bytes_mean": float(np.mean(mems)), "memory_bytes_std": float(np.std(mems))}
            if fid is not None:
                row[rounds]["fidelity_vs_sv"] = fid
        out[n] = row
        print("mps grid: n=%d done (%.1f ms per circuit at %d rounds)" % (n, row[rounds]["ms_per_circuit"], rounds),
              file=sys.stderr, flush=True)
    return out


def bench_adjoint(np, torch, qc, qsv, reps=3):
    """24 qubits, 6 layers of RX, RY, RZ + CZ ring (432 parameters, seed
    1005), H = sum Z_i Z_{i+1} + 0.7 sum X_i, complex64 with FP64 reductions:
    one forward pass plus one adjoint sweep per gradient vector."""
    n, layers = 24, 6
    params, ham = qc.gradient_workload(n, layers, qc.SEEDS["c5"])
    ops = qsv.OpList(qc.rot_ring_ansatz(n, params, layers))
    s = qsv.State(n, "c64")
    s.set_basis(0)
    s.adjoint(ops, ham)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.set_basis(0)
        e, g = s.adjoint(ops, ham)
    t_adj = (time.perf_counter() - t0) / reps
    fwd = {}
    for mode in ("fused", "pergate"):
        s.set_basis(0)
        s.apply_circuit(ops, mode=mode)
        s.expval(ham)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_basis(0)
        s.apply_circuit(ops, mode=mode)
        s.expval(ham)
        fwd[mode] = time.perf_counter() - t0
    s.close()
    nparam = params.size
    lst = qc.rot_ring_ansatz(n, params, layers)
    flops = adjoint_flops(lst, n, len(ham))
    return {"grads_per_s": 1.0 / t_adj, "params_per_s": nparam / t_adj, "ms_per_gradient": t_adj * 1e3,
            "roofline": {"bound": "alu", "achieved": flops / t_adj / 1e12,
                         "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / t_adj / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                         "algorithmic_flops": flops},
            "energy": e, "forward_fused_ms": fwd["fused"] * 1e3, "forward_pergate_ms": fwd["pergate"] * 1e3,
            "gradient_cost_in_fused_forwards": t_adj / fwd["fused"],
            "parameter_shift_equiv_ms": 2 * nparam * fwd["fused"] * 1e3,
            "speedup_vs_parameter_shift": 2 * nparam * fwd["fused"] / t_adj,
            "parameter_shift_pergate_equiv_ms": 2 * nparam * fwd["pergate"] * 1e3,
            "speedup_vs_pergate_parameter_shift": 2 * nparam * fwd["pergate"] / t_adj}


def bench_qft30(np, torch, qc, qsv, reps=3):
    """The 30-qubit QFT (H + controlled phases + swaps, 480 gates) on a seeded
    basis state, complex64, fused tile passes; the per-gate form beside it;
    the error against the closed form 2^-15 exp(2 pi i x y / 2^30) on 4096
    sampled amplitudes."""
    nq = 30
    qops = qc.qft(nq)
    qol = qsv.OpList(qops)
    x = qc.qft_input(nq, qc.SEEDS["c3"])
    s3 = qsv.State(nq, "c64")
    s3.set_basis(x)
    s3.apply_circuit(qol)      # warm-up (plan cache, code objects)
    ts = []
    for _ in range(reps):
        s3.set_basis(x)
        torch.cuda.synchronize()
        with Timer(s3.stream) as tm:
            s3.apply_circuit(qol)
        ts.append(tm.ms() / 1e3)
    t = float(np.median(ts))
    rng = np.random.default_rng(13)
    y = np.concatenate([np.arange(2048), rng.integers(0, 1 << nq, 2048)]).astype(np.int64)
    psi = s3.tensor[torch.as_tensor(y, device="cuda")].cpu().numpy().astype(np.complex128)
    ref = np.exp(2j * np.pi * ((x * y) % (1 << nq)) / (1 << nq)) / 2 ** (nq / 2)
    s3.set_basis(x)
    torch.cuda.synchronize()
    with Timer(s3.stream) as tm:
        s3.apply_circuit(qol, mode="pergate")
    t_pg = tm.ms() / 1e3
    passes = qsv.plan_info(nq, "c64", qol)["passes"]
    s3.close()
    torch.cuda.empty_cache()
    nbytes = (1 << nq) * 8
    return {"ms": t * 1e3, "gates_per_s": len(qops) / t, "passes": passes,
            "pergate_ms": t_pg * 1e3, "speedup_vs_pergate": t_pg / t,
            "roofline": {"bound": "hbm", "achieved": passes * 2 * nbytes / t / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": passes * 2 * nbytes / t / 1e9 / HBM_PEAK_GBS},
            "max_abs_err_closed_form_4096": float(np.abs(psi - ref).max())}


def bench_dense_blocks(np, torch, qc, qsv, n=28, reps=5):
    """Explicit dense k-qubit blocks (qsv_apply_fused, k = 4..6, Haar U(2^k))
    on a 28-qubit state: k >= 4 runs on the matrix cores (real embedding of
    the complex block).  Blocks on the low k qubits and on k high qubits;
    median time per block, with its algorithmic flops (8 * 2^k per
    amplitude) against the dense MFMA peak of the dtype and its bytes
    (one read and one write of the state) against HBM."""
    rng = np.random.default_rng(77)
    out = {}
    for dtype, peak in (("c64", 157.3), ("c128", 78.6)):
        s = qsv.State(n, dtype)
        s.set_basis(0)
        nbytes = (1 << n) * (8 if dtype == "c64" else 16)
        for k in (4, 5, 6):
            U = qc.haar_unitary(k, rng)
            for where, qs in (("low", list(range(k))), ("high", list(range(n - k, n)))):
                s.apply_fused(qs, U)  # warm-up (staged matrix, code object)
                ts = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    with Timer(s.stream) as tm:
                        s.apply_fused(qs, U)
                    ts.append(tm.ms() / 1e3)
                t = float(np.median(ts))
                fl = 8.0 * (1 << k) * (1 << n)
                out["%s_k%d_%s" % (dtype, k, where)] = {
                    "ms": t * 1e3, "tflops": fl / t / 1e12, "mfma_frac": fl / t / 1e12 / peak,
                    "hbm_gbs": 2 * nbytes / t / 1e9, "hbm_frac": 2 * nbytes / t / 1e9 / HBM_PEAK_GBS}
        s.close()
        torch.cuda.empty_cache()
    return out


def bench_c2_forms(np, torch, qc, qsv, ol, ngates, n, psi64):
    """The headline circuit in its other forms: complex128 fused and
    per-gate, complex64 per-gate; the complex64 fused state's deviation from
    the complex128 fused state (the complex128 path is held to the oracle
    within 1e-12 by the parity tests)."""
    out = {}
    s2 = qsv.State(n, "c128")
    s2.apply_circuit(ol, mode="fused")  # warm-up (plan cache, code objects)
    for mode in ("fused", "pergate"):
        s2.set_basis(0)
        torch.cuda.synchronize()
        with Timer(s2.stream) as tm:
            s2.apply_circuit(ol, mode=mode)
        t = tm.ms() / 1e3
        out["c128_" + mode] = {"gates_per_s": ngates / t, "ms": t * 1e3,
                               "norm_drift": abs(s2.norm() - 1.0)}
        if mode == "fused":
            ref = s2.tensor
            d = (psi64.to(torch.complex128) - ref).abs()
            nd = float(torch.linalg.vector_norm(d).item())
            nr = float(torch.linalg.vector_norm(ref).item())
            mx = float(d.max().item())
            del d
            out["c64_vs_c128"] = {"max_abs": mx, "max_abs_x2^(n/2)": mx * 2.0 ** (n / 2),
                                  "rel_l2": nd / nr}
    out["c128_fused"]["passes"] = qsv.plan_info(n, "c128", ol)["passes"]
    s2.close()
    torch.cuda.empty_cache()
    return out


def run_step(s, ol, ham, uniforms, mode="fused"):
    s.set_basis(0)
    s.apply_circuit(ol, mode=mode)
    e = s.expval(ham)
    nrm = s.norm()
    smp = s.sample(uniforms)
    return e, nrm, smp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--extras", action="store_true", help="also time the other forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline step only (no other forms or legs; for profiling)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-ref", action="store_true",
                    help="run one plain 2 GiB device copy first (reference for HBM counters)")
    ap.add_argument("--mps-circuits", type=int, default=10, help="circuits per cell of the MPS grid")
    ap.add_argument("--mps-chi", type=int, default=32, help="bond cap of the MPS grid (at most 64)")
    ap.add_argument("--only", choices=["c3_qft30", "dense_blocks", "c4_batched", "c5_adjoint", "f1_paper_rounds", "f2_h2_sweep",
                                       "f3_mps"],
                    help="run one of the extra workloads alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import qcircuits as qc
    from paper_1807_07914_amd import OpList, State
    from paper_1807_07914_amd import qsv

    if args.only:
        fn = {"c3_qft30": bench_qft30, "dense_blocks": bench_dense_blocks, "c4_batched": bench_batched, "c5_adjoint": bench_adjoint,
              "f1_paper_rounds": bench_rounds, "f2_h2_sweep": bench_h2_sweep,
              "f3_mps": bench_mps}[args.only]
        kw = {"circuits": args.mps_circuits, "chi_max": args.mps_chi} if args.only == "f3_mps" else {}
        print(json.dumps({args.only: fn(np, torch, qc, qsv, **kw)}))
        return

    n = args.n
    ops = qc.random_brickwork(n, 40, qc.SEEDS["c2"])
    ol = OpList(ops)
    ham = qc.zz_chain(n) + [(0.7, (("X", q),)) for q in range(n)]
    uniforms = np.random.default_rng(7).random(1024)
    plan = qsv.plan_info(n, "c64", ol)

    if args.copy_ref:
        a = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    s = State(n, "c64")
    stream = s.stream
    for _ in range(args.warmup):
        run_step(s, ol, ham, uniforms)
    torch.cuda.synchronize()

    # timed region: exactly K steps, bracketed by synchronisations
    circ_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.set_basis(0)
        with Timer(stream) as tm:
            s.apply_circuit(ol, mode="fused")
        s.expval(ham)           # synchronises the stream
        s.norm()
        s.sample(uniforms)
        circ_ms.append(tm.ms())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ms_per_step = elapsed * 1e3 / args.steps
    gates_per_s = len(ops) * args.steps / elapsed
    nbytes = (1 << n) * 8
    circ = float(np.median(circ_ms)) / 1e3
    launch_s = circ / plan["passes"]            # tile kernels run back to back
    flops_total = sum(op_flops(o) for o in ops) * (1 << n)
    flops_per_launch = flops_total / plan["passes"]
    achieved_tflops = flops_per_launch / launch_s / 1e12
    hbm_gbs = 2 * nbytes / launch_s / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash(TILE_SOURCES) and tr.get("n") == n:
            traffic = tr.get("bytes_per_launch")

    # the bound is the unit whose peak the tile pass comes closer to: its
    # algorithmic flops against the FP32 vector peak, or its algorithmic
    # bytes against HBM; the counter summary of the same kernel (when taken
    # from these sources) says what the hardware executed
    alu_frac = achieved_tflops / FP32_VECTOR_PEAK_TFLOPS
    hbm_frac = hbm_gbs / HBM_PEAK_GBS
    if alu_frac >= hbm_frac:
        roofline = {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": alu_frac}
    else:
        roofline = {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm_frac}
    roofline.update({"traffic": traffic, "kernel": "k_tile_pipe<float,13,5>",
                     "launch_ms": launch_s * 1e3, "algorithmic_bytes_per_launch": 2 * nbytes,
                     "algorithmic_flops_per_launch": flops_per_launch,
                     "alu_frac": alu_frac, "hbm_frac": hbm_frac})
    counters = load_counters(n)
    if counters:
        roofline["counters"] = counters

    result = {
        "metric": METRIC,
        "value": gates_per_s,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (f32 pairs), f64 reductions",
        "data": "synthetic",
        "config": {"workload": "random brickwork circuit, %d qubits, depth 40, Haar SU(2) + CZ, "
                               "seed 1002, complex64, fused tile passes, + expval/norm/1024 samples" % n,
                   "qubits": n, "gates": len(ops), "passes": plan["passes"]},
        "hbm_gbs_tile_pass": hbm_gbs,
        "roofline": roofline,
    }

    if args.headline_only:
        s.close()
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = cpu_baseline(ops, n, budget_s=args.cpu_budget)
        print(json.dumps(result))
        return

    # the headline circuit's other forms: per-gate complex64 (the plain
    # form the fused passes are compared with), complex128, and the
    # complex64 state's deviation from the complex128 one
    s.set_basis(0)
    torch.cuda.synchronize()
    with Timer(stream) as tm:
        s.apply_circuit(ol, mode="pergate")
    t = tm.ms() / 1e3
    forms = {"c64_pergate": {"gates_per_s": len(ops) / t, "ms": t * 1e3,
                             "hbm_gbs_equiv_full_pass": len(ops) * 2 * nbytes / t / 1e9},
             "c64_fused": {"gates_per_s": len(ops) / circ, "ms": circ * 1e3, "passes": plan["passes"],
                           "speedup_vs_pergate": t / circ}}
    s.set_basis(0)
    s.apply_circuit(ol, mode="fused")
    forms["c64_fused"]["norm_drift"] = abs(s.norm() - 1.0)
    forms.update(bench_c2_forms(np, torch, qc, qsv, ol, len(ops), n, s.tensor))
    s.close()
    torch.cuda.empty_cache()
    result["c2_forms"] = forms
    # the metric's other legs: the 30-qubit QFT, batched circuits/s and
    # adjoint gradients/s, each beside its plain per-gate form
    legs = {"c3_qft30": bench_qft30(np, torch, qc, qsv),
            "c4_batched": bench_batched(np, torch, qc, qsv),
            "c5_adjoint": bench_adjoint(np, torch, qc, qsv)}
    result["legs"] = legs
    result["batched_circuits_per_s"] = legs["c4_batched"]["circuits_per_s"]
    result["adjoint_grads_per_s"] = legs["c5_adjoint"]["grads_per_s"]
    result["c64_err_vs_c128"] = forms["c64_vs_c128"]

    if args.extras:
        ex = {}
        ex["f1_paper_rounds"] = bench_rounds(np, torch, qc, qsv)
        ex["f2_h2_sweep"] = bench_h2_sweep(np, torch, qc, qsv)
        ex["f3_mps"] = bench_mps(np, torch, qc, qsv, circuits=args.mps_circuits, chi_max=args.mps_chi)
        result["extras"] = ex

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(ops, n, budget_s=args.cpu_budget)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
