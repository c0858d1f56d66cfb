"""The largest registers of the accepted range that leave room on one GPU:
34 qubits in complex64 and 33 in complex128 (128 GiB each). Per-gate
launches there need more than 2^32 work-items and take their second grid
dimension. Checked on sampled amplitudes against closed forms: GHZ built by
per-gate kernels, and the QFT of a basis state by the fused plan (tile
passes and the bit-reversal pass), plus the norm."""
import numpy as np
import pytest

import qcircuits as qc

pytestmark = pytest.mark.gpu

CASES = [("c64", 34), ("c128", 33)]


def fresh_state(n, dtype):
    import torch
    from paper_1807_07914_amd import State
    torch.cuda.empty_cache()
    need = (1 << n) * (8 if dtype == "c64" else 16)
    free, _ = torch.cuda.mem_get_info()
    if free < need * 1.05:
        pytest.skip("the device has %.0f GiB free; the state needs %.0f GiB" % (free / 2 ** 30, need / 2 ** 30))
    return State(n, dtype)


def samples(n, seed, count=2048):
    import torch
    rng = np.random.default_rng(seed)
    idx = np.concatenate([[0, (1 << n) - 1], np.arange(1, count), rng.integers(0, 1 << n, count)])
    return torch.as_tensor(idx, dtype=torch.int64, device="cuda"), idx


@pytest.mark.parametrize("dtype,n", CASES)
def test_max_register_ghz_by_pergate_kernels(dtype, n):
    import torch
    s = fresh_state(n, dtype)
    s.set_basis(0)
    s.apply_circuit(qc.ghz(n), mode="pergate")
    ti, idx = samples(n, 11)
    got = s.tensor[ti].cpu().numpy().astype(np.complex128)
    norm = s.norm()
    s.close()
    del s
    torch.cuda.empty_cache()
    want = np.zeros(idx.size, dtype=np.complex128)
    want[(idx == 0) | (idx == (1 << n) - 1)] = 2 ** -0.5
    tol = 1e-6 if dtype == "c64" else 1e-14
    assert np.abs(got - want).max() <= tol
    assert abs(norm - 1.0) <= 10 * tol


@pytest.mark.parametrize("dtype,n", CASES)
def test_max_register_qft_by_fused_passes(dtype, n):
    import torch
    s = fresh_state(n, dtype)
    x = qc.qft_input(n, 1700 + n)
    s.set_basis(x)
    s.apply_circuit(qc.qft(n))
    ti, idx = samples(n, 12)
    got = s.tensor[ti].cpu().numpy().astype(np.complex128)
    norm = s.norm()
    s.close()
    del s
    torch.cuda.empty_cache()
    N = 1 << n
    ref = np.exp(2j * np.pi * ((x * idx.astype(object)) % N).astype(np.float64) / N) / 2 ** (n / 2)
    d = float(np.abs(got - ref).max()) * 2 ** (n / 2)
    assert d <= (1e-4 if dtype == "c64" else 1e-9), d
    assert abs(norm - 1.0) <= (1e-5 if dtype == "c64" else 1e-12)
