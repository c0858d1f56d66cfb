"""The race-check mode of fused plans (plan option race_check): every tile
and permutation pass runs out of place into a poisoned buffer first and must
write every amplitude and match the in-place pass bit for bit."""
import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def circuits(n):
    rng = np.random.default_rng(n)
    return {
        "brickwork": qc.random_brickwork(n, 10, 2100 + n),
        "qft": qc.qft(n),
        "random": qc.random_ops(n, 120, 2200 + n, dense_k=(1, 2)),
        "hea": qc.hea_circuit(n, rng.uniform(0, 2 * np.pi, (4, n, 2)), layers=4),
        "swaps": [qc.op("SWAP", i, n - 1 - i) for i in range(n // 2)] + qc.random_brickwork(n, 3, 2300 + n),
    }


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,tile", [(9, 6), (16, 0), (22, 0)])
def test_race_check_passes_and_keeps_the_result(dtype, n, tile):
    from paper_1807_07914_amd import State
    psi0 = qc.random_state(n, 2400 + n).astype(np.complex64 if dtype == "c64" else np.complex128)
    for name, ops in circuits(n).items():
        a = State(n, dtype)
        a.from_numpy(psi0)
        a.apply_circuit(ops, tile_qubits=tile, race_check=True)
        got = a.to_numpy()
        a.close()
        b = State(n, dtype)
        b.from_numpy(psi0)
        b.apply_circuit(ops, tile_qubits=tile)
        ref = b.to_numpy()
        b.close()
        assert np.array_equal(got, ref), name
        if n <= 16:
            assert np.abs(got - O.run(ops, n, psi=psi0.astype(np.complex128))).max() <= TOL[dtype], name


def test_race_check_reports_poison_left_in_the_output():
    # forced from the host: a state whose every word is the poison pattern,
    # moved bit for bit by a permutation pass, looks unwritten to the check
    from paper_1807_07914_amd import QsvError, State
    n = 16
    ops = [qc.op("SWAP", i, n - 1 - i) for i in range(n // 2)]
    words = np.full(2 << n, 0x7FBADBAD, dtype=np.uint32)
    s = State(n, "c64")
    s.from_numpy(words.view(np.complex64))
    with pytest.raises(QsvError, match="race check"):
        s.apply_circuit(ops, race_check=True)
    s.close()


def test_race_check_argument_rules():
    import torch
    from paper_1807_07914_amd import QsvError, State
    ops = qc.random_brickwork(10, 3, 2500)
    s = State(10, "c64", stream=torch.cuda.Stream())
    with pytest.raises(QsvError):
        s.apply_circuit(ops, mode="pergate", race_check=True)
    with pytest.raises(QsvError):
        s.apply_circuit(ops, graph=True, race_check=True)
    s.close()
