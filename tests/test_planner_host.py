"""CPU checks of the fused planner and its program encoding.

The tile-program emulator (tests/tile_emulator.py) decodes the exact words
the library would upload for the tile kernel; its output must match the CPU
oracle for every circuit family, both precisions and several tile sizes.
Pass counts are checked to be below the gate counts (fusion happens) and
stable for a fixed structure.
"""
import numpy as np
import pytest

import qcircuits as qc
from oracle import oracle as O
from paper_1807_07914_amd import qsv

import tile_emulator as E

TOL = {"c64": 2e-6, "c128": 1e-13}


def families(n, seed):
    rng = np.random.default_rng(seed)
    return {
        "random": qc.random_ops(n, 50, seed, dense_k=(1, 2, 3)),
        "brickwork": qc.random_brickwork(n, 5, seed),
        "rounds": qc.paper_rounds(n, 3, seed),
        "qft": qc.qft(n),
        "hea": qc.hea_circuit(n, rng.uniform(0, 2 * np.pi, (3, n, 2)), layers=3),
        "rotring": qc.rot_ring_ansatz(n, rng.uniform(0, 2 * np.pi, 2 * 3 * n), 2),
        "ghz": qc.ghz(n),
    }


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,tile", [(5, 0), (7, 6), (9, 7)])
def test_emulated_fused_plans_match_oracle(dtype, n, tile):
    psi0 = qc.random_state(n, 3 + n)
    for name, ops in families(n, 11 + n).items():
        ref = O.run(ops, n, psi=psi0.copy())
        got = E.emulate(n, dtype, ops, psi0, tile)
        assert np.abs(got - ref).max() <= TOL[dtype], name


def test_pass_counts_fuse_gates():
    ops = qc.random_brickwork(28, 40, qc.SEEDS["c2"])
    a = qsv.plan_info(28, "c64", ops)
    b = qsv.plan_info(28, "c64", ops)
    assert a == b and a["separate_ops"] == 0
    assert a["passes"] <= 40
    assert qsv.plan_info(30, "c64", qc.qft(30))["passes"] <= 8
    # a circuit that fits one tile is a single pass
    assert qsv.plan_info(10, "c128", qc.random_brickwork(10, 20, 1))["passes"] == 1


def test_plan_info_rejects_bad_input():
    with pytest.raises(qsv.QsvError):
        qsv.plan_info(4, "c64", [qc.op("H", 4)])
    with pytest.raises(qsv.QsvError):
        qsv.plan_info(10, "c64", qc.ghz(10), tile_qubits=20)
