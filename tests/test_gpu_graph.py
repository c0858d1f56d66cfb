"""Fused plans launched as the state's hipGraph (plan option graph = 1)
against the oracle, through the C ABI.

The graph is captured once per plan structure and replayed with each call's
program words, so every replay is checked: several circuits of one structure
with different angles, with the program's own eager work (other circuits,
reductions, host copies and synchronisations) between the replays, then a
structure change (a new capture) and a return to the first structure.
"""
import numpy as np
import pytest
import torch

import qcircuits as qc
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def circuit(n, depth, seed):
    return qc.random_brickwork(n, depth, seed)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [14, 24])
def test_graph_replays_match_oracle(dtype, n):
    from paper_1807_07914_amd import State
    st = torch.cuda.Stream()
    s = State(n, dtype, stream=st)
    e = State(n, dtype)   # eager work on the default stream between replays
    ham = qc.zz_chain(n)
    plan = [(6, 1), (6, 2), (6, 3), (9, 4), (6, 5), (9, 6), (6, 7)]   # (depth, seed): 6 -> 9 -> 6 re-captures
    for depth, seed in plan:
        ops = circuit(n, depth, 1200 + 10 * n + seed)
        s.set_basis(0)
        s.apply_circuit(ops, graph=True)
        e.set_basis(0)
        e.apply_circuit(ops)            # the same circuit without a graph
        torch.cuda.synchronize()
        got = s.to_numpy()
        ref = O.run(ops, n) if n <= 14 else None
        if ref is not None:
            assert np.abs(got - ref).max() <= TOL[dtype], (depth, seed)
        # with and without the graph the kernels and their order are the same
        assert np.array_equal(got, e.to_numpy()), (depth, seed)
        v = s.expval(ham)
        assert abs(v - e.expval(ham)) <= 10 * TOL[dtype] * len(ham)
    s.close()
    e.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_graph_replays_with_cnot_store_maps(dtype):
    # HEA circuits (CNOT ladders, applied by the rounds' store maps) with new
    # angles on every call: the same structure replays the captured graph
    from paper_1807_07914_amd import State
    n = 14
    st = torch.cuda.Stream()
    s = State(n, dtype, stream=st)
    e = State(n, dtype)
    rng = np.random.default_rng(1400)
    for rep in range(4):
        ops = qc.hea_circuit(n, rng.uniform(0, 2 * np.pi, (5, n, 2)), layers=5)
        s.set_basis(0)
        s.apply_circuit(ops, graph=True)
        e.set_basis(0)
        e.apply_circuit(ops)
        torch.cuda.synchronize()
        got = s.to_numpy()
        assert np.abs(got - O.run(ops, n)).max() <= TOL[dtype], rep
        assert np.array_equal(got, e.to_numpy()), rep
    s.close()
    e.close()


def test_graph_argument_checks():
    from paper_1807_07914_amd import QsvError, State
    ops = circuit(12, 4, 1300)
    s = State(12, "c64")            # the default stream is the null stream: no capture there
    with pytest.raises(QsvError):
        s.apply_circuit(ops, graph=True)
    s.close()
    s = State(12, "c64", stream=torch.cuda.Stream())
    with pytest.raises(QsvError):
        s.apply_circuit(ops, mode="pergate", graph=True)
    # a plan with a step outside the tile passes (a three-qubit matrix) runs without a graph
    U = qc.haar_unitary(3, np.random.default_rng(3))
    mixed = ops + [qc.op("U", 1, 5, 9, mat=U)] + ops
    s.set_basis(0)
    s.apply_circuit(mixed, graph=True)
    got = s.to_numpy()
    s.close()
    assert np.abs(got - O.run(mixed, 12)).max() <= TOL["c64"]


def test_graph_with_permutation_pass():
    # a plan that ends in a qubit-permutation pass (the 22-qubit QFT's bit
    # reversal) replays through the graph like the tile passes
    from paper_1807_07914_amd import State
    n = 22
    ops = qc.qft(n)
    s = State(n, "c64", stream=torch.cuda.Stream())
    e = State(n, "c64")
    for x0 in (qc.qft_input(n, 5), qc.qft_input(n, 6), 0):
        s.set_basis(x0)
        s.apply_circuit(ops, graph=True)
        e.set_basis(x0)
        e.apply_circuit(ops)
        torch.cuda.synchronize()
        got = s.to_numpy()
        assert np.array_equal(got, e.to_numpy())
        y = np.arange(0, 1 << n, 4099)
        ref = np.exp(2j * np.pi * ((x0 * y) % (1 << n)) / (1 << n)) / 2 ** (n / 2)
        assert np.abs(got[y] - ref).max() <= 1e-6
    s.close()
    e.close()
