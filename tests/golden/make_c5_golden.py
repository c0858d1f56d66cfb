"""Writes c5_gradients.json: the oracle's energy, parameter-shift
derivatives and central finite differences (h = 1e-5) for 16 parameters of
the 24-qubit gradient workload (6 layers of RX, RY, RZ per qubit + CZ ring,
seed 1005, H = sum Z_i Z_{i+1} (open chain) + 0.7 sum X_i): every 27th
parameter, which visits every layer and all three rotation axes.  Calls only
oracle/ and the seeded input generators; about 65 oracle forward passes at
24 qubits (minutes on a few host cores)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import qcircuits as qc  # noqa: E402
from oracle import oracle as O  # noqa: E402

n, layers = 24, 6
params, ham = qc.gradient_workload(n, layers, qc.SEEDS["c5"])
build = lambda p: qc.rot_ring_ansatz(n, p, layers)
indices = list(range(0, params.size, 27))
assert len(indices) == 16
energy = O.energy(build, params, ham, n)
grad = O.param_shift_grad(build, params, ham, n, indices=indices)
fd = O.finite_diff_grad(build, params, ham, n, indices=indices, h=1e-5)
out = {"n": n, "layers": layers, "seed": qc.SEEDS["c5"], "energy": energy,
       "indices": indices, "grad": [float(x) for x in grad], "fd": [float(x) for x in fd],
       "source": "oracle/oracle.py param_shift_grad (exact for exp(-i theta P/2)) and "
                 "finite_diff_grad (central, h = 1e-5), complex128"}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_gradients.json"), "w") as f:
    json.dump(out, f, indent=1)
print(out)
