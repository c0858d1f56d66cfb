"""Writes c5_gradients.json: the oracle's energy and parameter-shift
derivatives for selected parameters of the 24-qubit gradient workload
(6 layers of RX, RY, RZ per qubit + CZ ring, seed 1005,
H = sum Z_i Z_{i+1} (open chain) + 0.7 sum X_i).  Calls only oracle/ and the
seeded input generators."""
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
indices = [0, 1, 2, 215, 431]
energy = O.energy(build, params, ham, n)
grad = O.param_shift_grad(build, params, ham, n, indices=indices)
out = {"n": n, "layers": layers, "seed": qc.SEEDS["c5"], "energy": energy,
       "indices": indices, "grad": [float(x) for x in grad],
       "source": "oracle/oracle.py param_shift_grad (exact for exp(-i theta P/2)), complex128"}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_gradients.json"), "w") as f:
    json.dump(out, f, indent=1)
print(out)
