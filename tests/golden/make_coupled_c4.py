"""Write ``coupled_c4_history.json``: the FP64 oracle's macroscopic history
of the coupled workload at full length.

The workload (layer case, sec. 3.2.1; static/transport alternation of
sec. 3.1.1): a 512 x 512 layer with 20 seeded loops (plateaus +-0.2, erfc
edges sigma 2, radii 20-80, seed 4), a 4-voxel layer in a 512-voxel cell,
mu = 1, lambda = 1.5, threshold 0.01, mobility 1, strain rate 1e-3 from
eps13 = 0, minmod, Heun, Courant 0.4 with the step capped at 0.02, 5000
steps; one record every 100 steps.

Only the oracle (``oracle/``) computes: the inputs come from the seeded
generator shared with the GPU tests (float32 densities, as the library
receives them).  Run from the repository root:
    python3 tests/golden/make_coupled_c4.py
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import coupled as CP  # noqa: E402
from paper_1911_03225_amd import workloads as W  # noqa: E402

CONFIG = dict(n=512, seed=4, steps=5000, chunk=100, limiter="minmod", cfl=0.4, time_order=2, mu=1.0, lam=1.5,
              layer_h=4.0, cell_l3=512.0, tau0=0.01, mobility=1.0, strain_rate13=1e-3, dt_max=0.02, eps13=0.0)
KEYS = ("step", "t", "dt", "eps13", "sigma13", "phi_mean", "vmax", "sum11", "sum12", "sum_abs", "max_norm")


def main(out=os.path.join(HERE, "coupled_c4_history.json")):
    c = CONFIG
    phi, a11, a12 = W.plateau_rings(c["n"], c["n"], seed=c["seed"])
    t0 = time.time()
    _, _, hist = CP.coupled_run(a11, a12, c["steps"], c["chunk"], dx=1.0, limiter=c["limiter"], cfl=c["cfl"],
                                time_order=c["time_order"], mu=c["mu"], lam=c["lam"], layer_h=c["layer_h"],
                                cell_l3=c["cell_l3"], tau0=c["tau0"], mobility=c["mobility"],
                                strain_rate13=c["strain_rate13"], dt_max=c["dt_max"], eps13=c["eps13"],
                                phi_mean=float(phi.mean()))
    doc = {"config": dict(c, phi_mean0=float(phi.mean())),
           "source": "oracle/coupled.py (FP64), written by tests/golden/make_coupled_c4.py",
           "columns": list(KEYS),
           "history": [[r[k] for k in KEYS] for r in hist]}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=0)
    print("wrote %s (%d records, %.0f s)" % (out, len(hist), time.time() - t0))


if __name__ == "__main__":
    main()
