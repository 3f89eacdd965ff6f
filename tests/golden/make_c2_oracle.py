"""Writes c2_oracle.json: FP64 oracle results of the full T4L-sized
workload (8000 configurations, one snapshot) in occupancy mode and in
capped-repulsion mode, used by the full-size GPU parity test (the precision
study: FP32 scan, FP64 accumulation, error stated per result).  With
--stress it writes c2_stress_oracle.json: the same geometry with the tiny
case's atom parameters (q ~ N(0, 0.4) e, eps ~ U(0.05, 0.2) kcal/mol), whose
grids span a larger dynamic range.

Calls only oracle/ and the input generators.  Run from the repository root:
    python tests/golden/make_c2_oracle.py [--stress]
(about 10-20 minutes on 8 cores)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import estimators as est  # noqa: E402
from workload import synth  # noqa: E402


def run(mode, params):
    w = synth.config2(params=params)
    w.clash_mode = mode
    t = time.time()
    go, oo = oracle.receptor_grids(w)
    parts, boxes = oracle.scan(w, go, oo)
    B = est.bpmf(parts, w.T)
    vs = est.v_site(boxes, w.n_rec, w.h)
    dg = est.dg_standard(np.array([B]), np.ones(1), vs, w.T)
    lz = est.log_z(parts)
    out = {"B": B, "dG": dg, "v_site": vs, "psi_min": float(np.min(parts[:, 4])),
           "n_finite": int(parts[:, 3].sum()), "n_samples": int(parts[:, 2].sum()),
           "n_cfg": int(parts.shape[0]),
           "log_z_every_100th": [float(x) if np.isfinite(x) else None for x in lz[::100]],
           "seconds": time.time() - t}
    print(mode, {k: v for k, v in out.items() if k != "log_z_every_100th"}, flush=True)
    return out


if __name__ == "__main__":
    stress = "--stress" in sys.argv[1:]
    params = synth.TINY_PARAMS if stress else synth.CAVITY_PARAMS
    res = {"workload": "config 2: 2600-atom cavity receptor, 96^3 grid at 0.25 A, 25-atom ligand x 8 conformers "
                       "x 1000 rotations, 300 K, FP64 direct trilinear sums (oracle)"
                       + (", atom parameters q ~ N(0, 0.4) e, eps ~ U(0.05, 0.2) kcal/mol" if stress else ""),
           "occ": run("occ", params), "cap": run("cap", params)}
    name = "c2_stress_oracle.json" if stress else "c2_oracle.json"
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), name), "w") as f:
        json.dump(res, f, indent=1)
