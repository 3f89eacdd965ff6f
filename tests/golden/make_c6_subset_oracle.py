"""Writes c6_subset_oracle.json: FP64 oracle results of the whole-surface
workload (the T4L-sized receptor and ligand on the 62 A grid: 248^3 points
at 0.25 A, zero-padded to a 256^3 FFT, occupancy mode) for an evenly
strided subset of 16 of its 8000 configurations: per-configuration partials
and the BPMF pooled over the subset (Eq. 2), used by the full-size GPU check
of the 256-point path.

Calls only oracle/ and the input generators.  Run from the repository root:
    python tests/golden/make_c6_subset_oracle.py
(several minutes on 8 cores: the FP64 receptor grids of 15 M points and the
direct sums over about 9 M translations per configuration)."""
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

STRIDE = 500


if __name__ == "__main__":
    w = synth.config6()
    sel = np.arange(0, w.ligands[0].n_cfg, STRIDE)
    t = time.time()
    go, oo = oracle.receptor_grids(w)
    t_grid = time.time() - t
    print(f"grids {t_grid:.0f}s", flush=True)
    parts, boxes = oracle.scan(w, go, oo, cfgs=sel)
    out = {"workload": "config 6: 2600-atom cavity receptor on a 248^3 grid at 0.25 A (62 A) in a 256^3 FFT, "
                       "occupancy mode, 25-atom ligand x 8 conformers x 1000 rotations, 300 K, FP64 direct "
                       "trilinear sums (oracle); configurations 0, 500, ..., 7500",
           "configs": [int(c) for c in sel],
           "B": est.bpmf(parts, w.T),
           "partials": [[float(x) for x in row] for row in parts],
           "boxes": boxes.tolist(),
           "seconds": {"grids": t_grid, "scan": time.time() - t - t_grid}}
    print({k: v for k, v in out.items() if k not in ("partials", "boxes")}, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c6_subset_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
