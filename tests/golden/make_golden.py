"""Write the stored expected values under tests/golden/.

The paper prints no per-pixel values or worked example, so every stored value
here is written by this script, which calls only the FP64 oracle and the
seeded input generator.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import voronoi_image, config_seed  # noqa: E402

# 256x256 grayscale workload: sigma_s = 3 (r = 9), sigma_r = 0.1, one iteration,
# lambda at the paper's default 1024 and at the fallback 20
SAMPLES = [(0, 0), (0, 255), (17, 3), (128, 128), (200, 77), (255, 255), (99, 201), (63, 1)]


def main():
    f = voronoi_image(256, 256, config_seed(0, 0))
    out = {"workload": "grayscale 256x256, seed 0, sigma_s=3, r=9, sigma_r=0.1, n=1",
           "samples": SAMPLES, "cases": {}}
    for lam in (1024.0, 20.0):
        u = oracle.smooth(f, lam, 3.0, 0.1, radius=9)
        out["cases"][repr(lam)] = {
            "u": [float(u[i, j]) for i, j in SAMPLES],
            "u_mean": float(u.mean()),
            "u_l2": float(np.linalg.norm(u)),
        }
    with open(os.path.join(HERE, "config0_samples.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
