"""Regression pin: the oracle still reproduces its stored config-0 samples."""
import json
import os

import numpy as np

import oracle
from synth import voronoi_image, config_seed

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_config0_samples_reproduce():
    with open(os.path.join(HERE, "config0_samples.json")) as fh:
        gold = json.load(fh)
    f = voronoi_image(256, 256, config_seed(0, 0))
    for lam_s, case in gold["cases"].items():
        u = oracle.smooth(f, float(lam_s), 3.0, 0.1, radius=9)
        got = [u[i, j] for i, j in gold["samples"]]
        assert np.allclose(got, case["u"], rtol=0, atol=1e-13)
        assert abs(u.mean() - case["u_mean"]) < 1e-13
        assert abs(np.linalg.norm(u) - case["u_l2"]) < 1e-10
