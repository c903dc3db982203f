"""What the learned surrogate gains over the method without it (GPU).

A small surrogate (32^3 voxels, 3 levels from 16 channels) is trained from
scratch by the project's own kernels on supernova cubes that the plain
small-timestep SPH generates, then evaluated on held-out cubes against that
plain SPH.  Without the surrogate the galaxy has two choices for such a
region: keep its state for the 0.1 Myr (persistence: the explosion is
missed) or integrate it at the global 2,000 yr step (far above the Courant
limit right after the explosion).  The surrogate must beat persistence in the
loss's standardized channels and in the tail of the log-temperature error,
beat the fixed-step SPH, and take less time than the plain small-dt SPH it
replaces.
"""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_gain(gx, tmp_path):
    from paper_2510_23330_amd import sn_train
    m = sn_train.main(["--n-train", "48", "--n-test", "8", "--per-batch", "56", "--grid", "32",
                       "--base", "16", "--levels", "3", "--batch", "4", "--lr", "1e-3",
                       "--epochs", "400", "--train-seconds", "45", "--seed0", "7000",
                       "--out", str(tmp_path)])
    print(json.dumps({k: m[k] for k in ("mse_standardized", "surrogate_vs_sph",
                                        "persistence_vs_sph", "coarse_dt_sph_vs_sph", "timing")}))
    mse = m["mse_standardized"]
    assert mse["surrogate"] < 0.5 * mse["persistence"]
    s, p, c = m["surrogate_vs_sph"], m["persistence_vs_sph"], m["coarse_dt_sph_vs_sph"]
    assert s["log_T"]["p90"] < p["log_T"]["p90"]
    assert s["log_T"]["mean"] < p["log_T"]["mean"]
    assert s["log_T"]["mean"] < c["log_T"]["mean"]
    assert s["log_rho"]["mean"] < c["log_rho"]["mean"]
    assert m["timing"]["speedup"] > 1.0
