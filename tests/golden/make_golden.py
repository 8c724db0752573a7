#!/usr/bin/env python3
"""Write the stored expected values under tests/golden/.

Every value here comes from the float64 oracle (oracle/) on inputs from the
seeded generators (paper_2006_07057_amd/inputs.py, which holds none of the
method's arithmetic); nothing is taken from the GPU library.  The paper
prints no worked example with numbers for this path, so the fixtures are
oracle values, each stamped with the recipe that reproduces it:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2006_07057_amd import inputs  # noqa: E402


def gauss2d_1k():
    """Two 2-D Gaussians (the setting of Sec. 5's first experiment):
    x ~ N(0, I), y ~ N(1.5 1, I), n = m = 1000, uniform weights, eps = 0.5,
    r = 128 anchors from N(0, I) (sigma^2 = 1, q = 4 sigma^2 / eps), 200
    fixed iterations of Algorithm 1 from u = 1 on the dense K_theta."""
    c = inputs.gauss2d(0, n=1000, m=1000)
    eps, s2, r = 0.5, 1.0, 128
    q = oracle.q_from_sigma2(s2, eps)
    U = inputs.gaussian_anchors(0, r, 2, s2)
    div = oracle.divergence(c.X, c.Y, c.a, c.b, U, eps, q, fixed_iter=200)
    return {"recipe": "inputs.gauss2d(0, n=1000, m=1000); "
                      "inputs.gaussian_anchors(0, 128, 2, 1.0); eps=0.5; q=8; "
                      "200 fixed iterations (oracle.divergence)",
            "eps": eps, "q": q, "r": r, "fixed_iter": 200,
            "W_bar": div.value, "W_xy": div.w_xy, "W_xx": div.w_xx, "W_yy": div.w_yy}


def lambert_q():
    """Lemma 1's bandwidth q = z / (2 W0(z)), z = R^2 / (eps d)."""
    cases = [(1.0, 1.0, 1), (4.0, 0.1, 3), (2.5, 0.05, 64), (30.0, 10.0, 784),
             (1.0, 1.0, 128), (3.2, 0.1, 3)]
    return {"recipe": "oracle.lambert_q(R, eps, d)",
            "cases": [{"R": R, "eps": e, "d": d, "q": oracle.lambert_q(R, e, d)}
                      for (R, e, d) in cases]}


def accelerated_inputs():
    """Float32 row-normalised Gaussian features of two clouds and Dirichlet
    weights (the inputs of the accelerated fixture; the feature values are
    the oracle's, rounded to float32)."""
    rng = np.random.default_rng(11)
    n, m, r, eps = 400, 300, 64, 0.5
    X = rng.standard_normal((n, 2))
    Y = rng.standard_normal((m, 2)) + 1.0
    U = rng.standard_normal((r, 2))
    Ex = oracle.gaussian_log_features(X, U, eps, 8.0)
    Ey = oracle.gaussian_log_features(Y, U, eps, 8.0)
    Fx = np.exp(Ex - Ex.max(1)[:, None]).astype(np.float32)
    Fy = np.exp(Ey - Ey.max(1)[:, None]).astype(np.float32)
    a = inputs.dirichlet_weights(rng, n)
    b = inputs.dirichlet_weights(rng, m)
    return Fx, Fy, a, b


def accelerated_small():
    """Accelerated Sinkhorn (oracle.accelerated_sinkhorn) for 30 accepted
    steps from zero on accelerated_inputs(), and its dual value F."""
    Fx, Fy, a, b = accelerated_inputs()
    Px, Py = Fx.astype(np.float64), Fy.astype(np.float64)
    res = oracle.accelerated_sinkhorn(lambda v: Px @ (Py.T @ v), lambda u: Py @ (Px.T @ u),
                                      a, b, fixed_iter=30)
    F = oracle.dual_value(res.eta1, res.eta2, Px @ Py.T, a, b, 1.0)
    return {"recipe": "rng=default_rng(11); X~N(0,I_2) (400), Y~N(1,I_2) (300), "
                      "U~N(0,I_2) (64); features exp(E - max E) at eps=0.5, q=8 as "
                      "float32; a, b = inputs.dirichlet_weights(rng, .); 30 accepted "
                      "steps from zero, L0 = 1",
            "steps": 30, "trials": res.trials, "dual_value": F,
            "min_block_margin": min(res.margins), "min_test_margin": min(res.ls_margins)}


def main():
    for name, fn in (("gauss2d_1k", gauss2d_1k), ("lambert_q", lambert_q),
                     ("accelerated_small", accelerated_small)):
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(fn(), f, indent=1)
            f.write("\n")
        print("wrote", path)


if __name__ == "__main__":
    main()
