"""Pin of the MLP oracle's backward pass: central finite differences."""
import numpy as np

from oracle import mlp as OM


def test_oracle_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    n_in, H, n_out, B = 7, 5, 4, 6
    theta = rng.normal(scale=0.4, size=OM.n_params(n_in, H, n_out))
    X = rng.normal(size=(B, n_in))
    T = rng.normal(size=(B, n_out))
    _, g = OM.loss_and_grad(theta, X, T, n_in, H, n_out)
    h = 1e-6
    for i in rng.choice(theta.size, size=25, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (OM.loss_and_grad(tp, X, T, n_in, H, n_out)[0] - OM.loss_and_grad(tm, X, T, n_in, H, n_out)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd))
