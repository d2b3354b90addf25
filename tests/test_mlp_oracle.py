"""Pin of the FP64 network reference: its hand-written gradient equals central
finite differences of its loss (an independent route to the same derivative)."""
import numpy as np

from oracle import mlp_ref


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_in, H, n_out, B = 7, 5, 3, 4
    n = mlp_ref.n_params(n_in, H, n_out)
    w = rng.normal(scale=0.5, size=n)
    x = rng.normal(size=(B, n_in))
    t = rng.normal(size=(B, n_out))
    _, g = mlp_ref.loss_grad(w, x, t, n_in, H, n_out)
    eps = 1e-6
    fd = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = eps
        fd[i] = (mlp_ref.loss(w + e, x, t, n_in, H, n_out) - mlp_ref.loss(w - e, x, t, n_in, H, n_out)) / (2 * eps)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))
