"""The surrogate network's GPU kernels against the FP64 reference."""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _setup(n_in=70, H=48, n_out=20, B=37, seed=0, wscale=0.3):
    from paper_2311_15429_amd.mlp import Mlp
    rng = np.random.default_rng(seed)
    n = mlp_ref.n_params(n_in, H, n_out)
    w = rng.normal(scale=wscale, size=n)
    x = rng.normal(size=(B, n_in))
    t = rng.normal(size=(B, n_out))
    m = Mlp(n_in, H, n_out, max_batch=max(64, B), stream=torch.cuda.current_stream())
    m.set_params(torch.from_numpy(w.astype(np.float32)))
    return m, w.astype(np.float32).astype(np.float64), x.astype(np.float32), t.astype(np.float32)


@pytest.mark.parametrize("n_in", [70, 3000])
def test_forward_matches_reference(n_in):
    """n_in = 3000 runs the first layer and the skip as split-K products."""
    m, w, x, t = _setup(n_in=n_in)
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = mlp_ref.forward(w, x.astype(np.float64), m.n_in, m.n_hidden, m.n_out)
    assert np.max(np.abs(y - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n_in, H, n_out, B", [(300, 160, 20, 150), (8450, 256, 80, 990)])
def test_forward_matches_reference_several_tiles(n_in, H, n_out, B):
    """Products over several 128 x 128 output tiles with ragged edges in both
    directions, and the surrogate network's own shape (8450 inputs, 2 x 256
    hidden, 80 outputs) at an inference batch of 990 far pairs."""
    m, w, x, t = _setup(n_in=n_in, H=H, n_out=n_out, B=B, seed=4, wscale=1.0 / np.sqrt(n_in))
    y = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = mlp_ref.forward(w, x.astype(np.float64), m.n_in, m.n_hidden, m.n_out)
    assert np.max(np.abs(y - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n_in, H, n_out, B", [(70, 48, 20, 37), (3000, 48, 20, 37), (300, 160, 20, 150),
                                               (8450, 256, 80, 300)])
def test_gradient_matches_reference(n_in, H, n_out, B):
    """The backward products (transposed operands, split along K) at sizes
    from one ragged tile to the surrogate network's own shape."""
    m, w, x, t = _setup(n_in=n_in, H=H, n_out=n_out, B=B, seed=1,
                        wscale=0.3 if n_in < 300 else 1.0 / np.sqrt(n_in))
    loss, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    rl, rg = mlp_ref.loss_grad(w, x.astype(np.float64), t.astype(np.float64), m.n_in, m.n_hidden, m.n_out)
    g = g.cpu().numpy()
    assert abs(float(loss.cpu()) - rl) <= 1e-5 * abs(rl)
    assert np.max(np.abs(g - rg)) <= 1e-3 * np.max(np.abs(rg))
    # per block (W1, b1, ...), relative to that block's scale
    o = 0
    for size in [m.n_in * m.n_hidden, m.n_hidden, m.n_hidden ** 2, m.n_hidden, m.n_hidden * m.n_out, m.n_out,
                 m.n_in * m.n_out]:
        blk, rblk = g[o:o + size], rg[o:o + size]
        assert np.max(np.abs(blk - rblk)) <= 1e-3 * np.max(np.abs(rblk)) + 1e-9
        o += size


def test_training_reduces_loss_on_a_linear_map():
    """Adam steps on the GPU fit a fixed linear map of the inputs."""
    from paper_2311_15429_amd.mlp import Mlp
    rng = np.random.default_rng(3)
    n_in, H, n_out, B = 16, 32, 4, 64
    A = rng.normal(size=(n_in, n_out)) / np.sqrt(n_in)
    n = mlp_ref.n_params(n_in, H, n_out)
    w0 = rng.normal(scale=1.0 / np.sqrt(H), size=n).astype(np.float32)
    m = Mlp(n_in, H, n_out, max_batch=B, stream=torch.cuda.current_stream())
    m.set_params(torch.from_numpy(w0))
    first = last = None
    for it in range(400):
        x = rng.normal(size=(B, n_in)).astype(np.float32)
        t = (x @ A).astype(np.float32)
        loss = float(m.train_step(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), 3e-3).cpu())
        if it == 0:
            first = loss
        last = loss
    assert last < 0.05 * first
