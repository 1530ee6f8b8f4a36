"""GPU checks of the warm-start network kernels (matrix-core GEMMs, backward,
Adam) against the FP64 oracle, and of the learned cell update."""
import numpy as np
import pytest

from oracle import mlp as OM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return torch.device("cuda:0")


def _net(dev, n_in=37, H=24, n_out=19, seed=1):
    import paper_2409_01910_amd as bz

    ctx = bz.Context(N=8, L=4.0, n_theta=2, n_phi=4, n_rho=2)
    m = bz.MLP(ctx, n_in, H, n_out, seed=seed)
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=0.3, size=m.n_params).astype(np.float32)
    m.set_params(p)
    return ctx, m, p.astype(np.float64)


@pytest.mark.parametrize("B", [1, 50, 130])
def test_forward_matches_oracle(dev, B):
    ctx, m, p = _net(dev)
    rng = np.random.default_rng(B)
    X = rng.normal(size=(B, 37)).astype(np.float32)
    y32 = m.forward(torch.from_numpy(X).to(dev)).cpu().numpy()
    ybf = m.forward(torch.from_numpy(X).to(dev), bf16=True).cpu().numpy()
    ref, _ = OM.forward(p, X.astype(np.float64), 37, 24, 19)
    scale = np.abs(ref).max()
    assert np.abs(y32 - ref).max() < 1e-5 * scale
    assert np.abs(ybf - ref).max() < 3e-2 * scale


def test_gradient_matches_oracle(dev):
    ctx, m, p = _net(dev)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(70, 37)).astype(np.float32)
    T = rng.normal(size=(70, 19)).astype(np.float32)
    loss, g = m.grad(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev))
    lref, gref = OM.loss_and_grad(p, X.astype(np.float64), T.astype(np.float64), 37, 24, 19)
    assert abs(loss - lref) < 1e-5 * lref
    g = g.cpu().numpy()
    assert np.abs(g - gref).max() < 1e-4 * np.abs(gref).max()


def test_adam_steps_reduce_the_loss(dev):
    ctx, m, _ = _net(dev)
    rng = np.random.default_rng(9)
    X = torch.from_numpy(rng.normal(size=(256, 37)).astype(np.float32)).to(dev)
    W = rng.normal(size=(37, 19))
    T = torch.from_numpy(np.tanh(X.cpu().numpy() @ W * 0.2).astype(np.float32)).to(dev)
    l0, _ = m.grad(X, T)
    for _ in range(200):
        m.train_step(X, T, 3e-3)
    l1, _ = m.grad(X, T)
    assert l1 < 0.2 * l0


def test_learned_start_keeps_answers_and_never_costs_iterations(dev):
    # what the trained network gains is measured and printed; the assertions
    # are that the converged answers are unchanged and no cell needs more
    # updates on average than with the plain start
    import paper_2409_01910_amd as bz
    from paper_2409_01910_amd import warmstart as WS

    ctx = bz.Context(N=8, L=8.0, n_theta=2, n_phi=4, n_rho=3)
    dx = 40.0 / 128
    X, Y, _, _ = WS.make_dataset(ctx, 60, 8, dx, seed=7)
    mlp, hist = WS.train(ctx, X, Y, hidden=64, epochs=80, batch=64, lr=2e-3)
    print("loss", hist[0], hist[-1])
    assert hist[-1] < 0.9 * hist[0]  # training makes progress
    _, _, (fo, inflow, eps), _ = WS.make_dataset(ctx, 10, 8, dx, seed=7, start=1000)
    res = WS.compare(ctx, mlp, fo, inflow, eps, dx, tol=1e-8)
    print(res)
    assert res["plain"]["unconverged"] == 0 and res["learned"]["unconverged"] == 0
    # both reach the same fixed point of eq. inner_eqn (each within the inner tolerance)
    assert res["max_rel_diff"] < 1e-6
    assert res["learned"]["mean_iterations"] <= res["plain"]["mean_iterations"]
    print(f"gain: mean inner updates {res['plain']['mean_iterations']:.3f} -> {res['learned']['mean_iterations']:.3f}, "
          f"learned start kept in {res['learned']['learned_kept']} cells")
