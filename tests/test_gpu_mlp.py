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


def test_split_k_products_match_oracle(dev):
    # a long input (the first layer's K) and a long output (the backward
    # product's K) with a small batch take the split-K path
    import paper_2409_01910_amd as bz

    n_in, H, n_out, B = 4099, 40, 3000, 9
    ctx = bz.Context(N=8, L=4.0, n_theta=2, n_phi=4, n_rho=2)
    m = bz.MLP(ctx, n_in, H, n_out, seed=3)
    rng = np.random.default_rng(3)
    p = (rng.normal(size=m.n_params) / np.sqrt(n_in)).astype(np.float32)
    m.set_params(p)
    X = rng.normal(size=(B, n_in)).astype(np.float32)
    T = rng.normal(size=(B, n_out)).astype(np.float32)
    y = m.forward(torch.from_numpy(X).to(dev)).cpu().numpy()
    ybf = m.forward(torch.from_numpy(X).to(dev), bf16=True).cpu().numpy()
    ref, _ = OM.forward(p.astype(np.float64), X.astype(np.float64), n_in, H, n_out)
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() < 1e-5 * scale
    assert np.abs(ybf - ref).max() < 3e-2 * scale
    loss, g = m.grad(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev))
    lref, gref = OM.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n_in, H, n_out)
    assert abs(loss - lref) < 1e-5 * lref
    assert np.abs(g.cpu().numpy() - gref).max() < 1e-4 * np.abs(gref).max()


def test_trained_network_gain_in_the_scans(dev):
    # The learned start trained on the solver's own iterates, measured on
    # held-out heat slabs (16^3, 16 cells, MG-SGS-PFP to outer 1e-6; 16^3 does
    # not reach 1e-8, and below eps ~ 0.01 the V-cycles do not converge on this
    # coarse velocity grid, so the held-out eps are 0.3, 0.1, 0.05).  Asserted: training learns (loss below half its start),
    # every run converges, the converged states agree, and the work changes by
    # less than 5%: the network's guess is taken in few visits, because the
    # iterate before a scan already nearly solves the cell problem the network
    # can see (its upwind neighbour is not yet updated).  The counts are
    # printed; the 32^3 measurement is the benchmark's.
    import paper_2409_01910_amd as bz
    from paper_2409_01910_amd import warmstart as WS

    ctx = bz.Context(N=16, L=8.0, n_theta=4, n_phi=8, n_rho=4)
    train = [WS.heat_slab_instance(5, i, 16) for i in range(8)]
    X, Y, info = WS.sweep_dataset(ctx, train, n_snap=3)
    # 120 epochs (600 Adam steps): the dataset is the solver's own iterates less
    # the cells whose inner solve misses 1e-10, and which borderline cells miss
    # it moves with rounding-level changes of the collision term (361 to 372
    # samples seen), which after only 40 epochs left the loss at 0.45 to 0.58 of
    # its start
    mlp, hist, _ = WS.train(ctx, X, Y, hidden=64, epochs=120, batch=64, lr=2e-3)
    print(f"samples {info['samples']}, loss {hist[0]:.3e} -> {hist[-1]:.3e}", flush=True)
    assert hist[-1] < 0.5 * hist[0]
    plain_inner, learned_inner, taken = 0.0, 0.0, 0
    for i, e in enumerate((0.3, 0.1, 0.05)):
        inst = dict(WS.heat_slab_instance(5, 1000 + i, 16), eps=e)
        a = WS.time_to_residual([(ctx, None, 1e-6)], inst, tol=1e-6, return_field=True)
        b = WS.time_to_residual([(ctx, mlp, 1e-6)], inst, tol=1e-6, return_field=True)
        print(f"eps {inst['eps']:.4f}: plain {a['vcycles']} cycles {a['inner_per_visit']:.3f} updates/visit "
              f"(residual {a['final_residual']:.2e}), learned {b['vcycles']} cycles {b['inner_per_visit']:.3f} "
              f"updates/visit (residual {b['final_residual']:.2e}), taken {b['learned_taken']} of {b['visits']}",
              flush=True)
        assert a["reached"] and b["reached"]
        diff = (a["f"] - b["f"]).abs().max().item() / a["f"].abs().max().item()
        assert diff < 1e-4, diff  # both within the outer tolerance of the same state
        plain_inner += a["inner_per_visit"]
        learned_inner += b["inner_per_visit"]
        taken += b["learned_taken"]
    print(f"inner updates per visit: plain {plain_inner / 3:.4f}, learned {learned_inner / 3:.4f}; "
          f"learned starts taken: {taken}", flush=True)
    assert abs(learned_inner / plain_inner - 1.0) < 0.05
