"""GPU parity of the source iteration (eq. SI, BGK slabs) against the oracle,
through the C ABI: sweeps on ragged instances at first and second order, the
V-cycle with SI as smoother, graph replays, the converged state, and the
argument checks of the mode."""
import numpy as np
import pytest

from oracle import sweep as SW
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


INST = [dict(nx=5, eps=0.1, mass=1.0), dict(nx=1, eps=0.5, mass=0.9),
        dict(nx=4, eps=0.01, T_L=1.5, T_R=1.0, mass=1.2, xL=-1.0, xR=2.0)]


def _setup(bz, instances, order=1, N=8, L=6.0):
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=3)
    probs, f0 = [], []
    for d in instances:
        p = SW.Slab(spec=sp, nx=d["nx"], xL=d.get("xL", 0.0), xR=d.get("xR", 1.0), T_L=d.get("T_L", 1.0),
                    T_R=d.get("T_R", 2.0), eps=d["eps"], mass=d.get("mass", 1.0), collision="bgk", inner="si",
                    order=order)
        probs.append(p)
        f0.append(SW.initial_state(p, T=1.5))
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=3)
    fg = torch.from_numpy(np.concatenate(f0)).to("cuda:0").contiguous()
    slab = bz.Slab(ctx, instances, fg, collision="bgk", mode="si", order=order)
    return probs, f0, ctx, slab, fg


def _split(fg, instances):
    out, o, a = [], 0, fg.cpu().numpy()
    for d in instances:
        out.append(a[o:o + d["nx"]])
        o += d["nx"]
    return out


@pytest.mark.parametrize("order", [1, 2])
def test_si_sweeps_match_oracle(bz, order):
    print(f"si sweeps order {order}", flush=True)
    probs, f0, ctx, slab, fg = _setup(bz, INST, order)
    res, st = slab.sweep(3)
    got = _split(fg, INST)
    for i, p in enumerate(probs):
        f = f0[i]
        for _ in range(3):
            f = SW.sgs_iteration(p, f)
        err = np.max(np.abs(got[i] - f)) / f.max()
        print(f"  instance {i}: max rel diff {err:.3e}", flush=True)
        assert err < 1e-12, i
        ref = SW.outer_residual(p, f)
        assert abs(res[i] - ref) < 1e-10 * ref, i
    visits = 3 * 2 * sum(d["nx"] for d in INST)
    assert st["visits"] == visits and st["inner_iters"] == visits and st["fallbacks"] == 0


def test_si_vcycle_matches_oracle(bz):
    inst = [dict(nx=8, eps=0.1, mass=1.0)]
    print("si vcycle", flush=True)
    probs, f0, ctx, slab, fg = _setup(bz, inst)
    res, _ = slab.vcycle(1, coarsest=2, nu1=1, nu2=1, coarse_iters=3, tol=0.0)
    f = SW.vcycle(probs[0], f0[0], None, 2, 1, 1, 0.0, coarse_iters=3)
    f = f * (probs[0].mass / SW.total_mass(probs[0], f))
    got = _split(fg, inst)[0]
    assert np.max(np.abs(got - f)) < 1e-10 * f.max()
    assert abs(res[0] - SW.outer_residual(probs[0], f)) < 1e-9 * res[0]


def test_si_graph_replays_match_eager_sweeps(bz):
    print("si graph replays", flush=True)
    probs, f0, ctx, slab_e, fg_e = _setup(bz, INST)
    fg_g = fg_e.clone()
    slab_g = bz.Slab(ctx, INST, fg_g, collision="bgk", mode="si")
    graph = slab_g.capture(2)
    for rep in range(3):
        res_e, st_e = slab_e.sweep(2)
        res_g, st_g = graph.launch()
        torch.cuda.synchronize()
        _ = (fg_g * 2.0).sum().item()  # eager work between replays
        assert (fg_g - fg_e).abs().max().item() <= 1e-13 * fg_e.abs().max().item(), rep
        for a, b in zip(res_e, res_g):
            assert abs(a - b) <= 1e-12 * a, rep
    graph.close()
    slab_g.close()


def test_si_reaches_the_pfp_steady_state(bz):
    # 16^3, one instance: SI and SGS-PFP sweeps drive the outer residual below
    # 1e-9 from the same state and reach the same field
    inst = [dict(nx=4, eps=1.0, mass=1.0)]
    sp = Spec(d=3, N=16, L=6.0)
    p = SW.Slab(spec=sp, nx=4, eps=1.0, collision="bgk")
    f0 = SW.initial_state(p, T=1.5)
    ctx = bz.Context(N=16, L=6.0, n_theta=2, n_phi=4, n_rho=3)
    out = []
    for mode in ("si", "pfp"):
        fg = torch.from_numpy(f0.copy()).to("cuda:0").contiguous()
        slab = bz.Slab(ctx, inst, fg, collision="bgk", mode=mode, tol=1e-12, max_iter=200)
        for it in range(600):
            res, _ = slab.sweep(1)
            if res[0] < 1e-10:
                break
        print(f"  {mode}: {it + 1} iterations, residual {res[0]:.3e}", flush=True)
        assert res[0] < 1e-10
        out.append(fg.cpu().numpy())
    assert np.abs(out[0] - out[1]).max() < 1e-8 * out[1].max()


def test_si_mode_is_checked(bz):
    ctx = bz.Context(N=8, L=6.0, n_theta=2, n_phi=4, n_rho=2)
    K = ctx.K
    f = torch.ones((2, K), dtype=torch.float64, device="cuda:0")
    with pytest.raises(bz.BZError):
        bz.Slab(ctx, [dict(nx=2, eps=0.1)], f, collision="binary", mode="si")
    slab = bz.Slab(ctx, [dict(nx=2, eps=0.1)], f, collision="bgk", mode="si")
    with pytest.raises(bz.BZError):
        slab.attach_warmstart(bz.MLP(ctx, K + 6, 16, K))
    r = torch.zeros((1, K), dtype=torch.float64, device="cuda:0")
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(bz.BZError):
        ctx.cell_solve(r, one, one, 0.1, f[:1].contiguous(), mode="si")
    with pytest.raises(ValueError):
        bz.Slab(ctx, [dict(nx=2, eps=0.1)], f, collision="bgk", mode="sgs")
