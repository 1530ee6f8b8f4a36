"""Fixed-structure FAS V-cycles (no residual-based exits) against the oracle,
and their HIP-graph capture (bz_graph_capture_vcycles) against eager cycles,
through the C ABI."""
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


INST = [dict(nx=8, eps=0.1, mass=1.0), dict(nx=8, eps=0.02, T_L=1.3, T_R=1.9, mass=0.8)]


def _setup(bz, collision, fixed_inner=2, order=1):
    sp = Spec(d=3, N=8, L=6.0, n_theta=2, n_phi=4, n_rho=3)
    probs, f0 = [], []
    for d in INST:
        p = SW.Slab(spec=sp, nx=d["nx"], T_L=d.get("T_L", 1.0), T_R=d.get("T_R", 2.0), eps=d["eps"],
                    mass=d["mass"], collision=collision, fixed_inner=fixed_inner, order=order)
        probs.append(p)
        f0.append(SW.initial_state(p, T=1.5))
    ctx = bz.Context(N=8, L=6.0, n_theta=2, n_phi=4, n_rho=3)
    fg = torch.from_numpy(np.concatenate(f0)).to("cuda:0").contiguous()
    return probs, f0, ctx, fg


@pytest.mark.parametrize("collision,order", [("bgk", 1), ("binary", 1), ("binary", 2)])
def test_fixed_vcycle_matches_oracle(bz, collision, order):
    print(f"fixed vcycle {collision} order {order}", flush=True)
    probs, f0, ctx, fg = _setup(bz, collision, order=order)
    slab = bz.Slab(ctx, INST, fg, collision=collision, fixed_iters=2, order=order)
    res, _ = slab.vcycle(2, coarsest=2, nu1=1, nu2=1, coarse_iters=2, fixed_cycle=True)
    got = fg.cpu().numpy()
    for i, p in enumerate(probs):
        f = f0[i]
        for _ in range(2):
            f = SW.vcycle(p, f, None, 2, 1, 1, 0.0, coarse_iters=2, fixed=True)
            f = f * (p.mass / SW.total_mass(p, f))
        err = np.abs(got[8 * i:8 * i + 8] - f).max() / f.max()
        print(f"  instance {i}: max rel diff {err:.3e}", flush=True)
        assert err < 1e-10, i
        assert abs(res[i] - SW.outer_residual(p, f)) < 1e-9 * res[i], i


@pytest.mark.parametrize("collision", ["bgk", "binary"])
def test_captured_vcycles_match_eager_cycles(bz, collision):
    # the same state in two slabs: eager fixed cycles in one, replays of a graph
    # of two cycles in the other, with eager work and synchronisations between
    # the replays; every replay must match
    print(f"vcycle graph {collision}", flush=True)
    probs, f0, ctx, fg_e = _setup(bz, collision, fixed_inner=0)
    fg_g = fg_e.clone()
    slab_e = bz.Slab(ctx, INST, fg_e, collision=collision)
    slab_g = bz.Slab(ctx, INST, fg_g, collision=collision)
    graph = slab_g.capture_vcycles(2, coarsest=2, nu1=1, nu2=1, coarse_iters=3)
    start = fg_g.clone()
    for rep in range(3):
        res_e, st_e = slab_e.vcycle(2, coarsest=2, nu1=1, nu2=1, coarse_iters=3, fixed_cycle=True)
        res_g, st_g = graph.launch()
        torch.cuda.synchronize()
        _ = (fg_g * 2.0).sum().item()  # eager work between replays
        diff = (fg_g - fg_e).abs().max().item() / fg_e.abs().max().item()
        print(f"  replay {rep}: max rel diff {diff:.3e}, residuals {res_g}", flush=True)
        assert diff <= 1e-13, rep
        for a, b in zip(res_e, res_g):
            assert abs(a - b) <= 1e-12 * a, rep
        assert st_e["visits"] == st_g["visits"] and st_e["inner_iters"] == st_g["inner_iters"], rep
    assert (fg_g - start).abs().max().item() > 1e-6 * start.abs().max().item()
    graph.close()
    slab_g.close()
    slab_e.close()


def test_vcycle_capture_arguments_are_checked(bz):
    ctx = bz.Context(N=8, L=6.0, n_theta=2, n_phi=4, n_rho=2)
    f = torch.ones((6, ctx.K), dtype=torch.float64, device="cuda:0")
    slab = bz.Slab(ctx, [dict(nx=6, eps=0.1)], f, collision="bgk")
    with pytest.raises(bz.BZError):
        slab.capture_vcycles(1, coarsest=4)  # 6 cells do not halve down to 4
    with pytest.raises(bz.BZError):
        slab.capture_vcycles(0, coarsest=3)
    ctx2 = bz.Context(N=8, L=6.0, n_phi=8, n_rho=4, d=2)
    f2 = torch.ones((16, ctx2.K), dtype=torch.float64, device="cuda:0")
    walls = ((1.0, (0.0, 0.0)),) * 4
    cav = bz.Cavity(ctx2, 4, 4, 0.1, walls, f2)
    import ctypes

    o = bz.bz_mg_opts(2, 1, 1, 2, 0.0, 1)
    st = bz.bz_sweep_stats()
    res = ctypes.c_double(0.0)
    code = ctx2.lib.bz_cavity_vcycle(ctx2.h, cav.h, ctypes.byref(o), 1, ctypes.byref(res), ctypes.byref(st), None)
    assert code != 0  # the cavity keeps its residual-based exits
