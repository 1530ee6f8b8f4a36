"""GPU parity of the slab with one velocity dimension (the 1D1V BGK model of
Section 4.1) against the oracle, through the C ABI: SGS sweeps with the
source iteration, the plain and the preconditioned visit at first and second
order on ragged instances, V-cycles (with and without their exits), the
converged state, and the argument checks of d = 1 contexts."""
import numpy as np
import pytest

from oracle import sweep as SW
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCAN_TOL = 1e-11  # the Newton tolerance (1e-13) compounded over a scan's visits
N, L = 50, 6.0
INST = [dict(nx=5, eps=0.1, mass=1.0, xL=-0.5, xR=0.5), dict(nx=1, eps=1.0, mass=0.9),
        dict(nx=4, eps=0.01, T_L=1.5, T_R=1.0, mass=1.2, xL=-1.0, xR=2.0)]


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


def _setup(bz, instances, mode, fixed, order=1, limiter="none", bgk_nu=None, tol=1e-8):
    sp = Spec(d=1, N=N, L=L)
    probs, f0 = [], []
    for d in instances:
        p = SW.Slab(spec=sp, nx=d["nx"], xL=d.get("xL", 0.0), xR=d.get("xR", 1.0), T_L=d.get("T_L", 1.0),
                    T_R=d.get("T_R", 2.0), eps=d["eps"], mass=d.get("mass", 1.0), collision="bgk", bgk_nu=bgk_nu,
                    inner=mode, fixed_inner=fixed, order=order, limiter=limiter, tol_inner=tol)
        probs.append(p)
        f0.append(SW.initial_state(p, T=1.5))
    ctx = bz.Context(N=N, L=L, d=1)
    fg = torch.from_numpy(np.concatenate(f0)).to("cuda:0").contiguous()
    slab = bz.Slab(ctx, instances, fg, collision="bgk", bgk_nu=bgk_nu or 0.0, mode=mode, fixed_iters=fixed or 0,
                   order=order, limiter=limiter, tol=tol)
    return probs, f0, ctx, slab, fg


def _split(fg, instances):
    out, o, a = [], 0, fg.cpu().numpy()
    for d in instances:
        out.append(a[o:o + d["nx"]])
        o += d["nx"]
    return out


@pytest.mark.parametrize("mode,order,limiter", [("si", 1, "none"), ("fp", 1, "none"), ("pfp", 1, "none"),
                                                ("pfp", 2, "none"), ("pfp", 2, "minmod"), ("si", 2, "none")])
def test_sweeps_match_oracle(bz, mode, order, limiter):
    print(f"1v sweeps {mode} order {order} {limiter}", flush=True)
    fixed = None if mode == "si" else 3
    probs, f0, ctx, slab, fg = _setup(bz, INST, mode, fixed, order, limiter)
    res, st = slab.sweep(3)
    got = _split(fg, INST)
    fb_ref = 0
    for i, p in enumerate(probs):
        f = f0[i]
        for _ in range(3):
            f = SW.sgs_iteration(p, f)
        fb_ref += p.stats["fallback"]
        err = np.abs(got[i] - f).max() / f.max()
        ref = SW.outer_residual(p, f)
        print(f"  instance {i}: max rel diff {err:.3e}, residual {res[i]:.6e} vs {ref:.6e}", flush=True)
        assert err < SCAN_TOL, i
        assert abs(res[i] - ref) < 1e-9 * ref, i
    visits = 3 * 2 * sum(d["nx"] for d in INST)
    assert st["visits"] == visits
    assert st["inner_iters"] == visits * (1 if mode == "si" else 3)
    assert st["fallbacks"] == fb_ref


@pytest.mark.parametrize("fixed_cycle", [False, True])
def test_vcycle_matches_oracle(bz, fixed_cycle):
    inst = [dict(nx=8, eps=0.05, mass=1.0), dict(nx=8, eps=0.5, T_L=1.2, T_R=1.8, mass=0.8)]
    print(f"1v vcycle fixed={fixed_cycle}", flush=True)
    probs, f0, ctx, slab, fg = _setup(bz, inst, "pfp", 2)
    res, _ = slab.vcycle(2, coarsest=2, nu1=1, nu2=1, coarse_iters=3, tol=0.0, fixed_cycle=fixed_cycle)
    got = _split(fg, inst)
    for i, p in enumerate(probs):
        f = f0[i]
        for _ in range(2):
            f = SW.vcycle(p, f, None, 2, 1, 1, 0.0, coarse_iters=3, fixed=fixed_cycle)
            f = f * (p.mass / SW.total_mass(p, f))
        err = np.abs(got[i] - f).max() / f.max()
        print(f"  instance {i}: max rel diff {err:.3e}", flush=True)
        assert err < 1e-10, i
        assert abs(res[i] - SW.outer_residual(p, f)) < 1e-9 * res[i], i


def test_converged_state_matches_oracle(bz):
    inst = [dict(nx=16, eps=0.1, mass=1.0, xL=-0.5, xR=0.5)]
    probs, f0, ctx, slab, fg = _setup(bz, inst, "pfp", None, bgk_nu=1.0, tol=1e-11)
    for it in range(300):
        res, _ = slab.sweep(1)
        if res[0] < 1e-10:
            break
    print(f"  GPU: {it + 1} iterations, residual {res[0]:.3e}", flush=True)
    assert res[0] < 1e-10
    f_ref, hist = SW.solve_sgs(probs[0], f0[0], tol=1e-10, max_iter=300)
    assert hist[-1] < 1e-10
    got = fg.cpu().numpy()
    assert np.abs(got - f_ref).max() < 1e-8 * f_ref.max()


def test_one_velocity_arguments_are_checked(bz):
    ctx = bz.Context(N=N, L=L, d=1)
    f = torch.ones((4, N), dtype=torch.float64, device="cuda:0")
    with pytest.raises(bz.BZError):
        bz.Slab(ctx, [dict(nx=4, eps=0.1)], f, collision="binary")
    with pytest.raises(bz.BZError):
        bz.Slab(ctx, [dict(nx=4, eps=0.1)], f, collision="bgk", fallback="relax")
    with pytest.raises(bz.BZError):
        bz.Slab(ctx, [dict(nx=4, eps=0.1, bc_L="inflow", rho_L=1.0)], f, collision="bgk")
    slab = bz.Slab(ctx, [dict(nx=4, eps=0.1)], f, collision="bgk")
    with pytest.raises(bz.BZError):
        slab.capture(1)
    with pytest.raises(bz.BZError):
        slab.inflow()
    with pytest.raises(bz.BZError):
        slab.vcycle(1, coarsest=3)  # 4 cells do not halve down to 3
    with pytest.raises(bz.BZError):
        ctx.eval_Q(f)
    with pytest.raises(bz.BZError):
        bz.Context(N=66, L=L, d=1)
