"""GPU parity of the 2D SGS scans (lid-driven cavity, d = 2 velocities) against
the CPU oracle, through the C ABI.  The GPU visits anti-diagonals, the oracle
the lexicographic order: the iterates must agree one to one (fixed inner
iteration counts)."""
import numpy as np
import pytest

from oracle import cavity as CV
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LID = ((1.0, (0.0, 0.0)), (1.5, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.2, (0.5, 0.0)))


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


def _setup(bz, N, L, nx, ny, collision, fixed, mode="pfp", eps=0.1, walls=LID, M=8, nr=4, order=1, limiter="none"):
    sp = Spec(d=2, N=N, L=L, n_phi=M, n_rho=nr)
    prob = CV.Cavity(spec=sp, nx=nx, ny=ny, eps=eps, walls=walls, collision=collision, inner=mode,
                     fixed_inner=fixed, order=order, limiter=limiter)
    f0 = CV.initial_state(prob, T=1.2)
    ctx = bz.Context(N=N, L=L, n_phi=M, n_rho=nr, d=2)
    fg = torch.from_numpy(f0.reshape(nx * ny, -1).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, nx, ny, eps, walls, fg, collision=collision, mode=mode, fixed_iters=fixed or 0, order=order,
                    limiter=limiter)
    return prob, f0, ctx, cav, fg


@pytest.mark.parametrize("collision,mode,N,L,order", [("bgk", "pfp", 8, 4.0, 1), ("binary", "pfp", 8, 4.0, 1),
                                                      ("binary", "fp", 8, 4.0, 1), ("binary", "pfp", 12, 6.0, 1),
                                                      ("bgk", "pfp", 8, 4.0, 2), ("binary", "pfp", 8, 4.0, 2)])
def test_cavity_sweeps_match_oracle(bz, collision, mode, N, L, order):
    nx, ny = 3, 4
    print(f"cavity {collision} {mode} N={N} {nx}x{ny} order {order}", flush=True)
    prob, f0, ctx, cav, fg = _setup(bz, N, L, nx, ny, collision, fixed=2, mode=mode, order=order)
    res, st = cav.sweep(2)
    f = f0
    for _ in range(2):
        f = CV.sgs_iteration(prob, f)
    got = fg.cpu().numpy().reshape(nx, ny, -1)
    err = np.abs(got - f).max() / f.max()
    print(f"max rel diff {err:.3e}, residual {res:.6e} vs {CV.outer_residual(prob, f):.6e}", flush=True)
    assert err < 1e-10
    ref = CV.outer_residual(prob, f)
    assert abs(res - ref) < 1e-9 * ref
    assert st["visits"] == 2 * 4 * nx * ny and st["inner_iters"] == 2 * st["visits"]
    assert abs(CV.total_mass(prob, got) - 1.0) < 1e-13


def test_equilibrium_between_equal_walls_is_kept(bz):
    walls = ((1.0, (0.0, 0.0)),) * 4
    sp = Spec(d=2, N=16, L=8.0, n_phi=8, n_rho=4)
    prob = CV.Cavity(spec=sp, nx=3, ny=3, eps=0.1, walls=walls)
    f0 = CV.initial_state(prob)
    ctx = bz.Context(N=16, L=8.0, n_phi=8, n_rho=4, d=2)
    fg = torch.from_numpy(f0.reshape(9, -1).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, 3, 3, 0.1, walls, fg)
    assert cav.residual() < 1e-11
    res, _ = cav.sweep(1)
    assert np.abs(fg.cpu().numpy() - f0.reshape(9, -1)).max() < 1e-11 * f0.max()
    assert res < 1e-11


def test_cavity_converges_with_tolerance_based_inner_solves(bz):
    prob, f0, ctx, cav, fg = _setup(bz, 12, 6.0, 5, 5, "binary", fixed=None)
    hist = [cav.residual()]
    for _ in range(60):
        r, st = cav.sweep(1)
        hist.append(r)
        if r < 1e-8:
            break
    print("residuals", [f"{h:.2e}" for h in hist[::5]], flush=True)
    assert hist[-1] < 1e-8 < hist[0]
    assert abs(CV.total_mass(prob, fg.cpu().numpy().reshape(5, 5, -1)) - 1.0) < 1e-13


def test_cavity_rejects_bad_arguments(bz):
    ctx = bz.Context(N=8, L=4.0, n_phi=8, n_rho=4, d=2)
    fg = torch.zeros((4, 64), dtype=torch.float64, device="cuda:0")
    with pytest.raises(bz.BZError):  # normal wall velocity
        bz.Cavity(ctx, 2, 2, 0.1, ((1.0, (0.3, 0.0)),) + ((1.0, (0.0, 0.0)),) * 3, fg)
    with pytest.raises(bz.BZError):
        bz.Cavity(ctx, 2, 2, 0.0, ((1.0, (0.0, 0.0)),) * 4, fg)
    ctx3 = bz.Context(N=8, L=4.0, n_theta=2, n_phi=4, n_rho=2)
    f3 = torch.zeros((4, 512), dtype=torch.float64, device="cuda:0")
    with pytest.raises(bz.BZError):
        bz.Cavity(ctx3, 2, 2, 0.1, ((1.0, (0.0, 0.0)),) * 4, f3)


@pytest.mark.parametrize("collision,order", [("bgk", 1), ("binary", 1), ("binary", 2)])
def test_cavity_vcycle_matches_oracle(bz, collision, order):
    # one FAS V-cycle forced to descend (tol = 0) on a 4 x 8 grid: levels 4 x 8 and
    # 2 x 4 (coarsest 2), one pre- and one post-smoothing iteration, at most 3
    # coarsest iterations, then the mass rescale
    nx, ny = 4, 8
    print(f"cavity V-cycle {collision} {nx}x{ny} order {order}", flush=True)
    prob, f0, ctx, cav, fg = _setup(bz, 8, 4.0, nx, ny, collision, fixed=2, order=order)
    res, st = cav.vcycle(1, coarsest=2, nu1=1, nu2=1, coarse_iters=3, tol=0.0)
    f = CV.vcycle(prob, f0.copy(), None, coarsest=2, nu1=1, nu2=1, tol=0.0, coarse_iters=3)
    f = f * (prob.mass / CV.total_mass(prob, f))
    got = fg.cpu().numpy().reshape(nx, ny, -1)
    err = np.abs(got - f).max() / f.max()
    ref = CV.outer_residual(prob, f)
    print(f"max rel diff {err:.3e}, residual {res:.6e} vs {ref:.6e}, visits {st['visits']}", flush=True)
    assert err < 1e-10
    assert abs(res - ref) < 1e-9 * ref
    assert st["visits"] == prob.stats["visits"]


def test_cavity_vcycles_reach_the_sgs_state(bz):
    # MG-SGS-PFP and plain SGS-PFP converge to the same steady state
    nx = 8
    _, f0, ctx, cav, fg = _setup(bz, 8, 4.0, nx, nx, "binary", fixed=None)
    f1 = torch.from_numpy(f0.reshape(nx * nx, -1).copy()).to("cuda:0").contiguous()
    import paper_2409_01910_amd as bzm

    cav_sgs = bzm.Cavity(ctx, nx, nx, 0.1, LID, f1)
    for _ in range(40):
        r_mg, _ = cav.vcycle(1, coarsest=2, tol=1e-10)
        if r_mg < 1e-9:
            break
    for _ in range(80):
        r_sgs, _ = cav_sgs.sweep(1)
        if r_sgs < 1e-9:
            break
    print(f"residuals: MG {r_mg:.2e}, SGS {r_sgs:.2e}", flush=True)
    assert r_mg < 1e-9 and r_sgs < 1e-9
    assert (fg - f1).abs().max().item() < 1e-7 * f1.abs().max().item()
    with pytest.raises(bzm.BZError):  # 8 -> 4 -> 2 -> 1 would have to halve 1
        cav.vcycle(1, coarsest=0)


@pytest.mark.parametrize("collision,order", [("bgk", 1), ("binary", 1), ("binary", 2)])
def test_plates_uniform_in_y_match_oracle(bz, collision, order):
    # the slab between two plates with 2D velocities (one cell row, no y
    # transport): two SGS iterations, then one V-cycle forced to descend
    nx = 8
    walls = ((1.0, (0.0, 0.0)), (2.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)))
    print(f"plates {collision} order {order}", flush=True)
    sp = Spec(d=2, N=8, L=4.0, n_phi=8, n_rho=4)
    prob = CV.Cavity(spec=sp, nx=nx, ny=1, eps=0.1, walls=walls, collision=collision, fixed_inner=2, order=order,
                     uniform_y=True)
    f0 = CV.initial_state(prob, T=1.2)
    ctx = bz.Context(N=8, L=4.0, n_phi=8, n_rho=4, d=2)
    fg = torch.from_numpy(f0.reshape(nx, -1).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, nx, 1, 0.1, walls, fg, collision=collision, fixed_iters=2, order=order, uniform_y=True)
    res, st = cav.sweep(2)
    f = CV.sgs_iteration(prob, CV.sgs_iteration(prob, f0))
    err = np.abs(fg.cpu().numpy().reshape(nx, 1, -1) - f).max() / f.max()
    print(f"sweeps: max rel diff {err:.3e}", flush=True)
    assert err < 1e-10
    assert abs(res - CV.outer_residual(prob, f)) < 1e-9 * res
    assert st["visits"] == 2 * 2 * nx
    res, _ = cav.vcycle(1, coarsest=2, nu1=1, nu2=1, coarse_iters=3, tol=0.0)
    f = CV.vcycle(prob, f, None, coarsest=2, nu1=1, nu2=1, tol=0.0, coarse_iters=3)
    f = f * (prob.mass / CV.total_mass(prob, f))
    err = np.abs(fg.cpu().numpy().reshape(nx, 1, -1) - f).max() / f.max()
    print(f"V-cycle: max rel diff {err:.3e}", flush=True)
    assert err < 1e-10


def test_cavity_with_the_carleman_form_matches_oracle(bz):
    # the 2D scans with the Carleman form of the collision term (Maxwell molecules)
    nx, ny = 3, 4
    sp = Spec(d=2, N=8, L=4.0, n_phi=8, n_rho=4)
    prob = CV.Cavity(spec=sp, nx=nx, ny=ny, eps=0.1, walls=LID, collision="binary", q_method="carleman",
                     fixed_inner=2)
    f0 = CV.initial_state(prob, T=1.2)
    ctx = bz.Context(N=8, L=4.0, n_phi=8, n_rho=4, d=2, method=bz.BZ_METHOD_CARLEMAN)
    fg = torch.from_numpy(f0.reshape(nx * ny, -1).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, nx, ny, 0.1, LID, fg, fixed_iters=2)
    res, _ = cav.sweep(1)
    f = CV.sgs_iteration(prob, f0)
    ref = CV.outer_residual(prob, f)
    err = np.abs(fg.cpu().numpy().reshape(nx, ny, -1) - f).max() / f.max()
    print(f"Carleman cavity: max rel diff {err:.3e}", flush=True)
    assert err < 1e-10
    assert abs(res - ref) < 1e-9 * ref


def test_cavity_relaxed_step1_fallback_matches_oracle(bz):
    # one cell starts as a dense ring |v| = 2 in a cavity at rest: its first visit
    # violates eq. existence; with the relaxed step 1 it stays preconditioned
    from oracle.grid import velocity_nodes

    nx, ny = 3, 4
    sp = Spec(d=2, N=12, L=5.0, n_phi=8, n_rho=4)
    prob = CV.Cavity(spec=sp, nx=nx, ny=ny, eps=0.01, walls=LID, collision="bgk", fixed_inner=3, fallback="relax")
    f0 = CV.initial_state(prob, T=1.0)
    sv = np.sqrt((velocity_nodes(sp) ** 2).sum(1))
    ring = np.exp(-(sv - 2.0) ** 2 / 0.1)
    f0[1, 1] = 20.0 * ring * f0[0, 0].sum() / ring.sum()
    f0 *= 1.0 / CV.total_mass(prob, f0)
    ctx = bz.Context(N=12, L=5.0, n_phi=8, n_rho=4, d=2)
    fg = torch.from_numpy(f0.reshape(nx * ny, -1).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, nx, ny, 0.01, LID, fg, collision="bgk", fixed_iters=3, fallback="relax")
    _, st = cav.sweep(1)
    f = CV.sgs_iteration(prob, f0)
    err = np.abs(fg.cpu().numpy().reshape(nx, ny, -1) - f).max() / f.max()
    print(f"relaxed cavity: rel diff {err:.3e}, oracle relaxed {prob.stats['relaxed']}, fallbacks {st['fallbacks']}",
          flush=True)
    assert prob.stats["relaxed"] >= 1 and st["fallbacks"] == 0 == prob.stats["fallback"]
    assert err < 1e-10


def test_cavity_minmod_limited_second_order_matches_oracle(bz):
    nx, ny = 4, 5
    prob, f0, ctx, cav, fg = _setup(bz, 8, 4.0, nx, ny, "binary", fixed=2, order=2, limiter="minmod")
    res, _ = cav.sweep(2)
    f = CV.sgs_iteration(prob, CV.sgs_iteration(prob, f0))
    err = np.abs(fg.cpu().numpy().reshape(nx, ny, -1) - f).max() / f.max()
    print(f"minmod cavity: max rel diff {err:.3e}", flush=True)
    assert err < 1e-10
    assert abs(res - CV.outer_residual(prob, f)) < 1e-9 * res
