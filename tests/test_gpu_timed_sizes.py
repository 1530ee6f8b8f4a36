"""GPU parity at the velocity grids the benchmarks time, against the FP64 oracle
through the C ABI: the cell update at 16^3 and 32^3 (where the final pass of
the visit runs plane by plane), fallback cells included; the 1D scans at 16^3
and 32^3 (first and second order, inflow on a shifted grid); the 2D visits at
32^2 and 48^2 (every thread slot of the visit kernel live).  Small sphere and
radial rules keep the oracle fast; the cell update and the scans do not depend
on the rule's size beyond the collision term, whose full-rule parity is
covered at 32^3 by the collision tests.

Bounds, relative to the field's maximum:
  * a cell update after a fixed number of updates: 1e-12;
  * the cell update behind the collision term (Q, the penalty split, then the
    solve): 2e-12;
  * a scan (each visit's result feeds the next visit's right-hand side): 1e-11.
Every update ends in Newton solves for Maxwellian parameters that the library
stops at a moment residual of 1e-13 relative (the oracle at 1e-14), so the two
sides carry parameters that differ by up to that much, and a scan compounds it
over its visits (measured: up to 7e-12 on the shifted grid with the
conservation projection at 32^3).  Residuals agree to 1e-9 relative (a norm of
a difference of nearly equal terms)."""
import numpy as np
import pytest

import synth
from oracle import cell as OC, collision as OQ, sweep as SW, cavity as CV
from oracle.grid import Spec, velocity_nodes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ITER_TOL = 1e-12
COMP_TOL = 2e-12
SCAN_TOL = 1e-11
RES_TOL = 1e-9


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


def _T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _transport(sp, fl, fr, dx):
    v1 = velocity_nodes(sp)[:, 0]
    return (-np.maximum(v1, 0) * fl + np.minimum(v1, 0) * fr) / dx


# (N, L, dx, cells)
CELL_SIZES = [(16, 8.0, 1 / 32, 6), (32, 8.0, 1 / 32, 4)]


@pytest.mark.parametrize("size", CELL_SIZES)
@pytest.mark.parametrize("mode", ["pfp", "fp"])
def test_cell_solve_fixed_iterations_at_timed_sizes(bz, size, mode):
    N, L, dx, B = size
    print(f"cell_solve N={N} B={B} {mode}", flush=True)
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    fo, fl, fr, eps = synth.cell_inflow_batch(B, N, L, dx, seed=51)
    r = _transport(sp, fl, fr, dx)
    nu = np.array([OQ.nu_of(sp, fo[i]) for i in range(B)])
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    for n_it in (1, 3):
        g, st = ctx.cell_solve(_T(r), _T(nu), _T(eps), dx, _T(fo), mode=mode, fixed_iters=n_it)
        g = g.cpu().numpy()
        stats = ctx.decode_stats(st)
        worst = 0.0
        for i in range(B):
            go, so = OC.solve(sp, r[i], nu[i], eps[i], dx, fo[i], mode=mode, fixed_iters=n_it)
            err = np.max(np.abs(g[i] - go)) / np.abs(go).max()
            worst = max(worst, err)
            assert err < ITER_TOL, (i, n_it, err)
            assert stats["iterations"][i] == n_it
            if mode == "pfp":  # the plain mode reports every visit as the plain iteration
                assert bool(stats["fallback"][i]) == bool(so.fallback), i
            assert abs(stats["residual"][i] - so.residual) <= RES_TOL * so.residual + 1e-13 * (nu[i] / eps[i]) * \
                np.abs(go).max() * np.sqrt(sp.w * sp.K), i
        print(f"  {n_it} updates: max rel diff {worst:.3e}", flush=True)


@pytest.mark.parametrize("size", CELL_SIZES)
def test_cell_solve_reaches_the_theta_fixed_point_at_timed_sizes(bz, size):
    # the inner tolerance (absolute L2, Section 4) bounds the distance to the fixed
    # point by about tol / min(D) in the same norm, far below the bound used here
    N, L, dx, B = size
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    fo, fl, fr, eps = synth.cell_inflow_batch(B, N, L, dx, seed=52)
    r = _transport(sp, fl, fr, dx)
    nu = np.array([OQ.nu_of(sp, fo[i]) for i in range(B)])
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    g, st = ctx.cell_solve(_T(r), _T(nu), _T(eps), dx, _T(fo), mode="pfp", tol=1e-10, max_iter=200)
    g = g.cpu().numpy()
    stats = ctx.decode_stats(st)
    for i in range(B):
        gs, _ = OC.theta_solve(sp, r[i], nu[i], eps[i], dx)
        assert stats["status"][i] == 0
        err = np.max(np.abs(g[i] - gs)) / np.abs(gs).max()
        print(f"N={N} cell {i}: {stats['iterations'][i]} updates, rel diff to the fixed point {err:.3e}", flush=True)
        assert err < 1e-8


@pytest.mark.parametrize("N", [16, 32])
def test_fallback_visits_match_oracle_at_timed_sizes(bz, N):
    # a two-beam initial guess violates eq. existence at the first update: both
    # sides fall back to the plain iteration there, and the iterates after 1, 2
    # and 3 updates agree one to one (fallback flag included)
    L, dx, eps = 8.0, 1 / 32, 0.05
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    fo, fl, fr, _ = synth.cell_inflow_batch(1, N, L, dx, seed=53)
    r = _transport(sp, fl[0], fr[0], dx)
    nu = OQ.nu_of(sp, fo[0])
    g0 = synth.maxwellian_mixture([(5.0, np.array([2.5, 0, 0]), 0.3), (5.0, np.array([-2.5, 0, 0]), 0.3)], N, L)
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    for n_it in (1, 2, 3):
        g, st = ctx.cell_solve(_T(r[None]), _T(np.array([nu])), _T(np.array([eps])), dx, _T(g0[None]),
                               mode="pfp", fixed_iters=n_it)
        s = bz.Context.decode_stats(st)[0]
        go, so = OC.solve(sp, r, nu, eps, dx, g0, mode="pfp", fixed_iters=n_it)
        err = np.abs(g.cpu().numpy()[0] - go).max() / np.abs(go).max()
        print(f"N={N} fallback visit, {n_it} updates: flag {s['fallback']} vs {so.fallback}, rel diff {err:.3e}",
              flush=True)
        assert s["fallback"] == 1 and so.fallback
        assert err < ITER_TOL


@pytest.mark.parametrize("N,B", [(16, 5), (32, 3)])
def test_cell_fixed_point_composition_at_timed_sizes(bz, N, B):
    # Q (mass-projected corrected form), P = Q - nu (M - f), r = inflow - P / eps,
    # then the preconditioned solve from f_old; every cell compared, fallback
    # flags included
    L, dx = 8.0, 1 / 16
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    print(f"cell_fixed_point N={N} B={B}", flush=True)
    fo, fl, fr, eps = synth.cell_inflow_batch(B, N, L, dx, seed=54)
    inflow = _transport(sp, fl, fr, dx)
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=2)
    for n_it in (1, 3):
        g, st = ctx.cell_fixed_point(_T(fo), _T(inflow), _T(eps), dx, fixed_iters=n_it)
        g = g.cpu().numpy()
        stats = ctx.decode_stats(st)
        worst = 0.0
        for i in range(B):
            r = inflow[i] - OQ.penalty(sp, fo[i]) / eps[i]
            go, so = OC.solve(sp, r, OQ.nu_of(sp, fo[i]), eps[i], dx, fo[i], mode="pfp", fixed_iters=n_it)
            assert bool(stats["fallback"][i]) == bool(so.fallback), i
            err = np.max(np.abs(g[i] - go)) / np.abs(go).max()
            worst = max(worst, err)
            assert err < COMP_TOL, (i, n_it, err)
        print(f"  {n_it} updates: max rel diff {worst:.3e}", flush=True)


def _slab_setup(bz, N, L, inst, collision, fixed, order=1, shift=0.0, init="uniform"):
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=2, v1_shift=shift)
    probs, f0 = [], []
    for d in inst:
        coll = "binary" if collision == "binary_conserve" else collision
        p = SW.Slab(spec=sp, nx=d["nx"], xL=d.get("xL", 0.0), xR=d.get("xR", 1.0), T_L=d.get("T_L", 1.0),
                    T_R=d.get("T_R", 2.0), U_L=d.get("U_L", (0.0, 0.0, 0.0)), U_R=d.get("U_R", (0.0, 0.0, 0.0)),
                    eps=d["eps"], collision=coll, conserve="all" if collision == "binary_conserve" else "mass",
                    fixed_inner=fixed or None, order=order, bc_L=d.get("bc_L", "wall"), bc_R=d.get("bc_R", "wall"),
                    rho_L=d.get("rho_L", 1.0), rho_R=d.get("rho_R", 1.0))
        if init == "step":
            ML = SW.wall_maxwellian(sp, d["T_L"], d.get("U_L", (0.0, 0.0, 0.0))) * d.get("rho_L", 1.0)
            MR = SW.wall_maxwellian(sp, d["T_R"], d.get("U_R", (0.0, 0.0, 0.0))) * d.get("rho_R", 1.0)
            f = np.stack([ML if j < d["nx"] // 2 else MR for j in range(d["nx"])])
            p.mass = SW.total_mass(p, f)
            d["mass"] = p.mass
        else:
            f = SW.initial_state(p, T=1.5)
            p.mass = d.get("mass", 1.0)
        probs.append(p)
        f0.append(f)
    ctx = bz.Context(N=N, L=L, n_theta=2, n_phi=4, n_rho=2, v1_shift=shift)
    fg = torch.from_numpy(np.concatenate(f0)).to("cuda:0").contiguous()
    slab = bz.Slab(ctx, inst, fg, collision=collision, fixed_iters=fixed, order=order)
    return probs, f0, ctx, slab, fg


def _split(fg, inst):
    out, o = [], 0
    a = fg.cpu().numpy()
    for d in inst:
        out.append(a[o:o + d["nx"]])
        o += d["nx"]
    return out


def _check_slab(probs, f0, slab, fg, inst, n_iters=1):
    res, st = slab.sweep(n_iters)
    got = _split(fg, inst)
    for i in range(len(inst)):
        f = f0[i]
        for _ in range(n_iters):
            f = SW.sgs_iteration(probs[i], f)
        err = np.max(np.abs(got[i] - f)) / f.max()
        ref = SW.outer_residual(probs[i], f)
        print(f"  instance {i}: max rel diff {err:.3e}, residual {res[i]:.6e} vs {ref:.6e}", flush=True)
        assert err < SCAN_TOL, (i, err)
        assert abs(res[i] - ref) < RES_TOL * ref, i
    return st


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("order", [1, 2])
def test_binary_sgs_sweeps_at_timed_sizes(bz, N, order):
    # ragged instances: interior, two-cell and one-cell slabs
    inst = [dict(nx=4, eps=0.1, mass=1.0), dict(nx=2, eps=0.5, T_L=1.2, T_R=1.6, mass=0.9),
            dict(nx=1, eps=0.05, mass=1.1)]
    print(f"binary sgs N={N} order {order}", flush=True)
    probs, f0, ctx, slab, fg = _slab_setup(bz, N, 8.0, inst, "binary", fixed=3, order=order)
    st = _check_slab(probs, f0, slab, fg, inst)
    assert st["visits"] == 2 * 7 and st["inner_iters"] == 3 * st["visits"]


@pytest.mark.parametrize("N", [16, 32])
def test_inflow_sweeps_on_a_shifted_grid_at_timed_sizes(bz, N):
    inst = [dict(nx=4, eps=0.1, xL=-1.0, xR=1.0, bc_L="inflow", bc_R="inflow", rho_L=1.0, rho_R=1.6,
                 T_L=1.0, T_R=1.4, U_L=(1.5, 0.0, 0.0), U_R=(0.9, 0.0, 0.0))]
    print(f"inflow sgs N={N}", flush=True)
    probs, f0, ctx, slab, fg = _slab_setup(bz, N, 8.0, inst, "binary_conserve", fixed=3, shift=1.25, init="step")
    _check_slab(probs, f0, slab, fg, inst)


@pytest.mark.parametrize("N", [16, 32])
def test_tolerance_based_sweep_at_timed_sizes(bz, N):
    # inner solves stopped by the tolerance of Section 4 (1e-8): the number of
    # updates per visit is decided by a residual compared with a tolerance, so
    # the iterates agree to the tolerance, not to rounding
    inst = [dict(nx=4, eps=0.1, mass=1.0)]
    print(f"tolerance sgs N={N}", flush=True)
    probs, f0, ctx, slab, fg = _slab_setup(bz, N, 8.0, inst, "binary", fixed=0)
    res, st = slab.sweep(1)
    f = SW.sgs_iteration(probs[0], f0[0])
    got = _split(fg, inst)[0]
    err = np.max(np.abs(got - f)) / f.max()
    print(f"  max rel diff {err:.3e}; {st['inner_iters']} updates in {st['visits']} visits vs "
          f"{probs[0].stats['inner']} in {probs[0].stats['visits']}", flush=True)
    assert err < 1e-9
    assert st["inner_iters"] == probs[0].stats["inner"]


LID = ((1.0, (0.0, 0.0)), (1.5, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.2, (0.5, 0.0)))


@pytest.mark.parametrize("N,mode,method", [(32, "pfp", "sigma"), (48, "pfp", "sigma"), (48, "fp", "sigma"),
                                           (48, "pfp", "carleman")])
def test_cavity_visits_at_timed_sizes(bz, N, mode, method):
    # 3 x 3 cells: the middle anti-diagonals hold several cells; at 32^2 the visit
    # kernel's 4 x 256 point slots are all live, at 48^2 its 9 x 256
    nx = ny = 3
    L = 8.0
    print(f"cavity N={N} {mode} {method}", flush=True)
    sp = Spec(d=2, N=N, L=L, n_phi=8, n_rho=4)
    prob = CV.Cavity(spec=sp, nx=nx, ny=ny, eps=0.1, walls=LID, collision="binary", inner=mode, fixed_inner=2,
                     q_method=method)
    f0 = CV.initial_state(prob, T=1.2)
    ctx = bz.Context(N=N, L=L, n_phi=8, n_rho=4, d=2,
                     method=bz.BZ_METHOD_CARLEMAN if method == "carleman" else bz.BZ_METHOD_SIGMA)
    fg = torch.from_numpy(f0.reshape(nx * ny, -1).copy()).to("cuda:0").contiguous()
    cav = bz.Cavity(ctx, nx, ny, 0.1, LID, fg, mode=mode, fixed_iters=2)
    res, st = cav.sweep(1)
    f = CV.sgs_iteration(prob, f0)
    ref = CV.outer_residual(prob, f)
    err = np.abs(fg.cpu().numpy().reshape(nx, ny, -1) - f).max() / f.max()
    print(f"  max rel diff {err:.3e}, residual {res:.6e} vs {ref:.6e}", flush=True)
    assert err < ITER_TOL
    assert abs(res - ref) < RES_TOL * ref
    assert st["visits"] == 4 * nx * ny and st["inner_iters"] == 2 * st["visits"]
