"""Pins of the oracle's two-dimensional SGS scans (the lid-driven cavity; CPU
only): an exact equilibrium, the x <-> y transposition symmetry of the steady
state, which wall is which (hot wall, lid direction), and the mass rescale."""
import numpy as np
import pytest

from oracle import cavity as CV
from oracle.grid import Spec, velocity_nodes
from oracle.maxwellian import macroscopic


@pytest.mark.parametrize("collision", ["bgk", "binary"])
def test_uniform_maxwellian_between_equal_walls_is_a_steady_state(collision):
    # all walls at T = 1 at rest: the uniform unit-temperature Maxwellian is an
    # exact discrete steady state (Q vanishes by eq. discrete_Q, the wall
    # densities balance the outgoing fluxes); L = 8 keeps the one unpaired grid
    # node's Maxwellian value (v = L) below rounding
    sp = Spec(d=2, N=16, L=8.0, n_phi=8, n_rho=4)
    prob = CV.Cavity(spec=sp, nx=3, ny=3, eps=0.1, walls=((1.0, (0.0, 0.0)),) * 4, collision=collision)
    f0 = CV.initial_state(prob)
    assert CV.outer_residual(prob, f0) < 1e-11
    f1 = CV.sgs_iteration(prob, f0)
    assert np.abs(f1 - f0).max() < 1e-11 * f0.max()


def _converge(prob, tol=1e-11, max_iter=100):
    f = CV.initial_state(prob)
    for it in range(max_iter):
        f = CV.sgs_iteration(prob, f)
        if it % 5 == 4 and CV.outer_residual(prob, f) < tol:
            return f
    raise AssertionError("no convergence")


@pytest.mark.parametrize("order,limiter", [(1, "none"), (2, "none"), (2, "minmod")])
def test_steady_state_is_symmetric_under_transposition(order, limiter):
    # walls x = 0 and y = 0 at T = 1, x = 1 and y = 1 at T = 2: the problem is
    # invariant under (x, y, v_1, v_2) -> (y, x, v_2, v_1), the scans are not, so
    # only the converged state must be symmetric (and the scans' fixed point must
    # zero the residual of the same scheme)
    N = 8
    sp = Spec(d=2, N=N, L=4.0, n_phi=8, n_rho=4)
    walls = ((1.0, (0.0, 0.0)), (2.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (2.0, (0.0, 0.0)))
    prob = CV.Cavity(spec=sp, nx=4, ny=4, eps=0.1, walls=walls, collision="bgk", order=order, limiter=limiter)
    f = _converge(prob).reshape(4, 4, N, N)
    assert np.abs(f.transpose(1, 0, 3, 2) - f).max() < 1e-11 * f.max()
    assert abs(CV.total_mass(prob, f.reshape(4, 4, -1)) - 1.0) < 1e-13


def test_hot_wall_and_lid_direction():
    # left wall T = 1, right wall T = 2, bottom and top at T = 1.5, lid (y = 1)
    # moving in +x: the gas is hotter next to the right wall than next to the
    # left one, and the lid drives a clockwise vortex (U_1 > 0 under the lid,
    # < 0 along the bottom)
    N = 12
    sp = Spec(d=2, N=N, L=6.0, n_phi=8, n_rho=4)
    walls = ((1.0, (0.0, 0.0)), (2.0, (0.0, 0.0)), (1.5, (0.0, 0.0)), (1.5, (0.5, 0.0)))
    prob = CV.Cavity(spec=sp, nx=4, ny=4, eps=0.1, walls=walls, collision="bgk")
    f = _converge(prob, tol=1e-8)
    mac = [[macroscopic(sp, f[i, j]) for j in range(4)] for i in range(4)]
    T = np.array([[m[2] for m in row] for row in mac])
    U1 = np.array([[m[1][0] for m in row] for row in mac])
    assert (T[-1, :] > T[0, :]).all()
    assert (U1[:, -1] > 0).all() and (U1[:, 0] < 0).all()


def test_converged_state_is_a_fixed_point_of_the_vcycle():
    # FAS consistency (eq. coarse): at a converged fine state the coarse problem
    # R_H(f_H) = R_H(restrict f) + restrict(b - R_h f) is solved by restrict f
    # itself, so a V-cycle forced to descend (tol = 0) changes nothing beyond the
    # residual it starts from; a wrong coarse right-hand side would move f
    N = 8
    sp = Spec(d=2, N=N, L=4.0, n_phi=8, n_rho=4)
    walls = ((1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.5, 0.0)))
    prob = CV.Cavity(spec=sp, nx=4, ny=4, eps=0.1, walls=walls, collision="bgk")
    f = _converge(prob, tol=1e-12)
    g = CV.vcycle(prob, f.copy(), None, coarsest=2, nu1=0, nu2=0, tol=0.0)
    assert np.abs(g - f).max() < 1e-9 * f.max()
    # and from a perturbed state the V-cycle reduces the residual
    f1 = CV.sgs_iteration(prob, CV.initial_state(prob))
    r1 = CV.outer_residual(prob, f1)
    f2 = CV.mg_iteration(prob, f1, coarsest=2)
    assert CV.outer_residual(prob, f2) < 0.5 * r1


def test_second_order_transport_is_exact_on_quadratic_profiles_2d():
    # eqs. reconstruction and slope along both axes: for f = 1 + q(x, y) g(v) with
    # q quadratic (cross term included), the upwind flux differences with the
    # centred slopes equal v . grad q g exactly at interior cells; first order
    # is off by O(dx)
    sp = Spec(d=2, N=8, L=4.0, n_phi=8, n_rho=4)
    v = velocity_nodes(sp)
    g = np.exp(-0.3 * (v * v).sum(1))
    cx, cy, cxy = 0.7, -0.4, 0.5
    for order, exact in ((2, True), (1, False)):
        prob = CV.Cavity(spec=sp, nx=8, ny=7, eps=1.0, collision="bgk", order=order)
        x = (np.arange(prob.nx) + 0.5) * prob.dx
        y = (np.arange(prob.ny) + 0.5) * prob.dy
        X, Y = np.meshgrid(x, y, indexing="ij")
        q = cx * X * X + cy * Y * Y + cxy * X * Y
        f = 1.0 + q[:, :, None] * g[None, None, :]
        R = CV.residual_field(prob, f, np.zeros_like(f))
        qx, qy = 2 * cx * X + cxy * Y, 2 * cy * Y + cxy * X
        ref = (v[None, None, :, 0] * qx[:, :, None] + v[None, None, :, 1] * qy[:, :, None]) * g[None, None, :]
        err = np.abs(R[2:-2, 2:-2] - ref[2:-2, 2:-2]).max() / np.abs(ref).max()
        assert (err < 1e-12) if exact else (err > 1e-3), (order, err)


@pytest.mark.parametrize("collision,order", [("bgk", 1), ("binary", 1), ("binary", 2)])
def test_uniform_y_cavity_is_the_1d_slab(collision, order):
    # A cavity that does not vary along y (one cell row, no y transport, no y
    # walls, two scans per iteration) is the heat slab between two plates: its
    # SGS iterations and V-cycles must be those of the independently written 1D
    # slab oracle (pinned by its own closed forms) on the same 2D velocity grid.
    from oracle import sweep as SW

    sp = Spec(d=2, N=8, L=4.0, n_phi=8, n_rho=4)
    walls = ((1.0, (0.0, 0.0)), (2.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)))
    cav = CV.Cavity(spec=sp, nx=8, ny=1, eps=0.1, walls=walls, collision=collision, uniform_y=True, order=order,
                    fixed_inner=2)
    slab = SW.Slab(spec=sp, nx=8, eps=0.1, T_L=1.0, T_R=2.0, U_L=(0.0, 0.0), U_R=(0.0, 0.0), collision=collision,
                   order=order, fixed_inner=2)
    f = CV.initial_state(cav, T=1.2)
    g = f[:, 0, :].copy()
    f = CV.sgs_iteration(cav, f)
    g = SW.sgs_iteration(slab, g)
    assert np.abs(f[:, 0, :] - g).max() <= 1e-14 * g.max()
    f = CV.vcycle(cav, f, None, coarsest=2, nu1=1, nu2=1, tol=0.0)
    g = SW.vcycle(slab, g, None, coarsest=2, nu1=1, nu2=1, tol=0.0)
    assert np.abs(f[:, 0, :] - g).max() <= 1e-14 * g.max()
    assert abs(CV.outer_residual(cav, f) - SW.outer_residual(slab, g)) <= 1e-14 * SW.outer_residual(slab, g)
