"""Pins of the oracle with one velocity dimension (the 1D1V BGK model of
Section 4.1; CPU only): the discrete Maxwellian on the 50-node grid, the BGK
frequency |S^0| rho = 2 rho, the collisionless slab against its closed form
(half-range wall Maxwellians with the discrete zero-mass-flux balance), and
SGS-FP and SGS-PFP reaching the same iterates when the inner solves are tight."""
import numpy as np

from oracle import collision as OQ, sweep as SW
from oracle.grid import Spec, velocity_nodes
from oracle.maxwellian import discrete_maxwellian, gaussian, moments


def _spec():
    return Spec(d=1, N=50, L=6.0)


def test_grid_and_discrete_maxwellian():
    sp = _spec()
    v = velocity_nodes(sp)[:, 0]
    assert sp.K == 50 and abs(sp.w - 12.0 / 50) < 1e-15 and v[0] == -24 * sp.w and v[-1] == 25 * sp.w
    f = 0.7 * np.exp(-(v - 0.4) ** 2 / 1.6) + 0.3 * np.exp(-(v + 1.0) ** 2 / 0.5)
    M, th = discrete_maxwellian(sp, f, return_theta=True)
    assert np.abs(moments(sp, M) - moments(sp, f)).max() < 1e-13 * moments(sp, f).max()
    assert np.abs(discrete_maxwellian(sp, M) - M).max() < 1e-13 * M.max()
    # a discrete Gaussian is its own Maxwellian, with its own parameters
    th0 = np.array([-0.3, 0.5, 0.35])
    G = gaussian(sp, th0)
    _, th1 = discrete_maxwellian(sp, G, return_theta=True)
    assert np.abs(th1 - th0).max() < 1e-11


def test_bgk_frequency_is_two_rho():
    sp = _spec()
    v = velocity_nodes(sp)[:, 0]
    f = np.exp(-v * v / 2.0)
    rho = sp.w * f.sum()
    assert abs(OQ.bgk_nu_of(sp, f) - 2.0 * rho) < 1e-15 * rho


def test_collisionless_slab_is_the_half_range_wall_state():
    sp = _spec()
    v = velocity_nodes(sp)[:, 0]
    prob = SW.Slab(spec=sp, nx=6, eps=1e14, T_L=1.0, T_R=2.0, mass=1.0, collision="bgk", bgk_nu=1.0,
                   tol_inner=1e-13)
    f, hist = SW.solve_sgs(prob, SW.initial_state(prob, T=1.5), tol=1e-12, max_iter=50)
    assert hist[-1] < 1e-12
    ML = np.exp(-v * v / 2.0) / np.sqrt(2.0 * np.pi)
    MR = np.exp(-v * v / 4.0) / np.sqrt(4.0 * np.pi)
    # f = a ML for v > 0 and b MR for v < 0 in every cell, with zero discrete
    # mass flux and total mass 1; the v = 0 node, which transport leaves to the
    # collisions, is not part of the closed form
    a_over_b = np.sum(np.where(v < 0, -v * MR, 0.0)) / np.sum(np.where(v > 0, v * ML, 0.0))
    pos, neg = v > 0, v < 0
    a = f[:, pos] / ML[pos]
    b = f[:, neg] / MR[neg]
    assert np.abs(a - a.mean()).max() < 1e-10 * a.mean() and np.abs(b - b.mean()).max() < 1e-10 * b.mean()
    assert abs(a.mean() / b.mean() - a_over_b) < 1e-10 * a_over_b
    assert abs(SW.total_mass(prob, f) - 1.0) < 1e-13


def test_fp_and_pfp_iterates_coincide_with_tight_inner_solves():
    sp = _spec()
    out = []
    for inner in ("fp", "pfp"):
        prob = SW.Slab(spec=sp, nx=4, xL=-0.5, xR=0.5, eps=0.3, collision="bgk", bgk_nu=1.0, inner=inner,
                       tol_inner=1e-13, max_inner=2000)
        f = SW.initial_state(prob, T=1.5)
        for _ in range(3):
            f = SW.sgs_iteration(prob, f)
        out.append(f)
    assert np.abs(out[0] - out[1]).max() < 1e-11 * out[1].max()
