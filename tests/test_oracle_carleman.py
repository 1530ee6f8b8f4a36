"""Pins of the oracle's Carleman fast form for hard spheres (CPU only).

Each test checks the oracle against something other than itself: the
hard-sphere collision frequency of a Maxwellian in closed form, exact mass
conservation, exact grid symmetries, numerical quadrature of the two weight
functions, and the sigma form of the same operator."""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erf, j0

import synth
from oracle import carleman as CA, collision as C
from oracle.grid import Spec, velocity_nodes


def _hs(N, L=8.0, nt=4, nph=8, nr=8):
    return Spec(d=3, N=N, L=L, gamma=1.0, n_theta=nt, n_phi=nph, n_rho=nr)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_weight_functions_match_numerical_quadrature():
    sp = _hs(16)
    Rc = CA.carleman_radius(sp)
    # psi1(s) = 2 int_0^Rc rho cos(rho s) drho, across the series / closed-form switch
    for s in (0.0, 1e-7, 0.05, 0.5 / Rc * 0.999, 0.5 / Rc * 1.001, 0.4, 2.3, 7.9):
        ref = 2.0 * quad(lambda r: r * np.cos(r * s), 0.0, Rc, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        assert abs(CA.psi1(sp, s) - ref) <= 1e-12 * Rc * Rc, s
    # Phi2(t) = 2 pi int_0^Rc r J0(r t) dr
    for t in (0.0, 1e-9, 0.3, 1.7, 6.2):
        ref = 2.0 * np.pi * quad(lambda r: r * j0(r * t), 0.0, Rc, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        assert abs(CA.phi2(sp, t) - ref) <= 1e-12 * Rc * Rc, t


def test_hard_sphere_maxwellian_matches_closed_form():
    # For a Maxwellian the gain and loss terms both equal 4 pi M(v) nu(v), with
    # nu(v) = int |v - w| M(w) dw = rho sqrt(2T) (exp(-c^2)/sqrt(pi) + (c + 1/(2c)) erf(c)),
    # c = |v| / sqrt(2T): the mean relative speed, a closed form independent of
    # any spectral weight.  This fixes the Carleman constant 4 and both weights.
    # At T = 0.4 the truncation of x and y at sqrt(2) R drops a negligible part
    # of the collisions and 40^3 resolves the Gaussian.
    sp = _hs(40, nt=8, nph=16)
    v = velocity_nodes(sp)
    T = 0.4
    M = (2 * np.pi * T) ** -1.5 * np.exp(-(v * v).sum(1) / (2 * T))
    gain, loss = CA.q_carleman(sp, M, parts=True)
    c = np.sqrt((v * v).sum(1) / (2 * T))
    cs = np.maximum(c, 1e-300)
    nu = np.sqrt(2 * T) * (np.exp(-c * c) / np.sqrt(np.pi) + np.where(c > 0, (c + 0.5 / cs) * erf(c), 0.0))
    nu[c == 0] = np.sqrt(8 * T / np.pi)
    ref = 4 * np.pi * M * nu
    assert np.abs(gain - ref).max() < 1e-5 * ref.max()
    assert np.abs(loss - ref).max() < 1e-5 * ref.max()


def test_plain_form_conserves_mass_exactly():
    sp = _hs(16)
    f = synth.mixture_batch(1, 16, 8.0, seed=11)[0]
    gain, loss = CA.q_carleman(sp, f, parts=True)
    assert abs(np.sum(gain - loss)) < 1e-13 * np.sum(np.abs(gain))


def test_symmetries_reflection_swap_translation():
    sp = _hs(8, L=4.0)
    f = synth.mixture_batch(1, 8, 4.0, seed=7, T=(0.3, 0.5), speed=(0.0, 0.3))[0].reshape(8, 8, 8)
    Q = CA.q_carleman(sp, f.reshape(-1)).reshape(8, 8, 8)
    tol = 1e-13 * np.abs(Q).max()
    # the half-sphere rule is mapped onto itself (up to e -> -e) by swapping the
    # azimuthal axes (n_phi % 4 == 0) and by reflecting the polar axis
    Qs = CA.q_carleman(sp, f.transpose(0, 2, 1).reshape(-1)).reshape(8, 8, 8)
    assert np.abs(Qs - Q.transpose(0, 2, 1)).max() < tol
    ref = (8 - 2 - np.arange(8)) % 8
    Qr = CA.q_carleman(sp, f[ref].reshape(-1)).reshape(8, 8, 8)
    assert np.abs(Qr - Q[ref]).max() < tol
    Qt = CA.q_carleman(sp, np.roll(f, 1, axis=1).reshape(-1)).reshape(8, 8, 8)
    assert np.abs(Qt - np.roll(Q, 1, axis=1)).max() < tol


def test_direction_rule_converges_and_agrees_with_the_sigma_form():
    f = synth.mixture_batch(1, 16, 8.0, seed=5)[0]
    q32 = CA.q_carleman(_hs(16, nt=4, nph=8), f)
    q128 = CA.q_carleman(_hs(16, nt=8, nph=16), f)
    g, l = C.q_fsm(_hs(16, nt=8, nph=16, nr=16), f, parts=True)
    scale = max(np.abs(g - l).max(), np.abs(l).max())
    assert np.abs(q32 - q128).max() < 1e-3 * scale
    # two discretisations of the same hard-sphere operator
    assert np.abs(q128 - (g - l)).max() < 2e-2 * scale


def test_rejects_other_kernels():
    with pytest.raises(ValueError):
        CA.q_carleman(Spec(d=3, N=8, L=4.0, gamma=0.0), np.ones(512))


def _bkw2d(sp, t=1.0):
    v2 = (velocity_nodes(sp) ** 2).sum(1)
    K = 1.0 - 0.5 * np.exp(-t / 8.0)
    dK = np.exp(-t / 8.0) / 16.0
    E = np.exp(-v2 / (2 * K))
    poly = 2 * K - 1 + (1 - K) * v2 / (2 * K)
    f = E / (2 * np.pi * K * K) * poly
    df = E / (2 * np.pi * K * K) * (v2 / (2 * K * K) * poly - 2 / K * poly + 2 - v2 / (2 * K * K)) * dK
    return f, 2 * np.pi * df


def test_2d_maxwell_carleman_matches_bkw_closed_form():
    # 2D Maxwell molecules, B = 1: the 2D BKW solution (K = 1 - exp(-t/8)/2) gives
    # Q[f] = 2 pi df/dt; this fixes the Carleman constant 2 and both weights.  The
    # error is the sqrt(2) R truncation and the grid: it falls to 1.3e-8 on a
    # wider, finer box
    errs = []
    for N, L in ((24, 8.0), (64, 12.0)):
        sp = Spec(d=2, N=N, L=L, n_phi=32)
        f, ref = _bkw2d(sp)
        errs.append(np.abs(CA.q_carleman_2d(sp, f) - ref).max() / np.abs(ref).max())
    assert errs[1] < 1e-7 < errs[0]


def test_2d_maxwell_carleman_conserves_mass_and_agrees_with_the_sigma_form():
    sp = Spec(d=2, N=48, L=8.0, n_phi=32, n_rho=24)
    f = synth.mixture_batch(1, 48, 8.0, d=2, seed=9)[0]
    gain, loss = CA.q_carleman_2d(sp, f, parts=True)
    assert abs(np.sum(gain - loss)) < 1e-13 * np.sum(np.abs(gain))
    g, l = C.q_fsm(sp, f, parts=True)
    scale = max(np.abs(g - l).max(), np.abs(l).max())
    # two discretisations of one operator, truncated differently (sqrt(2) R for x
    # and y, 2R for |g|): on this broad mixture they differ by 7e-3
    assert np.abs((gain - loss) - (g - l)).max() < 2e-2 * scale
    with pytest.raises(ValueError):
        CA.q_carleman_2d(Spec(d=2, N=8, L=4.0, gamma=1.0, n_phi=8), np.ones(64))
