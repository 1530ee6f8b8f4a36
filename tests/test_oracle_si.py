"""Pins of the oracle's source iteration (eq. SI, BGK; CPU only): its fixed
point is the steady state the SGS scans reach, and it converges more slowly
than SGS as eps falls (the paper's amplification factors 1 - O(eps^2) for SI
against 1 - O(eps) for SGS, Section 3.1); with eps huge both reduce to the
collisionless transport solve."""
import numpy as np

from oracle import sweep as SW
from oracle.grid import Spec


def _run(inner, eps, tol=1e-10, max_iter=400):
    sp = Spec(d=3, N=8, L=6.0)
    prob = SW.Slab(spec=sp, nx=4, eps=eps, collision="bgk", inner=inner, tol_inner=1e-12)
    return SW.solve_sgs(prob, SW.initial_state(prob, T=1.5), tol=tol, max_iter=max_iter)


def test_si_reaches_the_sgs_steady_state():
    f_si, h_si = _run("si", 1.0)
    f_sgs, h_sgs = _run("pfp", 1.0)
    assert h_si[-1] < 1e-10 and h_sgs[-1] < 1e-10
    assert np.abs(f_si - f_sgs).max() < 1e-8 * f_sgs.max()


def test_si_slows_down_faster_than_sgs_as_eps_falls():
    rates = {}
    for inner in ("si", "pfp"):
        for eps in (1.0, 0.1):
            _, h = _run(inner, eps, tol=1e-12, max_iter=60)
            h = np.array(h)
            tail = h[-10:] if len(h) > 12 else h[len(h) // 2:]
            rates[inner, eps] = (tail[-1] / tail[0]) ** (1.0 / (len(tail) - 1))
    # per-iteration reduction factors: SI degrades from eps = 1 to 0.1 far more than SGS
    assert rates["si", 0.1] > rates["pfp", 0.1]
    assert (1.0 - rates["si", 0.1]) / (1.0 - rates["si", 1.0]) < (1.0 - rates["pfp", 0.1]) / (1.0 - rates["pfp", 1.0])


def test_si_is_the_transport_solve_without_collisions():
    # no v_1 = 0 node: there the transport part vanishes and the collision term
    # decides the value however large eps is
    sp = Spec(d=3, N=8, L=6.0, v1_shift=0.5)
    out = []
    for inner in ("si", "pfp"):
        prob = SW.Slab(spec=sp, nx=6, eps=1e12, collision="bgk", inner=inner, tol_inner=1e-14)
        f = SW.initial_state(prob, T=1.5)
        for _ in range(3):
            f = SW.sgs_iteration(prob, f)
        out.append(f)
    assert np.abs(out[0] - out[1]).max() < 1e-10 * out[1].max()
