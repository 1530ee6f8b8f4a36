"""Pins of the oracle's scans with the binary collision operator (CPU only).

Section 3.3 (eq. SGS) lags P = Q - nu (M - f) (eq. Pf) over a scan and puts
-P/eps into the right-hand side of every visit.  At a fixed point of the scans
each visit's equation c g + r = (nu/eps)(M[g] - g) holds with g = f, which
rearranges to transport(f) = (P + nu (M - f))/eps = Q/eps: the outer residual,
built from Q alone, must vanish there, whatever nu is.  A slip in the split
(a sign, a dropped term) moves the fixed point and leaves a residual of the
size of nu (M - f)/eps, which these pins catch (the planted-mistake tests
show it on the same problems).
"""
import numpy as np

from oracle import cavity as CV, collision as C, maxwellian as MX, sweep as SW
from oracle.grid import Spec


def _binary_slab(nx=4):
    # 8^3 on [-4, 4)^3 with the grid shifted by half a node along v_1, so that no
    # node has v_1 = 0: there transport does not damp the lagged collision term,
    # and on a grid this coarse the truncated kernel's small loss frequency in the
    # tails makes that mode decay by under 1% per iteration
    sp = Spec(d=3, N=8, L=4.0, n_theta=2, n_phi=4, n_rho=3, v1_shift=0.5)
    return SW.Slab(spec=sp, nx=nx, eps=1.0, collision="binary", tol_inner=1e-12, max_inner=200)


def test_penalty_of_a_discrete_maxwellian_vanishes():
    # eq. discrete_Q makes the discrete Maxwellian an exact equilibrium, and
    # nu (M - f) vanishes at f = M, so P[M] = 0 to rounding (Section 3.3)
    sp = Spec(d=3, N=8, L=6.0, n_theta=2, n_phi=4, n_rho=3)
    import synth

    f = synth.mixture_batch(1, 8, 6.0, seed=41)[0]
    M = MX.discrete_maxwellian(sp, f)
    P = C.penalty(sp, M)
    _, loss = C.q_fsm(sp, M, parts=True)
    assert np.abs(P).max() < 1e-13 * np.abs(loss).max()
    # away from equilibrium the split is not trivial: P differs from Q by nu (M - f)
    Pf = C.penalty(sp, f)
    Qf = C.q_corrected(sp, f, conserve="mass")
    assert np.abs(Pf - Qf).max() > 1e-2 * np.abs(Qf).max()


def test_binary_slab_scans_converge_to_a_zero_of_the_q_residual():
    prob = _binary_slab()
    f, hist = SW.solve_sgs(prob, SW.initial_state(prob, T=1.5), tol=1e-9, max_iter=100)
    assert hist[-1] <= 1e-9, hist[-5:]
    # the converged state is not a global equilibrium: the walls differ, the
    # collision term is far from zero, and the temperature rises to the hot wall
    Q, M, nu = SW.all_collision(prob, f)
    assert np.abs(Q).max() > 1e-3 * np.abs(f).max() / prob.eps
    T = [MX.macroscopic(prob.spec, f[j])[2] for j in range(prob.nx)]
    assert all(T[j + 1] > T[j] for j in range(prob.nx - 1)), T


def _final_or_inf(run):
    """Last outer residual of a run, or inf when the run drives an iterate to a
    state whose discrete Maxwellian does not exist (Newton fails)."""
    try:
        return run()[-1]
    except RuntimeError:
        return np.inf


def test_planted_penalty_sign_slip_is_caught_on_the_slab(monkeypatch):
    # plant P = Q + nu (M - f) in the oracle's scans: the scans then either settle
    # to a state whose Q residual does not vanish or leave the physical states
    monkeypatch.setattr(SW, "penalty_split", lambda Q, M, f, nu: Q + np.asarray(nu)[..., None] * (M - f))
    prob = _binary_slab()
    assert _final_or_inf(lambda: SW.solve_sgs(prob, SW.initial_state(prob, T=1.5), tol=1e-9, max_iter=40)[1]) > 1e-4


def _binary_cavity():
    sp = Spec(d=2, N=8, L=4.0, n_phi=8, n_rho=4)
    walls = ((1.0, (0.0, 0.0)), (1.5, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.4, 0.0)))
    return CV.Cavity(spec=sp, nx=3, ny=3, eps=1.0, walls=walls, collision="binary", tol_inner=1e-12, max_inner=200)


def _cavity_run(prob, tol, max_iter):
    f = CV.initial_state(prob)
    hist = [CV.outer_residual(prob, f)]
    for _ in range(max_iter):
        f = CV.sgs_iteration(prob, f)
        hist.append(CV.outer_residual(prob, f))
        if hist[-1] <= tol:
            break
    return f, hist


def test_binary_cavity_scans_converge_to_a_zero_of_the_q_residual():
    prob = _binary_cavity()
    f, hist = _cavity_run(prob, 1e-9, 60)
    assert hist[-1] <= 1e-9, hist[-5:]
    Q, _, _ = CV.all_collision(prob, f)
    assert np.abs(Q).max() > 1e-3 * np.abs(f).max() / prob.eps


def test_planted_penalty_sign_slip_is_caught_on_the_cavity(monkeypatch):
    monkeypatch.setattr(CV, "penalty_split", lambda Q, M, f, nu: Q + np.asarray(nu)[..., None] * (M - f))
    prob = _binary_cavity()
    assert _final_or_inf(lambda: _cavity_run(prob, 1e-9, 20)[1]) > 1e-4
