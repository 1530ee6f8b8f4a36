"""Pins of the oracle's learned warm start inside the slab scans (CPU only).

The warm start changes only where a visit's inner iteration starts.  Pins:
  * a network whose output is the visit's exact inner solution (built from the
    independent theta-Newton fixed point) is chosen, and the visit then needs a
    single update, where the plain start needs several; a planted choice that
    ignores the candidate fails this;
  * the choice goes to the candidate with the smaller inner residual: a network
    that outputs zero (candidate = the local Maxwellian) is never chosen over
    a cell's own non-equilibrium state on this problem, and the scan then
    equals the plain scan exactly;
  * converged states do not depend on the network.
"""
import numpy as np

from oracle import cell as OC, mlp as OM, sweep as SW
from oracle.grid import Spec


def _prob(**kw):
    sp = Spec(d=3, N=8, L=4.0, n_theta=2, n_phi=4, n_rho=3, v1_shift=0.5)
    return SW.Slab(spec=sp, nx=3, eps=0.1, collision="binary", **kw)


def _first_visit_solution(prob, f):
    """Exact inner solution of the forward scan's first visit (its r has no fresh
    neighbour), by the theta-Newton fixed point."""
    Q, M, nu = SW.all_collision(prob, f)
    P = SW.penalty_split(Q, M, f, nu)
    T = SW.transport_part(prob, f)
    r = T[0] - P[0] / prob.eps
    g, _ = OC.theta_solve(prob.spec, r, nu[0], prob.eps, prob.dx)
    return g, M[0]


def _network(K, b3):
    H = 3
    p = np.zeros(OM.n_params(K + 6, H, K))
    p[-K:] = b3
    return (p, K + 6, H, K, 1.0)


def _fresh(prob):
    prob.stats = {"inner": 0, "fallback": 0, "visits": 0, "learned": 0}


def test_exact_network_output_is_chosen_and_converges_in_one_update():
    # one cell: its visit has no fresh neighbour, so the problem the network sees
    # is exactly the visit's
    prob = _prob(tol_inner=1e-9)
    prob.nx = 1
    f1 = SW.sgs_iteration(prob, SW.initial_state(prob, T=1.5))
    g_star, M0 = _first_visit_solution(prob, f1)
    _fresh(prob)
    plain = SW.scan(prob, f1, True)
    plain_updates = prob.stats["inner"]
    prob.warm = _network(prob.spec.K, g_star - M0)
    _fresh(prob)
    warm = SW.scan(prob, f1, True)
    assert prob.stats["learned"] == 1
    # the visit started at its own solution: one update, the same result
    assert prob.stats["inner"] == 1 < plain_updates
    assert np.abs(warm[0] - g_star).max() < 1e-9 * g_star.max()
    assert np.abs(warm[0] - plain[0]).max() < 1e-7 * g_star.max()


def test_planted_ignored_candidate_is_caught(monkeypatch):
    # plant a choice that never takes the candidate: the first visit then needs as
    # many updates as the plain start, which the pin above rejects
    prob = _prob(tol_inner=1e-9)
    prob.nx = 1
    f1 = SW.sgs_iteration(prob, SW.initial_state(prob, T=1.5))
    g_star, M0 = _first_visit_solution(prob, f1)
    _fresh(prob)
    SW.scan(prob, f1, True)
    plain_updates = prob.stats["inner"]
    prob.warm = _network(prob.spec.K, g_star - M0)
    monkeypatch.setattr(SW, "warm_starts", lambda prob_, f, P, nu, b: [None] * prob_.nx)
    _fresh(prob)
    SW.scan(prob, f1, True)
    assert prob.stats["learned"] == 0 and prob.stats["inner"] == plain_updates > 1


def test_zero_network_keeps_the_plain_scan():
    prob = _prob(fixed_inner=3)
    f1 = SW.sgs_iteration(prob, SW.initial_state(prob, T=1.5))
    _fresh(prob)
    plain = SW.sgs_iteration(prob, f1)
    prob.warm = _network(prob.spec.K, np.zeros(prob.spec.K))
    _fresh(prob)
    warm = SW.sgs_iteration(prob, f1)
    assert prob.stats["learned"] == 0
    assert np.array_equal(warm, plain)


def test_converged_state_does_not_depend_on_the_network():
    # a network that is taken at the first visit (its output is that visit's exact
    # solution from the initial state) and not later: same converged state
    sp = Spec(d=3, N=8, L=6.0)
    base = SW.Slab(spec=sp, nx=4, eps=0.1, collision="bgk", tol_inner=1e-11)
    f0 = SW.initial_state(base, T=1.5)
    g_star, M0 = _first_visit_solution(base, f0)
    out = []
    for warm in (None, _network(sp.K, g_star - M0)):
        prob = SW.Slab(spec=sp, nx=4, eps=0.1, collision="bgk", tol_inner=1e-11, warm=warm)
        f, hist = SW.solve_sgs(prob, f0, tol=1e-9, max_iter=200)
        assert hist[-1] < 1e-9
        assert (prob.stats["learned"] >= 1) == (warm is not None)
        out.append(f)
    assert np.abs(out[0] - out[1]).max() < 1e-8 * out[0].max()
