"""Pins of the oracle's learned warm start in the 2D scans (CPU only).

The candidates change only where a visit's inner iteration starts:
  * in a one-cell cavity the first visit's right-hand side is the transport
    part the network sees, so a network that outputs that visit's exact
    solution (the independent theta-Newton fixed point) is chosen, and the
    visit then needs a single update where the plain start needs several; a
    planted choice that ignores the candidate fails this;
  * a network that outputs zero (candidate = the local Maxwellian) is not
    chosen over a cell's own non-equilibrium state here, and the scan equals
    the plain scan exactly;
  * converged states do not depend on the network.
"""
import numpy as np

from oracle import cavity as CV, cell as OC, collision as OQ, mlp as OM
from oracle.grid import Spec


def _spec():
    return Spec(d=2, N=8, L=6.0, n_phi=8, n_rho=3)


def _network(K, b3):
    H = 3
    p = np.zeros(OM.n_params(K + 5, H, K))
    p[-K:] = b3
    return (p, K + 5, H, K, 1.0)


def _first_visit_solution(prob, f):
    Q, M, nu = CV.all_collision(prob, f)
    P = OQ.penalty_split(Q, M, f, nu)
    T = CV.transport_part(prob, f)
    r = T[0, 0] - P[0, 0] / prob.eps
    g, _ = OC.theta_solve(prob.spec, r, nu[0, 0], prob.eps, (prob.dx, prob.dy))
    return g, M[0, 0]


def _one_cell(**kw):
    return CV.Cavity(spec=_spec(), nx=1, ny=1, eps=0.2, collision="binary", tol_inner=1e-9, **kw)


def _fresh(prob):
    prob.stats = {"inner": 0, "fallback": 0, "visits": 0, "learned": 0}


def test_exact_network_output_is_chosen_and_converges_in_one_update():
    prob = _one_cell()
    f1 = CV.sgs_iteration(prob, CV.initial_state(prob))
    g_star, M0 = _first_visit_solution(prob, f1)
    _fresh(prob)
    plain = CV.scan(prob, f1, 1, 1)
    plain_updates = prob.stats["inner"]
    prob.warm = _network(prob.spec.K, g_star - M0)
    _fresh(prob)
    warm = CV.scan(prob, f1, 1, 1)
    assert prob.stats["learned"] == 1
    assert prob.stats["inner"] == 1 < plain_updates
    assert np.abs(warm[0, 0] - g_star).max() < 1e-9 * g_star.max()
    assert np.abs(warm[0, 0] - plain[0, 0]).max() < 1e-7 * g_star.max()


def test_planted_ignored_candidate_is_caught(monkeypatch):
    prob = _one_cell()
    f1 = CV.sgs_iteration(prob, CV.initial_state(prob))
    g_star, M0 = _first_visit_solution(prob, f1)
    _fresh(prob)
    CV.scan(prob, f1, 1, 1)
    plain_updates = prob.stats["inner"]
    prob.warm = _network(prob.spec.K, g_star - M0)
    monkeypatch.setattr(CV, "warm_choice", lambda *a: False)
    _fresh(prob)
    CV.scan(prob, f1, 1, 1)
    assert prob.stats["learned"] == 0 and prob.stats["inner"] == plain_updates > 1


def test_zero_network_keeps_the_plain_scan():
    prob = CV.Cavity(spec=_spec(), nx=3, ny=2, eps=0.1, collision="binary", fixed_inner=3)
    f1 = CV.sgs_iteration(prob, CV.initial_state(prob))
    _fresh(prob)
    plain = CV.sgs_iteration(prob, f1)
    prob.warm = _network(prob.spec.K, np.zeros(prob.spec.K))
    _fresh(prob)
    warm = CV.sgs_iteration(prob, f1)
    assert prob.stats["learned"] == 0
    assert np.array_equal(warm, plain)


def test_converged_state_does_not_depend_on_the_network():
    out = []
    for with_net in (False, True):
        prob = CV.Cavity(spec=_spec(), nx=2, ny=2, eps=0.3, collision="bgk", tol_inner=1e-11)
        f0 = CV.initial_state(prob)
        if with_net:
            one = CV.Cavity(spec=_spec(), nx=2, ny=2, eps=0.3, collision="bgk")
            Q, M, nu = CV.all_collision(one, f0)
            T = CV.transport_part(one, f0)
            g, _ = OC.theta_solve(one.spec, T[0, 0], nu[0, 0], one.eps, (one.dx, one.dy))
            prob.warm = _network(prob.spec.K, g - M[0, 0])
        f, hist = f0, []
        for _ in range(200):
            hist.append(CV.outer_residual(prob, f))
            if hist[-1] < 1e-9:
                break
            f = CV.sgs_iteration(prob, f)
        assert hist[-1] < 1e-9
        assert (prob.stats["learned"] >= 1) == with_net
        out.append(f)
    assert np.abs(out[0] - out[1]).max() < 1e-8 * out[0].max()
