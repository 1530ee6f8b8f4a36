"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms (BKW, collisionless slab), invariants (mass conservation, symmetry,
equilibrium), an independent physical-space quadrature, and brute-force limits."""
import numpy as np
import pytest

import synth
from oracle import cell, collision as C, maxwellian as MX, physical as PH, sweep as SW
from oracle.grid import Spec, velocity_nodes


# ------------------------------------------------------------------ Maxwellian
def test_discrete_maxwellian_moments_and_idempotence():
    sp = Spec(d=3, N=16, L=8.0)
    f = synth.mixture_batch(1, 16, 8.0, seed=11)[0]
    M, th = MX.discrete_maxwellian(sp, f, return_theta=True)
    m_f, m_M = MX.moments(sp, f), MX.moments(sp, M)
    assert np.max(np.abs(m_f - m_M) / np.abs(m_f).max()) < 1e-13
    M2 = MX.discrete_maxwellian(sp, M)
    assert np.max(np.abs(M2 - M)) < 1e-13 * M.max()


def test_gaussian_input_returns_its_parameters():
    sp = Spec(d=3, N=16, L=8.0)
    th = MX.theta_from_macro(sp, 1.3, np.array([0.3, -0.2, 0.1]), 1.2)
    th[0] += 0.01  # any Gaussian of this form is its own discrete Maxwellian
    G = MX.gaussian(sp, th)
    _, th2 = MX.discrete_maxwellian(sp, G, return_theta=True)
    assert np.max(np.abs(th2 - th)) < 1e-12


def test_resolved_maxwellian_matches_continuous_parameters():
    # a well-resolved continuous Maxwellian sampled on the grid: the discrete
    # parameters approach the continuous ones (eq. maxwellian)
    sp = Spec(d=3, N=32, L=8.0)
    rho, U, T = 0.9, np.array([0.2, 0.1, -0.3]), 1.1
    f = synth.maxwellian_mixture([(rho, U, T)], 32, 8.0)
    _, th = MX.discrete_maxwellian(sp, f, return_theta=True)
    assert np.max(np.abs(th - MX.theta_from_macro(sp, rho, U, T))) < 1e-8


# ------------------------------------------------------------------ collision
def _narrow(N, L, seed=3):
    return synth.mixture_batch(1, N, L, seed=seed, T=(0.15, 0.25), speed=(0.0, 0.3))[0]


def test_sigma_exact_sum_conserves_mass():
    sp = Spec(d=3, N=8, L=4.0)
    f = _narrow(8, 4.0)
    D = C.q_direct(sp, f)
    g, l = C.q_direct(sp, f, parts=True)
    assert abs(MX.moments(sp, D)[0]) < 1e-13 * sp.w * np.abs(l).sum()


def test_fast_form_converges_to_sigma_exact_sum():
    f = _narrow(8, 4.0)
    D = C.q_direct(Spec(d=3, N=8, L=4.0), f)
    errs = []
    for nt in (4, 8, 16):
        sp = Spec(d=3, N=8, L=4.0, n_theta=nt, n_phi=2 * nt, n_rho=nt)
        errs.append(np.abs(C.q_fsm(sp, f) - D).max() / np.abs(D).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-11


def test_mass_projection_removes_only_quadrature_mass():
    """The collision integral conserves mass, and so does the sigma-exact sum.  The
    mass-projected fast form conserves it to rounding, keeps the corrected form
    exact at equilibrium, and changes Q by an amount that vanishes as the sphere
    rule is refined (so it removes only quadrature error)."""
    f = _narrow(8, 4.0)
    changes = []
    for nt in (4, 8, 16):
        sp = Spec(d=3, N=8, L=4.0, n_theta=nt, n_phi=2 * nt, n_rho=nt)
        M = MX.discrete_maxwellian(sp, f)
        Q = C.q_corrected(sp, f, M)
        Qp = C.q_corrected(sp, f, M, conserve="mass")
        _, loss = C.q_fsm(sp, f, parts=True)
        assert abs(MX.moments(sp, Qp)[0]) < 1e-14 * sp.w * np.abs(loss).sum()
        assert np.abs(C.q_corrected(sp, M, M, conserve="mass")).max() == 0.0
        changes.append(np.abs(Qp - Q).max() / np.abs(Q).max())
    assert changes[0] > changes[1] > changes[2]
    assert changes[2] < 1e-9


def test_conservation_projection_is_the_least_change_that_conserves():
    """conserve_project: zero mass, momentum and energy to rounding; a projection
    (idempotent); exact at equilibrium; and no other change with those moments is
    smaller in the sum of dQ^2 / M (checked against random admissible changes)."""
    sp = Spec(d=3, N=8, L=6.0, n_theta=4, n_phi=8, n_rho=4)
    f = synth.mixture_batch(1, 8, 6.0, seed=4, T=(0.8, 1.2), speed=(0.0, 0.3))[0]
    M = MX.discrete_maxwellian(sp, f)
    Q = C.q_corrected(sp, f, M)
    Qp = C.q_corrected(sp, f, M, conserve="all")
    m = MX.moments(sp, Qp)
    scale = sp.w * np.abs(Q).sum() * np.array([1.0, sp.L, sp.L, sp.L, sp.L ** 2])
    assert np.all(np.abs(m) < 1e-13 * scale), m
    assert np.abs(C.conserve_project(sp, Qp, M) - Qp).max() < 1e-13 * np.abs(Qp).max()
    assert np.abs(C.q_corrected(sp, M, M, conserve="all")).max() == 0.0
    dQ = Qp - Q
    base = np.sum(dQ * dQ / M)
    rng = np.random.default_rng(0)
    for _ in range(5):
        h = rng.normal(size=sp.K) * M  # an arbitrary direction, made admissible below
        h = C.conserve_project(sp, h, M)  # zero invariant moments
        other = dQ + 1e-3 * np.abs(dQ).max() * h / np.abs(h).max()
        assert np.sum(other * other / M) > base


@pytest.mark.slow
def test_fast_form_matches_physical_space_quadrature():
    # independent pin of the whole Fourier derivation: direct quadrature of the
    # truncated integral for an analytic mixture, at nodes with |v| + R_g <= L
    N, L = 32, 8.0
    sp = Spec(d=3, N=N, L=L, n_theta=8, n_phi=16, n_rho=16)
    rng = np.random.default_rng([5, 0])
    params = synth.mixture_params(rng, T=(0.8, 1.2), speed=(0.0, 0.5))
    f = synth.maxwellian_mixture(params, N, L)
    g, l = C.q_fsm(sp, f, parts=True)
    v = velocity_nodes(sp)
    idx = [i for i in range(len(v)) if np.linalg.norm(v[i]) < 1.9][::331][:2]
    gp, lp = PH.q_physical(params, v[idx], 3, sp.R_g, n_rho=32, n_sph=12)
    scale = np.abs(l).max()
    assert np.max(np.abs(g[idx] - gp)) < 1e-7 * scale
    assert np.max(np.abs(l[idx] - lp)) < 1e-7 * scale


def test_bkw_closed_form():
    # Bobylev-Krook-Wu solution for Maxwell molecules (3D, kernel normalised to
    # one over the sphere): Q[f] = df/dt; with B = 1 the operator is 4 pi times that.
    errs = []
    for N, nt, nr in [(16, 8, 8), (24, 8, 12)]:
        sp = Spec(d=3, N=N, L=8.0, n_theta=nt, n_phi=2 * nt, n_rho=nr)
        v = velocity_nodes(sp)
        v2 = (v * v).sum(1)
        t = 6.5
        K = 1 - np.exp(-t / 6)
        dK = np.exp(-t / 6) / 6

        def fb(K):
            return np.exp(-v2 / (2 * K)) / (2 * (2 * np.pi * K) ** 1.5) * ((5 * K - 3) / K + (1 - K) / K ** 2 * v2)

        dfb = (np.exp(-v2 / (2 * K)) / (2 * (2 * np.pi * K) ** 1.5)
               * (v2 / (2 * K * K) * ((5 * K - 3) / K + (1 - K) / K ** 2 * v2)
                  - 1.5 / K * ((5 * K - 3) / K + (1 - K) / K ** 2 * v2)
                  + 3 / K ** 2 + (K - 2) / K ** 3 * v2)) * dK
        Q = C.q_fsm(sp, fb(K))
        errs.append(np.abs(Q - 4 * np.pi * dfb).max() / np.abs(4 * np.pi * dfb).max())
    assert errs[1] < 0.2 * errs[0]
    assert errs[1] < 1e-2


def test_maxwellian_is_near_equilibrium_and_corrected_form_exact():
    sp = Spec(d=3, N=32, L=8.0, n_theta=4, n_phi=8, n_rho=8)
    f = synth.mixture_batch(1, 32, 8.0, seed=2, T=(0.8, 1.2), speed=(0.0, 0.3))[0]
    M = MX.discrete_maxwellian(sp, f)
    g, l = C.q_fsm(sp, M, parts=True)
    assert np.abs(g - l).max() < 1e-6 * np.abs(l).max()  # spectral accuracy
    assert np.abs(C.q_corrected(sp, M, M)).max() == 0.0  # eq. discrete_Q


def test_symmetries_reflection_swap_translation():
    sp = Spec(d=3, N=8, L=4.0, n_theta=4, n_phi=8, n_rho=4)
    f = _narrow(8, 4.0, seed=7).reshape(8, 8, 8)
    Q = C.q_fsm(sp, f.reshape(-1)).reshape(8, 8, 8)
    # swapping the two azimuthal axes maps the sigma rule onto itself (n_phi % 4 == 0)
    Qs = C.q_fsm(sp, f.transpose(0, 2, 1).reshape(-1)).reshape(8, 8, 8)
    assert np.abs(Qs - Q.transpose(0, 2, 1)).max() < 1e-13 * np.abs(Q).max()
    # reflection v -> -v on the periodic grid: index j -> N-2-j (mod N), on the polar axis
    ref = (8 - 2 - np.arange(8)) % 8
    Qr = C.q_fsm(sp, f[ref].reshape(-1)).reshape(8, 8, 8)
    assert np.abs(Qr - Q[ref]).max() < 1e-13 * np.abs(Q).max()
    # translation by one node along axis 2 (the operator is translation invariant)
    Qt = C.q_fsm(sp, np.roll(f, 1, axis=2).reshape(-1)).reshape(8, 8, 8)
    assert np.abs(Qt - np.roll(Q, 1, axis=2)).max() < 1e-13 * np.abs(Q).max()


# ------------------------------------------------------------------ cell solve
def _cell_case(i=0, N=8, L=6.0, dx=1 / 32):
    sp = Spec(d=3, N=N, L=L, n_theta=2, n_phi=4, n_rho=4)
    fo, fl, fr, _ = synth.cell_inflow_batch(i + 1, N, L, dx)
    v1 = velocity_nodes(sp)[:, 0]
    r = (-np.maximum(v1, 0) * fl[i] + np.minimum(v1, 0) * fr[i]) / dx
    return sp, r, C.nu_of(sp, fo[i]), fo[i], dx


@pytest.mark.parametrize("eps", [1.0, 0.01])
def test_fp_and_pfp_reach_the_theta_newton_fixed_point(eps):
    sp, r, nu, g0, dx = _cell_case()
    gs, _ = cell.theta_solve(sp, r, nu, eps, dx)
    scale = np.abs(gs).max()
    assert cell.inner_residual(sp, gs, r, nu, eps, dx) < 1e-10 * (nu / eps) * scale
    g1, s1 = cell.solve(sp, r, nu, eps, dx, g0, mode="pfp", tol=1e-11)
    g2, s2 = cell.solve(sp, r, nu, eps, dx, g0, mode="fp", tol=1e-11, max_iter=5000)
    assert not s1.fallback
    assert np.abs(g1 - gs).max() < 1e-8 * scale
    assert np.abs(g2 - gs).max() < 1e-5 * scale  # FP converges slowly at small eps
    # eq. macro holds at the fixed point (conservation of the discrete Maxwellian)
    c = cell.transport_coef(sp, dx)
    macro = MX.moments(sp, c * gs + r)
    assert np.max(np.abs(macro)) < 1e-9 * np.max(np.abs(MX.moments(sp, np.abs(c * gs) + np.abs(r))))
    # the preconditioned iteration does not slow down as eps -> 0 (Section 3.2)
    assert s1.iterations < s2.iterations


def test_pfp_falls_back_when_existence_fails():
    sp, r, nu, g0, dx = _cell_case()
    # shift r by a constant so that s_0 = sum w (c (M[g0] - g0) - r) < 0: eq. existence fails
    c = cell.transport_coef(sp, dx)
    s0 = sp.w * np.sum(c * (MX.discrete_maxwellian(sp, g0) - g0) - r)
    r_bad = r + (s0 + 1e-3 * abs(s0)) / (sp.w * sp.K)
    _, st = cell.solve(sp, r_bad, nu, 0.01, dx, g0, mode="pfp", fixed_iters=2)
    assert st.fallback
    _, st = cell.solve(sp, r, nu, 0.01, dx, g0, mode="pfp", fixed_iters=2)
    assert not st.fallback


def test_weighted_newton_reports_a_singular_jacobian_as_failure():
    # Step 1 with a weight that leaves fewer than d + 2 nodes has a singular
    # Jacobian; that is a Newton failure, after which the visit falls back
    # (Section 3.2), not an error
    sp = Spec(d=3, N=8, L=6.0, n_theta=2, n_phi=4, n_rho=2)
    target = MX.moments(sp, MX.gaussian(sp, MX.theta_from_macro(sp, 1.0, np.zeros(3), 1.0)))
    for keep in (0, 1):
        c = np.zeros(sp.K)
        c[:keep] = 1.0
        _, _, ok = MX.solve_weighted_gaussian(sp, target, weight=c)
        assert not ok


def test_large_eps_limit():
    # eps -> infinity: (|v_1|/dx) g = -r wherever v_1 != 0
    sp, r, nu, g0, dx = _cell_case()
    gs, _ = cell.theta_solve(sp, r, nu, 1e12, dx)
    c = cell.transport_coef(sp, dx)
    m = c > 0
    assert np.abs(gs[m] + r[m] / c[m]).max() < 1e-8 * np.abs(r[m] / c[m]).max()


# ------------------------------------------------------------------ sweep
@pytest.mark.parametrize("order", [1, 2])
def test_collisionless_slab_closed_form(order):
    # eps huge, BGK (P == 0): right-movers carry the left wall Maxwellian, left-movers
    # the right one; the discrete zero-flux condition fixes rho_L/rho_R, the mass C the
    # scale.  The solution is uniform in x, so the second-order slopes vanish on it.
    sp = Spec(d=3, N=8, L=6.0)
    prob = SW.Slab(spec=sp, nx=6, eps=1e12, collision="bgk", T_L=1.0, T_R=2.0, mass=1.3, order=order)
    f, hist = SW.solve_sgs(prob, SW.initial_state(prob), tol=1e-12, max_iter=60)
    v1 = velocity_nodes(sp)[:, 0]
    ML, MR = SW.wall_maxwellian(sp, 1.0, (0, 0, 0)), SW.wall_maxwellian(sp, 2.0, (0, 0, 0))
    a = np.sum(np.where(v1 > 0, v1, 0) * ML)
    b = np.sum(np.where(v1 < 0, -v1, 0) * MR)
    # rho_L a = rho_R b (no net flux), and mass: dx w sum_j (rho_L sum_{v1>0} ML + rho_R sum_{v1<0} MR) = C
    rho_L = b / a  # with rho_R = 1
    unit = np.where(v1 > 0, rho_L * ML, 0.0) + np.where(v1 < 0, MR, 0.0)
    # nodes with v_1 = 0 are not transported (g = M[g] there), so the total mass fixes
    # only a common scale: f / unit must be one constant over every cell and node
    m = (v1 != 0) & (unit > 1e-6 * unit.max())
    ratio = f[:, m] / unit[None, m]
    assert hist[-1] < 1e-10
    # the state error at a residual of 1e-12 grows with the contraction rate,
    # which is slower for the wider second-order stencil
    assert np.ptp(ratio) < (1e-10 if order == 1 else 1e-9) * ratio.mean()


def test_penalty_frequency_is_the_mean_binary_loss_frequency():
    # Hard spheres: nu equals the Maxwellian average of the exact loss frequency
    # 4 pi int |v - w| M(w) dw (closed form with erf), integrated radially here;
    # Maxwell molecules: nu = 4 pi rho exactly (Section 4.1.2)
    from scipy.integrate import quad
    from scipy.special import erf

    T, rho = 1.0, 1.3
    sp = Spec(d=3, N=32, L=8.0, gamma=1.0)
    v = velocity_nodes(sp)
    M = rho * (2 * np.pi * T) ** -1.5 * np.exp(-(v * v).sum(1) / (2 * T))

    def nu_hs(r):
        c = r / np.sqrt(2 * T)
        if c == 0.0:
            return rho * np.sqrt(8 * T / np.pi)
        return rho * np.sqrt(2 * T) * (np.exp(-c * c) / np.sqrt(np.pi) + (c + 0.5 / c) * erf(c))

    dens = lambda r: 4 * np.pi * r * r * (2 * np.pi * T) ** -1.5 * np.exp(-r * r / (2 * T))
    mean = quad(lambda r: dens(r) * 4 * np.pi * nu_hs(r), 0.0, 40.0, epsabs=0, epsrel=1e-12, limit=200)[0]
    assert abs(C.nu_of(sp, M) - mean) < 1e-8 * mean
    sp0 = Spec(d=3, N=32, L=8.0, gamma=0.0)
    assert C.nu_of(sp0, M) == 4 * np.pi * MX.moments(sp0, M)[0]


def test_second_order_transport_is_exact_on_quadratic_profiles():
    # With the slopes of eq. slope, the upwind flux difference of a profile
    # quadratic in x is exact at interior cells (the slope terms cancel the
    # O(dx) error of first-order upwinding, |v_1| c dx for f = c x^2).
    sp = Spec(d=3, N=8, L=6.0, n_theta=2, n_phi=4, n_rho=2)
    v1 = velocity_nodes(sp)[:, 0]
    g = np.exp(-0.3 * (velocity_nodes(sp) ** 2).sum(1))  # any velocity profile
    for order, exact in ((2, True), (1, False)):
        prob = SW.Slab(spec=sp, nx=10, eps=1.0, collision="bgk", order=order)
        x = prob.xL + (np.arange(prob.nx) + 0.5) * prob.dx
        c = 0.7
        f = 1.0 + c * x[:, None] ** 2 * g[None, :]
        R = SW.residual_field(prob, f, np.zeros_like(f))
        ref = v1[None, :] * 2.0 * c * x[:, None] * g[None, :]
        err = np.abs(R[2:-2] - ref[2:-2]).max() / np.abs(ref).max()
        assert (err < 1e-12) if exact else (err > 1e-3), (order, err)


@pytest.mark.slow
def test_sgs_fp_and_pfp_reach_the_same_state():
    # Section 4.1: with inner solves tight enough, SGS-FP and SGS-PFP follow the
    # same outer history and reach the same state.  The plain iteration needs
    # ~740 updates per visit here (eps = 0.1), hence the runtime (~70 s).
    sp = Spec(d=3, N=8, L=6.0)
    out, hists = [], []
    for inner in ("pfp", "fp"):
        prob = SW.Slab(spec=sp, nx=4, eps=0.1, collision="bgk", inner=inner, tol_inner=1e-11, max_inner=5000)
        f, hist = SW.solve_sgs(prob, SW.initial_state(prob, T=1.5), tol=1e-9, max_iter=200)
        out.append(f)
        hists.append(np.array(hist))
    assert np.abs(out[0] - out[1]).max() < 1e-8 * out[0].max()
    assert len(hists[0]) == len(hists[1])
    assert np.allclose(hists[0], hists[1], rtol=0.05, atol=0.0)


def test_multigrid_reaches_the_sgs_state():
    sp = Spec(d=3, N=8, L=6.0)
    prob = SW.Slab(spec=sp, nx=8, eps=0.1, collision="bgk")
    f_sgs, _ = SW.solve_sgs(prob, SW.initial_state(prob, T=1.5), tol=1e-9, max_iter=300)
    prob2 = SW.Slab(spec=sp, nx=8, eps=0.1, collision="bgk")
    f_mg, hist = SW.solve_mg(prob2, SW.initial_state(prob2, T=1.5), coarsest=2, tol=1e-9)
    assert hist[-1] < 1e-9
    assert np.abs(f_mg - f_sgs).max() < 1e-7 * f_sgs.max()
    # a converged state is a fixed point of the V-cycle
    f_again = SW.vcycle(prob2, f_mg, None, 2, 1, 1, 0.0)
    assert np.abs(f_again - f_mg).max() < 1e-7 * f_mg.max()


def test_inflow_equilibrium_is_a_steady_state_on_a_shifted_grid():
    # Equal inflow Maxwellians on both sides and the same Maxwellian in every cell:
    # transport vanishes cell by cell and the corrected collision term of a sampled
    # Gaussian is exactly zero, so the outer residual is zero to rounding and one
    # SGS iteration leaves the state unchanged; the grid is shifted along v_1 and
    # the bulk velocity is not a node, so the physical v_1 enters every upwind split
    sp = Spec(d=3, N=8, L=6.0, n_theta=2, n_phi=4, n_rho=3, v1_shift=1.25)
    U = (2.0, 0.3, 0.0)
    M = SW.wall_maxwellian(sp, 1.3, U) * 0.7
    prob = SW.Slab(spec=sp, nx=5, eps=0.1, bc_L="inflow", bc_R="inflow", rho_L=0.7, rho_R=0.7,
                   T_L=1.3, T_R=1.3, U_L=U, U_R=U, xL=-1.0, xR=1.0)
    f0 = np.repeat(M[None], 5, axis=0)
    prob.mass = SW.total_mass(prob, f0)
    scale = np.abs(cell.transport_coef(sp, prob.dx) * M).max()
    assert SW.outer_residual(prob, f0) < 1e-12 * scale
    f1 = SW.sgs_iteration(prob, f0)
    assert np.abs(f1 - f0).max() < 1e-12 * M.max()


def test_collisionless_inflow_closed_form_on_a_shifted_grid():
    # eps -> infinity, BGK: physical right-movers carry the left inflow Maxwellian,
    # left-movers the right one, in every cell; no physical v_1 is zero on this grid
    sp = Spec(d=3, N=8, L=6.0, v1_shift=1.0)
    v1 = sp.v1_shift + velocity_nodes(sp)[:, 0]
    assert np.all(v1 != 0.0)
    ML = SW.wall_maxwellian(sp, 1.0, (2.0, 0.0, 0.0)) * 1.0
    MR = SW.wall_maxwellian(sp, 1.8, (0.8, 0.0, 0.0)) * 2.2
    exact = np.where(v1 > 0, ML, MR)
    prob = SW.Slab(spec=sp, nx=6, eps=1e12, collision="bgk", bc_L="inflow", bc_R="inflow", rho_L=1.0, rho_R=2.2,
                   T_L=1.0, T_R=1.8, U_L=(2.0, 0.0, 0.0), U_R=(0.8, 0.0, 0.0))
    prob.mass = SW.total_mass(prob, np.repeat(exact[None], 6, axis=0))
    f = SW.initial_state(prob)
    for _ in range(3):
        f = SW.sgs_iteration(prob, f)
    assert np.abs(f - exact[None]).max() < 1e-10 * exact.max()


def test_relaxed_step1_keeps_the_preconditioned_iteration_and_reaches_the_fixed_point():
    # Section 3.2's remark: when eq. existence fails, step 1 with a relaxation
    # factor tau >= 1 has a solvable right-hand side.  A start of two cold beams
    # along v_1 (more |v_1|-weighted mass than its Maxwellian) violates eq.
    # existence at the first update; the relaxed iteration stays preconditioned
    # and reaches the fixed point of the independent theta-Newton solve, while the
    # plain-iteration fallback is still far from it after 100 updates
    sp, r, nu, _, dx = _cell_case()
    g0 = synth.maxwellian_mixture([(5.0, np.array([2.5, 0, 0]), 0.3), (5.0, np.array([-2.5, 0, 0]), 0.3)], 8, 6.0)
    eps = 0.01
    g, st = cell.solve(sp, r, nu, eps, dx, g0, mode="pfp", tol=1e-11, fallback="relax")
    assert st.relaxed >= 1 and not st.fallback and st.iterations < 20
    gs, _ = cell.theta_solve(sp, r, nu, eps, dx)
    assert np.abs(g - gs).max() < 1e-10 * np.abs(gs).max()
    _, st_fp = cell.solve(sp, r, nu, eps, dx, g0, mode="pfp", tol=1e-11)
    assert st_fp.fallback and st_fp.iterations == 100
    # at tau = 0 the relaxed right-hand side is step 1's: without a violation nothing changes
    sp, r, nu, g0, dx = _cell_case()
    g1, s1 = cell.solve(sp, r, nu, eps, dx, g0, mode="pfp", fixed_iters=3, fallback="relax")
    g2, s2 = cell.solve(sp, r, nu, eps, dx, g0, mode="pfp", fixed_iters=3)
    assert s1.relaxed == 0 and np.array_equal(g1, g2)


def test_minmod_limited_slopes_create_no_new_extrema():
    # With the minmod limiter the reconstructed face values f_j -+ s_j/2 stay
    # within the range of the neighbouring cell values (no new extrema: the
    # interior face values never leave [min, max] of the cells they join), the
    # slope vanishes at a local extremum and next to a jump, and on a monotone
    # smooth profile the slope is the smaller one-sided difference; the unlimited
    # centred slopes overshoot at a jump
    sp = Spec(d=3, N=4, L=4.0, n_theta=2, n_phi=4, n_rho=2)
    x = np.linspace(0.0, 1.0, 12)
    profiles = [np.where(x < 0.5, 1.0, 3.0), np.sin(6 * x) + 2.0, np.exp(x)]
    for prof in profiles:
        f = np.repeat(prof[:, None], sp.K, axis=1)
        for lim, bounded in (("minmod", True), ("none", False)):
            prob = SW.Slab(spec=sp, nx=12, order=2, limiter=lim, collision="bgk")
            s = SW.slopes(prob, f)[:, 0]
            east, west = prof + 0.5 * s, prof - 0.5 * s
            lo = np.minimum(prof[1:-2], prof[2:-1])
            hi = np.maximum(prof[1:-2], prof[2:-1])
            inside = np.all((east[1:-2] >= lo - 1e-15) & (east[1:-2] <= hi + 1e-15)
                            & (west[2:-1] >= lo - 1e-15) & (west[2:-1] <= hi + 1e-15))
            if bounded:
                assert inside
            elif prof is profiles[0]:
                assert not inside  # the centred slope overshoots at the jump
    # zero at a jump's neighbours and at extrema; the smaller difference on a monotone profile
    prob = SW.Slab(spec=sp, nx=12, order=2, limiter="minmod", collision="bgk")
    fj = np.repeat(profiles[0][:, None], sp.K, axis=1)
    assert np.all(SW.slopes(prob, fj)[1:-1, 0] == 0.0)
    fe = np.repeat(profiles[2][:, None], sp.K, axis=1)
    d = np.diff(profiles[2])
    assert np.allclose(SW.slopes(prob, fe)[1:-1, 0], np.minimum(d[1:], d[:-1]), rtol=0, atol=1e-15)
