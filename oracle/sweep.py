"""Spatial discretisation, SGS scans and the FAS multigrid V-cycle on a 1D slab
(oracle; test infrastructure only).

Section 2.1: upwind finite volumes (eq. upwind) with linear reconstruction
(eq. reconstruction) and slopes (eq. slope; zero slopes give first order).
Section 3.1/3.3: the SGS method (eqs. SGS_BGK and SGS) with the BGK-penalty
split P[f] = Q[f,f] - nu (M[f] - f) (eq. Pf) treated explicitly, each cell
visit solving eq. inner_eqn.  Section 4: diffuse walls (eq. boundary), the
total-mass constraint (eq. mass_conserv) enforced by a uniform rescale after
every iteration, the outer residual, and the nonlinear multigrid of
eq. coarse with H = 2h and the parameters of tab. mg.

Readings where the paper is silent (each stated in the design notes):
  * the wall density comes from the discrete zero-mass-flux balance on the grid
    rather than the continuous sqrt(2 pi / T) formula;
  * the wall-adjacent face value is the latest value of the adjacent cell
    (minus/plus half its slope at second order), and the ghost slope is 0;
  * the inner solve starts from the cell's current value;
  * the mass rescale happens after each full SGS iteration on the finest
    level, or after each V-cycle, never inside coarse-level smoothing;
  * restriction averages two children, prolongation injects the coarse
    correction piecewise-constantly, the coarsest level is smoothed until its
    residual drops 10x or 20 iterations pass, and a V-cycle stops descending
    once a level's residual is below the outer tolerance.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cell as cellmod
from .collision import bgk_nu_of, nu_of, penalty_split, q_corrected, q_fsm
from .grid import Spec, phi_vectors, sphere_area, transport_v1, velocity_nodes
from .maxwellian import discrete_maxwellian, moments


@dataclass
class Slab:
    spec: Spec
    nx: int
    xL: float = 0.0
    xR: float = 1.0
    T_L: float = 1.0
    T_R: float = 2.0
    U_L: tuple = (0.0, 0.0, 0.0)
    U_R: tuple = (0.0, 0.0, 0.0)
    eps: float = 0.1
    mass: float = 1.0
    bc_L: str = "wall"  # "wall": diffuse wall (eq. boundary); "inflow": given Maxwellian rho_L M(T_L, U_L)
    bc_R: str = "wall"
    rho_L: float = 1.0  # inflow densities (unused at walls)
    rho_R: float = 1.0
    order: int = 1
    limiter: str = "none"  # second order: "none" (eq. slope) or "minmod"
    collision: str = "binary"  # "binary" (Q^FSM with eq. discrete_Q) or "bgk" (P == 0)
    q_method: str = "sigma"  # binary: "sigma" (collision.q_fsm) or "carleman" (carleman.q_carleman, gamma = 1)
    conserve: str = "mass"  # binary: project Q onto zero mass ("mass") or all five invariants ("all")
    bgk_nu: float | None = None  # constant nu for "bgk"; None -> |S^{d-1}| rho
    inner: str = "pfp"
    tol_inner: float = 1e-8
    max_inner: int = 100
    fixed_inner: int | None = None
    # learned warm start: (flat parameters, n_in, hidden, n_out, output scale) of
    # the network of oracle.mlp, or None for the plain start g0 = f_j
    warm: tuple | None = None
    stats: dict = field(default_factory=lambda: {"inner": 0, "fallback": 0, "visits": 0, "learned": 0})

    @property
    def dx(self) -> float:
        return (self.xR - self.xL) / self.nx

    def coarse(self) -> "Slab":
        c = Slab(**{k: getattr(self, k) for k in self.__dataclass_fields__ if k not in ("nx", "stats")},
                 nx=self.nx // 2)
        return c


def wall_maxwellian(spec: Spec, T: float, U) -> np.ndarray:
    """Unit-density Maxwellian of eq. boundary at the grid nodes, U in physical velocity."""
    v = velocity_nodes(spec).copy()
    v[:, 0] += spec.v1_shift
    d = spec.d
    r2 = ((v - np.asarray(U[:d])) ** 2).sum(1)
    return (2.0 * np.pi * T) ** (-d / 2.0) * np.exp(-r2 / (2.0 * T))


def minmod(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """sign(a) min(|a|, |b|) where a and b agree in sign, else 0."""
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def slopes(prob: Slab, f: np.ndarray) -> np.ndarray:
    """eq. slope (one-sided at the ends, centred inside); zeros at first order.
    With limiter="minmod" the inside slopes are minmod(f_{j+1} - f_j, f_j - f_{j-1})
    (a nonlinear limiter, which the explicit treatment of the slopes in eq. SGS
    allows, Section 3.1); the end cells keep their one-sided differences."""
    s = np.zeros_like(f)
    if prob.order == 1 or prob.nx < 2:
        return s
    s[0] = f[1] - f[0]
    s[-1] = f[-1] - f[-2]
    if prob.limiter == "minmod":
        s[1:-1] = minmod(f[2:] - f[1:-1], f[1:-1] - f[:-2])
    else:
        s[1:-1] = 0.5 * (f[2:] - f[:-2])
    return s


def ghosts(prob: Slab, f: np.ndarray, s: np.ndarray):
    """Left/right ghost distributions.  At a diffuse wall rho_w M_w, with rho_w
    from the zero-mass-flux condition of eq. boundary (discrete flux balance on
    the grid, physical v_1); at an inflow boundary the given rho M(T, U)."""
    spec = prob.spec
    v1 = transport_v1(spec)
    ML = wall_maxwellian(spec, prob.T_L, prob.U_L)
    MR = wall_maxwellian(spec, prob.T_R, prob.U_R)
    if prob.bc_L == "inflow":
        rho_L = prob.rho_L
    else:
        face_L = f[0] - 0.5 * s[0]
        rho_L = np.sum(np.where(v1 < 0, -v1, 0.0) * face_L) / np.sum(np.where(v1 > 0, v1, 0.0) * ML)
    if prob.bc_R == "inflow":
        rho_R = prob.rho_R
    else:
        face_R = f[-1] + 0.5 * s[-1]
        rho_R = np.sum(np.where(v1 > 0, v1, 0.0) * face_R) / np.sum(np.where(v1 < 0, -v1, 0.0) * MR)
    return rho_L * ML, rho_R * MR


def collision_terms(prob: Slab, f_j: np.ndarray):
    """(Q, M, nu) for one cell: the steady-state preserving Q^FSM (eq. discrete_Q),
    projected (collision.mass_project, or conserve_project for conserve="all"), in
    binary mode, or nu (M - f) in BGK
    mode."""
    spec = prob.spec
    M, theta = discrete_maxwellian(spec, f_j, return_theta=True)
    if prob.collision == "bgk":
        nu = prob.bgk_nu if prob.bgk_nu is not None else bgk_nu_of(spec, f_j)
        return nu * (M - f_j), M, nu
    if prob.q_method == "carleman":
        from .carleman import q_carleman as op
    else:
        op = q_fsm
    return q_corrected(spec, f_j, M, op=op, conserve=prob.conserve), M, nu_of(spec, f_j, theta)


def residual_field(prob: Slab, f: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Discrete v.grad f - Q/eps per cell (eq. fully_discrete rearranged)."""
    spec = prob.spec
    v1 = transport_v1(spec)
    vp, vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
    s = slopes(prob, f)
    gl, gr = ghosts(prob, f, s)
    fe = np.concatenate([gl[None], f, gr[None]])
    se = np.concatenate([np.zeros_like(gl)[None], s, np.zeros_like(gr)[None]])
    minus = fe + 0.5 * se  # f^-_{j+1/2} = f_j + s_j/2 for j = 0..nx+1
    plus = fe - 0.5 * se  # f^+_{j-1/2} = f_j - s_j/2
    R = np.empty_like(f)
    for j in range(1, prob.nx + 1):
        R[j - 1] = (vp * (minus[j] - minus[j - 1]) + vm * (plus[j + 1] - plus[j])) / prob.dx - Q[j - 1] / prob.eps
    return R


def norm(prob: Slab, R: np.ndarray) -> float:
    """sqrt(sum_j dx sum_k w R^2): the L2(Omega x R^d) norm of Section 4."""
    return float(np.sqrt(prob.dx * prob.spec.w * np.sum(R * R)))


def all_collision(prob: Slab, f: np.ndarray):
    Q = np.empty_like(f)
    M = np.empty_like(f)
    nu = np.empty(prob.nx)
    for j in range(prob.nx):
        Q[j], M[j], nu[j] = collision_terms(prob, f[j])
    return Q, M, nu


def transport_part(prob: Slab, f: np.ndarray, s: np.ndarray | None = None) -> np.ndarray:
    """Transport part of the right-hand side r of eq. r for every cell, with both
    neighbours and the wall ghosts taken from f (and the slopes s of f): what a
    visit's r would be, less -P/eps, if no neighbour had been updated yet."""
    spec = prob.spec
    v1 = transport_v1(spec)
    vp, vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
    if s is None:
        s = slopes(prob, f)
    gl, gr = ghosts(prob, f, s)
    s_e = np.concatenate([np.zeros((1, spec.K)), s, np.zeros((1, spec.K))])
    T = np.empty_like(f)
    for j in range(prob.nx):
        left = f[j - 1] if j > 0 else gl
        right = f[j + 1] if j < prob.nx - 1 else gr
        T[j] = (-vp * left + vm * right) / prob.dx - (vp * s_e[j] - v1 * s_e[j + 1] + vm * s_e[j + 2]) / (2.0 * prob.dx)
    return T


def warm_starts(prob: Slab, f: np.ndarray, P: np.ndarray, nu: np.ndarray, b: np.ndarray | None):
    """Initial guesses of a scan's visits with the learned warm start (not part of
    the paper's method; it changes only where each inner iteration starts).

    Before the scan, every cell gets a second candidate G_j = M[f_j] + scale * y_j,
    y_j the network's output for the features of the cell's transport part with
    both neighbours taken from the iterate before the scan (oracle.mlp.features).
    The visit starts from G_j when the preconditioned step 1 from G_j is
    solvable (eq. existence for the right-hand side below) and its inner residual
        |c g + r_old - (nu/eps)(M[g] - g)|_{L2}
    is smaller than that of f_j, where r_old is the visit's right-hand side with
    the upwind neighbour taken from the iterate before the scan (the fresh one is
    not known yet), i.e. the transport part minus P/eps (minus the FAS source)."""
    from . import mlp as mlpmod

    spec = prob.spec
    params, n_in, H, n_out, scale = prob.warm
    T = transport_part(prob, f)
    c = cellmod.transport_coef(spec, prob.dx)
    phi = phi_vectors(spec)
    lam = nu / prob.eps
    out = []
    for j in range(prob.nx):
        Mf, th = discrete_maxwellian(spec, f[j], return_theta=True)
        x = mlpmod.features(spec, T[j], th, prob.eps, prob.dx)
        y, _ = mlpmod.forward(params, x[None, :], n_in, H, n_out)
        G = Mf + scale * y[0]
        r_old = T[j] - P[j] / prob.eps - (b[j] if b is not None else 0.0)
        res_f = np.sum((c * f[j] + r_old - lam[j] * (Mf - f[j])) ** 2)
        try:
            MG = discrete_maxwellian(spec, G)
        except RuntimeError:
            out.append(None)
            continue
        # the preconditioned step 1 from G must be solvable (eq. existence)
        if not cellmod.existence_ok(spec, spec.w * phi.T @ (c * (MG - G) - r_old)):
            out.append(None)
            continue
        res_G = np.sum((c * G + r_old - lam[j] * (MG - G)) ** 2)
        out.append(G if res_G < res_f else None)
    return out


def scan(prob: Slab, f: np.ndarray, forward: bool, b: np.ndarray | None = None, lagged=None) -> np.ndarray:
    """One SGS scan (the first or second line of eq. SGS): P and nu from the iterate
    before the scan, slopes from the previous scan, cells visited in order.

    With lagged = (M, nu) (source iteration, BGK only) each visit makes the single
    update g = (|v_1|/dx + nu/eps)^{-1} ((nu/eps) M_j - r) with M and nu taken from
    the iterate at the start of the iteration, eq. SI: the scan then solves the
    transport equation of the velocities it sweeps along exactly."""
    spec = prob.spec
    v1 = transport_v1(spec)
    vp, vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
    dx, eps = prob.dx, prob.eps
    if lagged is not None:
        M, nu = lagged
        Q = nu[:, None] * (M - f)  # BGK: P = 0
    else:
        Q, M, nu = all_collision(prob, f)
    P = penalty_split(Q, M, f, nu)
    s = slopes(prob, f)
    warm = warm_starts(prob, f, P, nu, b) if prob.warm is not None else [None] * prob.nx
    f = f.copy()
    order = range(prob.nx) if forward else range(prob.nx - 1, -1, -1)
    for j in order:
        s_e = np.concatenate([np.zeros((1, spec.K)), s, np.zeros((1, spec.K))])
        if j == 0 or j == prob.nx - 1:
            gl, gr = ghosts(prob, f, s)
        left = f[j - 1] if j > 0 else gl
        right = f[j + 1] if j < prob.nx - 1 else gr
        r = (-vp * left + vm * right) / dx
        r -= (vp * s_e[j] - v1 * s_e[j + 1] + vm * s_e[j + 2]) / (2.0 * dx)
        r -= P[j] / eps
        if b is not None:
            r -= b[j]
        if lagged is not None:
            lam = nu[j] / eps
            f[j] = (lam * M[j] - r) / (cellmod.transport_coef(spec, dx) + lam)
            prob.stats["inner"] += 1
            prob.stats["visits"] += 1
            continue
        g0 = f[j] if warm[j] is None else warm[j]
        g, st = cellmod.solve(spec, r, nu[j], eps, dx, g0, mode=prob.inner, tol=prob.tol_inner,
                              max_iter=prob.max_inner, fixed_iters=prob.fixed_inner)
        prob.stats["learned"] = prob.stats.get("learned", 0) + int(warm[j] is not None)
        prob.stats["inner"] += st.iterations
        prob.stats["fallback"] += int(st.fallback)
        prob.stats["visits"] += 1
        f[j] = g
    return f


def total_mass(prob: Slab, f: np.ndarray) -> float:
    return float(prob.dx * prob.spec.w * np.sum(f))


def sgs_iteration(prob: Slab, f: np.ndarray, b: np.ndarray | None = None, rescale: bool = True):
    """One iteration: a forward and a backward scan (eq. SGS), then the mass rescale.
    With inner = "si" it is the source iteration of eq. SI (BGK): M[f^n] and nu^n
    are lagged over both scans, each visit one explicit update."""
    if prob.inner == "si":
        if prob.collision != "bgk":
            raise ValueError("the source iteration is the BGK scheme of eq. SI")
        _, M, nu = all_collision(prob, f)
        f = scan(prob, f, True, b, lagged=(M, nu))
        f = scan(prob, f, False, b, lagged=(M, nu))
    else:
        f = scan(prob, f, True, b)
        f = scan(prob, f, False, b)
    if rescale:
        f = f * (prob.mass / total_mass(prob, f))
    return f


def outer_residual(prob: Slab, f: np.ndarray, b: np.ndarray | None = None) -> float:
    Q, _, _ = all_collision(prob, f)
    R = residual_field(prob, f, Q)
    if b is not None:
        R = R - b
    return norm(prob, R)


def solve_sgs(prob: Slab, f0: np.ndarray, tol: float = 1e-5, max_iter: int = 1000):
    """Plain SGS iteration to the outer tolerance.  Returns (f, residual history)."""
    f = f0.copy()
    hist = []
    for _ in range(max_iter):
        res = outer_residual(prob, f)
        hist.append(res)
        if res < tol:
            break
        f = sgs_iteration(prob, f)
    return f, hist


# ---------------------------------------------------------------- multigrid


def restrict(f: np.ndarray) -> np.ndarray:
    """Average of two children (H = 2h)."""
    return 0.5 * (f[0::2] + f[1::2])


def prolong(e: np.ndarray) -> np.ndarray:
    """Piecewise-constant injection of a coarse correction."""
    return np.repeat(e, 2, axis=0)


def level_R(prob: Slab, f: np.ndarray) -> np.ndarray:
    Q, _, _ = all_collision(prob, f)
    return residual_field(prob, f, Q)


def vcycle(prob: Slab, f: np.ndarray, b: np.ndarray | None, coarsest: int, nu1: int, nu2: int,
           tol: float, coarse_iters: int = 20, fixed: bool = False):
    """One FAS V-cycle for R_h(f) = b (eq. coarse).  The coarsest level is
    smoothed until its residual falls tenfold or coarse_iters iterations pass,
    and a level whose residual is below tol does not descend; with fixed = True
    neither exit is taken (every level descends, the coarsest level runs
    exactly coarse_iters iterations)."""
    if b is None:
        b = np.zeros_like(f)
    for _ in range(nu1):
        f = sgs_iteration(prob, f, b, rescale=False)
    if prob.nx <= coarsest:
        r0 = norm(prob, b - level_R(prob, f))
        for _ in range(coarse_iters):
            if not fixed and norm(prob, b - level_R(prob, f)) <= 0.1 * r0:
                break
            f = sgs_iteration(prob, f, b, rescale=False)
        return f
    res = b - level_R(prob, f)
    if not fixed and norm(prob, res) < tol:
        return f
    cp = prob.coarse()
    fc0 = restrict(f)
    bc = level_R(cp, fc0) + restrict(res)
    fc = vcycle(cp, fc0.copy(), bc, coarsest, nu1, nu2, tol, coarse_iters, fixed)
    prob.stats["inner"] += cp.stats["inner"]
    prob.stats["visits"] += cp.stats["visits"]
    prob.stats["fallback"] += cp.stats["fallback"]
    f = f + prolong(fc - fc0)
    for _ in range(nu2):
        f = sgs_iteration(prob, f, b, rescale=False)
    return f


def solve_mg(prob: Slab, f0: np.ndarray, coarsest: int = 4, nu1: int = 1, nu2: int = 1, tol: float = 1e-5,
             max_cycles: int = 200):
    """MG-SGS-PFP: V-cycles with a mass rescale after each."""
    f = f0.copy()
    hist = []
    for _ in range(max_cycles):
        res = outer_residual(prob, f)
        hist.append(res)
        if res < tol:
            break
        f = vcycle(prob, f, None, coarsest, nu1, nu2, tol)
        f = f * (prob.mass / total_mass(prob, f))
    return f, hist


def initial_state(prob: Slab, rho: float = 1.0, T: float = 1.0) -> np.ndarray:
    """Uniform Maxwellian scaled to the total mass C."""
    spec = prob.spec
    M = wall_maxwellian(spec, T, (0.0,) * spec.d) * rho
    f = np.repeat(M[None], prob.nx, axis=0)
    return f * (prob.mass / total_mass(prob, f))
