"""SGS scans on a two-dimensional spatial domain (oracle; test infrastructure
only): the lid-driven cavity on [0, 1]^2 with diffuse walls, first-order
upwind finite volumes, two-dimensional velocities.

The paper extends its 1D method to two space dimensions (Section 3 remarks
that the extension is direct; Section 4.2 runs a lid-driven cavity).  For cell
(i, j) of an nx x ny grid the first-order upwind form of eq. fully_discrete is
  [v_1^+ (f_ij - f_{i-1,j}) + v_1^- (f_{i+1,j} - f_ij)] / dx
  + [v_2^+ (f_ij - f_{i,j-1}) + v_2^- (f_{i,j+1} - f_ij)] / dy = Q[f_ij] / eps.
A symmetric Gauss-Seidel iteration in 2D is four scans, each visiting the cells
in lexicographic order along one pair of axis directions:
(+x, +y), (-x, -y), (-x, +y), (+x, -y).  Within a scan a visit uses the latest
values of the four neighbours; the collision split P = Q - nu (M - f) of
eq. Pf is evaluated from the iterate before the scan, and the visit solves
eq. inner_eqn with the upwind diagonal c = |v_1|/dx + |v_2|/dy.

Readings, as in the 1D oracle: the ghost value at a diffuse wall is rho_w M_w
on the incoming half-space, with rho_w from the discrete zero-mass-flux balance
against the adjacent cell's latest value; the total mass is restored by a
uniform rescale after each full iteration; the outer residual is the L2(Omega x
R^d) norm sqrt(dx dy sum w R^2).

Second order (order = 2) applies the linear reconstruction of eqs.
reconstruction and slope along each axis: slopes s^x, s^y centred inside and
one-sided at the first and last cell of each line, zero in the ghosts, taken
from the iterate before each scan.  The face values f -+ s/2 enter the fluxes,
so a visit's right-hand side gains the static terms
  -(v1+ s^x_{i-1} - v1 s^x_i + v1- s^x_{i+1}) / (2 dx) - (same along y) / (2 dy),
and a wall's density balances the outgoing flux of the adjacent face value.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cell as cellmod
from .collision import bgk_nu_of, nu_of, penalty_split, q_corrected, q_fsm
from .grid import Spec, phi_vectors, velocity_nodes
from .maxwellian import discrete_maxwellian

SCANS = ((1, 1), (-1, -1), (-1, 1), (1, -1))


@dataclass
class Cavity:
    spec: Spec  # d = 2
    nx: int
    ny: int
    eps: float = 0.1
    # diffuse walls x = 0, x = 1, y = 0, y = 1: (T, (U_1, U_2)), velocity tangential
    walls: tuple = ((1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.5, 0.0)))
    mass: float = 1.0
    collision: str = "binary"  # "binary" (mass-projected corrected Q) or "bgk"
    q_method: str = "sigma"  # binary: "sigma" (collision.q_fsm) or "carleman" (carleman.q_carleman_2d, gamma = 0)
    bgk_nu: float | None = None
    inner: str = "pfp"
    tol_inner: float = 1e-8
    max_inner: int = 100
    fixed_inner: int | None = None
    fallback: str = "fp"  # inner solve when eq. existence fails: "fp" or "relax" (cell.solve)
    order: int = 1
    limiter: str = "none"  # second order: "none" (eq. slope) or "minmod" along each axis
    # uniform_y: the problem does not vary along y (ny = 1): no y transport and no
    # y walls, two scans (+x, -x) per iteration, multigrid coarsens x only.  This
    # is the 1D slab between two plates with 2D velocities.
    uniform_y: bool = False
    # learned warm start: (flat parameters, n_in, hidden, n_out, output scale) of
    # the network of oracle.mlp, or None for the plain start g0 = f_ij
    warm: tuple | None = None
    stats: dict = field(default_factory=lambda: {"inner": 0, "fallback": 0, "visits": 0, "learned": 0})

    @property
    def dx(self) -> float:
        return 1.0 / self.nx

    @property
    def dy(self) -> float:
        return 1.0 / self.ny


def wall_maxwellian(spec: Spec, T: float, U) -> np.ndarray:
    """Unit-density Maxwellian (2 pi T)^{-1} exp(-|v - U|^2 / 2T) at the nodes."""
    v = velocity_nodes(spec)
    return (2.0 * np.pi * T) ** -1.0 * np.exp(-((v - np.asarray(U)) ** 2).sum(1) / (2.0 * T))


def ghost(prob: Cavity, side: int, f_adj: np.ndarray) -> np.ndarray:
    """rho_w M_w for wall `side` (0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1), with
    rho_w balancing the outgoing flux of the adjacent cell's f_adj."""
    v = velocity_nodes(prob.spec)
    T, U = prob.walls[side]
    Mw = wall_maxwellian(prob.spec, T, U)
    vn = v[:, side // 2] * (1.0 if side % 2 == 0 else -1.0)  # velocity along the inward normal
    rho_w = np.sum(np.where(vn < 0, -vn, 0.0) * f_adj) / np.sum(np.where(vn > 0, vn, 0.0) * Mw)
    return rho_w * Mw


def slopes(prob: Cavity, f: np.ndarray):
    """(s^x, s^y) of eq. slope along each axis: centred inside, one-sided at the
    ends of each line; zeros at first order; minmod inside with limiter="minmod"."""
    from .sweep import minmod

    sx, sy = np.zeros_like(f), np.zeros_like(f)
    if prob.order == 1:
        return sx, sy
    lim = prob.limiter == "minmod"
    if prob.nx > 1:
        sx[0], sx[-1] = f[1] - f[0], f[-1] - f[-2]
        sx[1:-1] = minmod(f[2:] - f[1:-1], f[1:-1] - f[:-2]) if lim else 0.5 * (f[2:] - f[:-2])
    if prob.ny > 1:
        sy[:, 0], sy[:, -1] = f[:, 1] - f[:, 0], f[:, -1] - f[:, -2]
        sy[:, 1:-1] = minmod(f[:, 2:] - f[:, 1:-1], f[:, 1:-1] - f[:, :-2]) if lim else 0.5 * (f[:, 2:] - f[:, :-2])
    return sx, sy


def scans(prob: Cavity):
    return SCANS[:2] if prob.uniform_y else SCANS


def neighbours(prob: Cavity, f: np.ndarray, i: int, j: int, sx=None, sy=None):
    """(west, east, south, north) values for cell (i, j): cells or wall ghosts;
    a wall balances the flux of the adjacent face value f -+ s/2."""
    hx = 0.0 if sx is None else 0.5 * sx[i, j]
    hy = 0.0 if sy is None else 0.5 * sy[i, j]
    W = f[i - 1, j] if i > 0 else ghost(prob, 0, f[i, j] - hx)
    E = f[i + 1, j] if i < prob.nx - 1 else ghost(prob, 1, f[i, j] + hx)
    if prob.uniform_y:
        return W, E, None, None
    S = f[i, j - 1] if j > 0 else ghost(prob, 2, f[i, j] - hy)
    N = f[i, j + 1] if j < prob.ny - 1 else ghost(prob, 3, f[i, j] + hy)
    return W, E, S, N


def collision_terms(prob: Cavity, f_ij: np.ndarray):
    """(Q, M, nu): the mass-projected corrected Q (binary) or nu (M - f) (BGK)."""
    spec = prob.spec
    M, theta = discrete_maxwellian(spec, f_ij, return_theta=True)
    if prob.collision == "bgk":
        nu = prob.bgk_nu if prob.bgk_nu is not None else bgk_nu_of(spec, f_ij)
        return nu * (M - f_ij), M, nu
    if prob.q_method == "carleman":
        from .carleman import q_carleman_2d as op
    else:
        op = q_fsm
    return q_corrected(spec, f_ij, M, op=op, conserve="mass"), M, nu_of(spec, f_ij, theta)


def all_collision(prob: Cavity, f: np.ndarray):
    Q, M = np.empty_like(f), np.empty_like(f)
    nu = np.empty((prob.nx, prob.ny))
    for i in range(prob.nx):
        for j in range(prob.ny):
            Q[i, j], M[i, j], nu[i, j] = collision_terms(prob, f[i, j])
    return Q, M, nu


def transport_terms(prob: Cavity, f: np.ndarray, i: int, j: int, slx, sly) -> np.ndarray:
    """The transport part of a visit's right-hand side for cell (i, j): the
    upwind neighbour terms (cells or wall ghosts) of f and, at second order, the
    static reconstruction terms of the slopes (slx, sly)."""
    v = velocity_nodes(prob.spec)
    v1p, v1m = np.maximum(v[:, 0], 0.0), np.minimum(v[:, 0], 0.0)
    v2p, v2m = np.maximum(v[:, 1], 0.0), np.minimum(v[:, 1], 0.0)
    zero = np.zeros(prob.spec.K)
    W, E, S, N = neighbours(prob, f, i, j, slx, sly)
    r = (-v1p * W + v1m * E) / prob.dx
    if not prob.uniform_y:
        r = r + (-v2p * S + v2m * N) / prob.dy
    if prob.order == 2:
        xw = slx[i - 1, j] if i > 0 else zero
        xe = slx[i + 1, j] if i < prob.nx - 1 else zero
        ys = sly[i, j - 1] if j > 0 else zero
        yn = sly[i, j + 1] if j < prob.ny - 1 else zero
        r -= (v1p * xw - v[:, 0] * slx[i, j] + v1m * xe) / (2.0 * prob.dx)
        if not prob.uniform_y:
            r -= (v2p * ys - v[:, 1] * sly[i, j] + v2m * yn) / (2.0 * prob.dy)
    return r


def transport_part(prob: Cavity, f: np.ndarray) -> np.ndarray:
    """transport_terms of every cell with all neighbours (and the wall ghosts)
    from f: what a visit's r would be, less -P/eps, if no neighbour had been
    updated yet."""
    slx, sly = slopes(prob, f)
    T = np.empty_like(f)
    for i in range(prob.nx):
        for j in range(prob.ny):
            T[i, j] = transport_terms(prob, f, i, j, slx, sly)
    return T


def warm_candidates(prob: Cavity, f: np.ndarray):
    """Learned candidates of a scan (not part of the paper's method): before the
    scan every cell gets G_ij = M[f_ij] + scale * y_ij, y_ij the network's output
    for the features (oracle.mlp.features: the transport part of f times dx, the
    moments of M[f_ij], log10 eps; K + 5 inputs with two velocity dimensions)."""
    from . import mlp as mlpmod

    spec = prob.spec
    params, n_in, H, n_out, scale = prob.warm
    T = transport_part(prob, f)
    G = np.empty_like(f)
    for i in range(prob.nx):
        for j in range(prob.ny):
            Mf, th = discrete_maxwellian(spec, f[i, j], return_theta=True)
            x = mlpmod.features(spec, T[i, j], th, prob.eps, prob.dx)
            y, _ = mlpmod.forward(params, x[None, :], n_in, H, n_out)
            G[i, j] = Mf + scale * y[0]
    return G


def warm_choice(prob: Cavity, g: np.ndarray, G: np.ndarray, r: np.ndarray, nu: float) -> bool:
    """The visit starts from G instead of g when M[G] exists, the preconditioned
    step 1 from G is solvable (eq. existence) and G's inner residual
    |c G + r - (nu/eps)(M[G] - G)| with the visit's own r (fresh neighbours
    included) is below g's."""
    spec = prob.spec
    dxs = prob.dx if prob.uniform_y else (prob.dx, prob.dy)
    c = cellmod.transport_coef(spec, dxs)
    lam = nu / prob.eps
    try:
        MG = discrete_maxwellian(spec, G)
    except RuntimeError:
        return False
    phi = phi_vectors(spec)
    if not cellmod.existence_ok(spec, spec.w * phi.T @ (c * (MG - G) - r)):
        return False
    Mg = discrete_maxwellian(spec, g)
    res_g = np.sum((c * g + r - lam * (Mg - g)) ** 2)
    res_G = np.sum((c * G + r - lam * (MG - G)) ** 2)
    return bool(res_G < res_g)


def scan(prob: Cavity, f: np.ndarray, sx: int, sy: int, b: np.ndarray | None = None) -> np.ndarray:
    spec = prob.spec
    Q, M, nu = all_collision(prob, f)
    P = penalty_split(Q, M, f, nu)
    slx, sly = slopes(prob, f)
    G = warm_candidates(prob, f) if prob.warm is not None else None
    f = f.copy()
    for i in (range(prob.nx) if sx > 0 else range(prob.nx - 1, -1, -1)):
        for j in (range(prob.ny) if sy > 0 else range(prob.ny - 1, -1, -1)):
            r = transport_terms(prob, f, i, j, slx, sly)
            r -= P[i, j] / prob.eps
            if b is not None:
                r -= b[i, j]
            dxs = prob.dx if prob.uniform_y else (prob.dx, prob.dy)
            g0 = f[i, j]
            if G is not None and warm_choice(prob, f[i, j], G[i, j], r, nu[i, j]):
                g0 = G[i, j]
                prob.stats["learned"] = prob.stats.get("learned", 0) + 1
            g, st = cellmod.solve(spec, r, nu[i, j], prob.eps, dxs, g0, mode=prob.inner,
                                  tol=prob.tol_inner, max_iter=prob.max_inner, fixed_iters=prob.fixed_inner,
                                  fallback=prob.fallback)
            prob.stats["relaxed"] = prob.stats.get("relaxed", 0) + st.relaxed
            prob.stats["inner"] += st.iterations
            prob.stats["fallback"] += int(st.fallback)
            prob.stats["visits"] += 1
            f[i, j] = g
    return f


def total_mass(prob: Cavity, f: np.ndarray) -> float:
    return float(prob.dx * prob.dy * prob.spec.w * np.sum(f))


def sgs_iteration(prob: Cavity, f: np.ndarray, b: np.ndarray | None = None, rescale: bool = True) -> np.ndarray:
    for sx, sy in scans(prob):
        f = scan(prob, f, sx, sy, b)
    return f * (prob.mass / total_mass(prob, f)) if rescale else f


def residual_field(prob: Cavity, f: np.ndarray, Q: np.ndarray) -> np.ndarray:
    v = velocity_nodes(prob.spec)
    v1p, v1m = np.maximum(v[:, 0], 0.0), np.minimum(v[:, 0], 0.0)
    v2p, v2m = np.maximum(v[:, 1], 0.0), np.minimum(v[:, 1], 0.0)
    sx, sy = slopes(prob, f)
    R = np.empty_like(f)
    for i in range(prob.nx):
        for j in range(prob.ny):
            W, E, S, N = neighbours(prob, f, i, j, sx, sy)
            # face values: east/north faces f + s/2 and west/south faces f - s/2 of
            # each cell; ghosts carry no slope
            xw = 0.5 * sx[i - 1, j] if i > 0 else 0.0
            xe = 0.5 * sx[i + 1, j] if i < prob.nx - 1 else 0.0
            ys = 0.5 * sy[i, j - 1] if j > 0 else 0.0
            yn = 0.5 * sy[i, j + 1] if j < prob.ny - 1 else 0.0
            fe, fw = f[i, j] + 0.5 * sx[i, j], f[i, j] - 0.5 * sx[i, j]
            fn, fs = f[i, j] + 0.5 * sy[i, j], f[i, j] - 0.5 * sy[i, j]
            R[i, j] = (v1p * (fe - (W + xw)) + v1m * ((E - xe) - fw)) / prob.dx
            if not prob.uniform_y:
                R[i, j] += (v2p * (fn - (S + ys)) + v2m * ((N - yn) - fs)) / prob.dy
            R[i, j] -= Q[i, j] / prob.eps
    return R


def norm(prob: Cavity, R: np.ndarray) -> float:
    """sqrt(dx dy sum w R^2): the L2(Omega x R^d) norm of Section 4."""
    return float(np.sqrt(prob.dx * prob.dy * prob.spec.w * np.sum(R * R)))


def level_R(prob: Cavity, f: np.ndarray) -> np.ndarray:
    Q, _, _ = all_collision(prob, f)
    return residual_field(prob, f, Q)


def outer_residual(prob: Cavity, f: np.ndarray, b: np.ndarray | None = None) -> float:
    R = level_R(prob, f)
    return norm(prob, R if b is None else R - b)


# ---------------------------------------------------------------- multigrid
# The nonlinear multigrid of eq. coarse on the 2D grid, H = 2h in both
# directions, with the readings of the 1D oracle: restriction averages the four
# children, prolongation injects the coarse correction piecewise constantly,
# the coarsest level is smoothed until its residual falls 10x or coarse_iters
# iterations pass, and a V-cycle stops descending once a level's residual is
# below the outer tolerance.


def coarse(prob: Cavity) -> Cavity:
    return Cavity(**{k: getattr(prob, k) for k in prob.__dataclass_fields__ if k not in ("nx", "ny", "stats")},
                  nx=prob.nx // 2, ny=prob.ny if prob.uniform_y else prob.ny // 2)


def restrict(f: np.ndarray) -> np.ndarray:
    if f.shape[1] == 1:  # uniform in y: two children along x
        return 0.5 * (f[0::2] + f[1::2])
    return 0.25 * (f[0::2, 0::2] + f[1::2, 0::2] + f[0::2, 1::2] + f[1::2, 1::2])


def prolong(e: np.ndarray) -> np.ndarray:
    if e.shape[1] == 1:
        return np.repeat(e, 2, axis=0)
    return np.repeat(np.repeat(e, 2, axis=0), 2, axis=1)


def vcycle(prob: Cavity, f: np.ndarray, b: np.ndarray | None, coarsest: int, nu1: int, nu2: int, tol: float,
           coarse_iters: int = 20) -> np.ndarray:
    """One FAS V-cycle for R_h(f) = b (eq. coarse); levels halve nx and ny until
    min(nx, ny) <= coarsest."""
    if b is None:
        b = np.zeros_like(f)
    for _ in range(nu1):
        f = sgs_iteration(prob, f, b, rescale=False)
    if (prob.nx if prob.uniform_y else min(prob.nx, prob.ny)) <= coarsest:
        r0 = norm(prob, b - level_R(prob, f))
        for _ in range(coarse_iters):
            if norm(prob, b - level_R(prob, f)) <= 0.1 * r0:
                break
            f = sgs_iteration(prob, f, b, rescale=False)
        return f
    res = b - level_R(prob, f)
    if norm(prob, res) < tol:
        return f
    cp = coarse(prob)
    fc0 = restrict(f)
    bc = level_R(cp, fc0) + restrict(res)
    fc = vcycle(cp, fc0.copy(), bc, coarsest, nu1, nu2, tol, coarse_iters)
    for k in ("inner", "visits", "fallback", "learned"):
        prob.stats[k] = prob.stats.get(k, 0) + cp.stats.get(k, 0)
    f = f + prolong(fc - fc0)
    for _ in range(nu2):
        f = sgs_iteration(prob, f, b, rescale=False)
    return f


def mg_iteration(prob: Cavity, f: np.ndarray, coarsest: int = 5, nu1: int = 1, nu2: int = 1,
                 tol: float = 1e-5) -> np.ndarray:
    """One V-cycle followed by the mass rescale (MG-SGS-PFP).  The defaults are
    the first-order 2D parameters of tab. mg (coarsest grid 5 x 5, one pre- and
    one post-smoothing step)."""
    f = vcycle(prob, f, None, coarsest, nu1, nu2, tol)
    return f * (prob.mass / total_mass(prob, f))


def initial_state(prob: Cavity, rho: float = 1.0, T: float = 1.0) -> np.ndarray:
    """Uniform Maxwellian at rest scaled to the total mass; shape [nx, ny, K]."""
    M = wall_maxwellian(prob.spec, T, (0.0, 0.0)) * rho
    f = np.broadcast_to(M, (prob.nx, prob.ny, prob.spec.K)).copy()
    return f * (prob.mass / total_mass(prob, f))
