"""Inner (per-cell) nonlinear problem and its iterations (oracle; test
infrastructure only).

eq. inner_eqn:  (|v_1|/dx) g + r = (nu/eps) (M[g] - g)  for the unknown g.
  * FP  (eq. fix_point):  g <- D^{-1} ((nu/eps) M[g] - r),  D = |v_1|/dx + nu/eps.
  * PFP (eqs. step1, step2): step 1 finds the Gaussian M' with
        sum w phi (|v_1|/dx) M' = sum w phi ((|v_1|/dx)(M[g] - g) - r),
    step 2 sets g <- D^{-1} ((nu/eps) M' - r).  Step 1 is solvable only if the
    right-hand side s satisfies eq. existence (s_0 > 0, s_0 s_{d+1} > sum s_i^2);
    otherwise the visit continues with FP (Section 3.2).  The alternative of the
    remark in Section 3.2 (fallback="relax") revises step 1 with a relaxation
    factor tau: its right-hand side becomes
        s_tau = sum w phi (c ((1 + tau) M[g] - g) - r) / (1 + tau),
    which is s at tau = 0 and tends to the moments of c M[g] (the plain
    iteration) as tau grows.  Reading: each update takes the smallest tau in
    {0, 1, 2, 4, ..., 2^20} whose s_tau satisfies eq. existence.
  * The residual |(|v_1|/dx) g + r - (nu/eps)(M[g] - g)|_{L2(R^d)} stops both
    (Section 4, tolerance 1e-8).  It is evaluated after every update.
  * ``theta_solve`` finds the fixed point independently: since M[g] depends
    on g only through its moments, g* = D^{-1}((nu/eps) M_theta - r) where theta
    solves sum w phi [D^{-1}((nu/eps) M_theta - r) - M_theta] = 0 (Newton).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .grid import Spec, phi_vectors, transport_v1, velocity_nodes
from .maxwellian import discrete_maxwellian, gaussian, moments, solve_weighted_gaussian, theta_from_macro


def transport_coef(spec: Spec, dx) -> np.ndarray:
    """c_k = |v_{k,1}| / dx with the physical v_1 (velocity axis 0, the slowest array
    axis).  In two space dimensions dx is the pair (dx, dy) and the upwind
    diagonal is c_k = |v_{k,1}| / dx + |v_{k,2}| / dy."""
    if isinstance(dx, tuple):
        v = velocity_nodes(spec)
        return np.abs(v[:, 0]) / dx[0] + np.abs(v[:, 1]) / dx[1]
    return np.abs(transport_v1(spec)) / dx


def inner_residual(spec: Spec, g, r, nu, eps, dx, Mg=None) -> float:
    """L2(R^d) norm of (|v_1|/dx) g + r - (nu/eps)(M[g] - g) with weight w."""
    if Mg is None:
        Mg = discrete_maxwellian(spec, g)
    c = transport_coef(spec, dx)
    res = c * g + r - (nu / eps) * (Mg - g)
    return float(np.sqrt(spec.w * np.sum(res * res)))


@dataclass
class SolveStats:
    iterations: int = 0
    fallback: bool = False
    residual: float = np.inf
    history: list = None
    relaxed: int = 0  # updates whose step 1 used the relaxation factor


def existence_ok(spec: Spec, s: np.ndarray) -> bool:
    """eq. existence: s_0 > 0 and s_0 s_{d+1} > sum_i s_i^2."""
    return bool(s[0] > 0.0 and s[0] * s[-1] > np.sum(s[1:-1] ** 2))


def solve(spec: Spec, r, nu, eps, dx, g0, mode: str = "pfp", tol: float = 1e-8, max_iter: int = 100,
          fixed_iters: int | None = None, fallback: str = "fp"):
    """Iterate FP or PFP from g0.  With ``fixed_iters`` exactly that many updates are
    made (tolerance ignored), for one-to-one comparisons of iterates.  fallback:
    "fp" (continue the visit with FP when eq. existence fails) or "relax" (the
    relaxed step 1 described above; FP only if its Newton fails)."""
    c = transport_coef(spec, dx)
    lam = nu / eps
    D = c + lam
    phi = phi_vectors(spec)
    g = np.array(g0, dtype=np.float64)
    Mg, th_g = discrete_maxwellian(spec, g, return_theta=True)
    theta_step = th_g.copy()
    st = SolveStats(history=[], relaxed=0)
    relax = fallback == "relax"
    fallback = mode == "fp"
    n = fixed_iters if fixed_iters is not None else max_iter
    for k in range(n):
        if not fallback:
            s = spec.w * phi.T @ (c * (Mg - g) - r)
            ok = existence_ok(spec, s)
            if not ok and relax:
                cM = spec.w * phi.T @ (c * Mg)
                tau = 1.0
                while tau <= 2.0 ** 20:
                    s_tau = (s + tau * cM) / (1.0 + tau)
                    if existence_ok(spec, s_tau):
                        s, ok = s_tau, True
                        st.relaxed += 1
                        break
                    tau *= 2.0
            if ok:
                th, _, conv = solve_weighted_gaussian(spec, s, weight=c, theta0=theta_step)
                ok = conv and th[-1] > 0.0
            if ok:
                theta_step = th
                Mstep = gaussian(spec, th)
            else:
                fallback = True
                st.fallback = True
        if fallback:
            Mstep = Mg
        g = (lam * Mstep - r) / D
        Mg, th_g = discrete_maxwellian(spec, g, return_theta=True)
        res = float(np.sqrt(spec.w * np.sum((c * g + r - lam * (Mg - g)) ** 2)))
        st.history.append(res)
        st.iterations = k + 1
        st.residual = res
        if fixed_iters is None and res <= tol:
            break
    return g, st


def theta_solve(spec: Spec, r, nu, eps, dx, theta0=None, tol: float = 1e-14, max_iter: int = 100):
    """Fixed point of eq. inner_eqn by Newton in the Maxwellian parameters (independent
    of the FP/PFP iterations).  Returns g*."""
    c = transport_coef(spec, dx)
    lam = nu / eps
    D = c + lam
    phi = phi_vectors(spec)
    v = velocity_nodes(spec)
    pt = phi.copy()
    pt[:, -1] *= -1.0
    if theta0 is None:
        # start from the Maxwellian of the eps -> 0 limit guess g ~ -r/c balanced: use moments of |r|
        m = moments(spec, np.abs(r) / (c + lam) + 1e-300)
        rho = m[0]
        U = m[1 : 1 + spec.d] / rho
        T = max((m[-1] / rho - U @ U) / spec.d, 0.1)
        theta = theta_from_macro(spec, rho, U, T)
    else:
        theta = np.array(theta0, dtype=np.float64)

    def F(th):
        Mt = np.exp(th[0] + v @ th[1 : 1 + spec.d] - th[-1] * (v * v).sum(1))
        return spec.w * phi.T @ ((lam * Mt - r) / D - Mt), Mt

    Fv, Mt = F(theta)
    for _ in range(max_iter):
        scale = spec.w * np.sum(np.abs(phi.T @ Mt), axis=None) + 1e-300
        if np.max(np.abs(Fv)) <= tol * scale:
            break
        J = spec.w * (phi * ((lam / D - 1.0) * Mt)[:, None]).T @ pt
        step = np.linalg.solve(J, -Fv)
        t = 1.0
        n0 = np.max(np.abs(Fv))
        while True:
            F1, M1 = F(theta + t * step)
            if np.isfinite(F1).all() and np.max(np.abs(F1)) < n0 and theta[-1] + t * step[-1] > 0:
                break
            t *= 0.5
            if t < 1e-8:
                break
        theta = theta + t * step
        Fv, Mt = F1, M1
    return (lam * Mt - r) / D, theta
