"""Training data, training and time-to-residual runs of the learned warm start.

Every step of the method runs in libbz through the C ABI: the slab scans and
V-cycles that produce the training states, the transport part of eq. r of
each cell (bz_slab_inflow), the cell solves that give the targets
(bz_cell_fixed_point to a tight tolerance), the discrete Maxwellians, the
feature map, the MLP forward/backward/Adam kernels, and the learned start
inside the scans (bz_ws_attach).  This module moves tensors between those
calls and keeps the books.

Family (heat slabs between plates): x in [0, 1], nx cells, diffuse walls at
rest with T_L = 1 and T_R ~ U(1.5, 2.5), eps log-uniform in [0.005, 1], total
mass 1, initial state the Maxwellian u = 0, T = 1.5; instance i draws from
numpy.random.default_rng([seed, i]).

Training pairs come from the solver's own iterates: the states after V-cycles
0, 1, ..., n_snap - 1 of each training instance.  (Two-dimensional cavities,
below, take the state after the next V-cycle as the target, since the library
has no single-cell solve with two-dimensional velocities.)  For each cell of a state the
input is the network's feature row of the cell's transport part (both
neighbours from that state) and the target is g* - M[f_j], g* the solution
of the cell's inner problem with that transport part (the visit the learned
start stands in for), divided by the output scale.
"""
from __future__ import annotations

import time

import numpy as np

from . import Cavity, Context, MLP, Slab


def heat_slab_instance(seed: int, i: int, nx: int):
    rng = np.random.default_rng([seed, i])
    T_R = float(rng.uniform(1.5, 2.5))
    eps = float(np.exp(rng.uniform(np.log(0.005), np.log(1.0))))
    return dict(nx=nx, eps=eps, T_L=1.0, T_R=T_R, mass=1.0)


def initial_field(ctx: Context, nx: int, T0: float = 1.5):
    """Uniform Maxwellian u = 0, T = T0 of total mass 1 on [0, 1] (input data)."""
    import torch

    import synth

    N, L = ctx.params.N, ctx.params.L
    m = synth.maxwellian_mixture([(1.0, np.zeros(3), T0)], N, L)
    f0 = np.repeat(m[None], nx, axis=0)
    f0 *= 1.0 / ((1.0 / nx) * (2.0 * L / N) ** 3 * f0.sum())
    return torch.from_numpy(f0).to(f"cuda:{ctx.params.device}").contiguous()


MG = dict(coarsest=4, nu1=1, nu2=1, coarse_iters=20)


def sweep_dataset(ctx: Context, instances, n_snap: int = 4, tol: float = 1e-10):
    """Features X [n, K + 6] (float32) and targets g* - M[f_old] [n, K] (float32)
    from the states of V-cycles 0 .. n_snap - 1 of every instance; cells whose
    inner solve did not reach tol are left out.  Returns (X, Y, info)."""
    import torch

    Xs, Ys, dropped, t0 = [], [], 0, time.perf_counter()
    for d in instances:
        f = initial_field(ctx, d["nx"])
        slab = Slab(ctx, [d], f)
        dx = 1.0 / d["nx"]
        eps = torch.full((d["nx"],), d["eps"], dtype=torch.float64, device=f.device)
        for k in range(n_snap):
            if k > 0:
                slab.vcycle(1, tol=1e-8, **MG)
            T = slab.inflow()
            theta, M, _ = ctx.maxwellian(f)
            X = ctx.features(T, theta, eps, dx)
            g, st = ctx.cell_fixed_point(f, T, eps, dx, tol=tol, max_iter=400)
            ok = torch.from_numpy(ctx.decode_stats(st)["status"] == 0).to(f.device) & torch.isfinite(g).all(1)
            dropped += int((~ok).sum().item())
            Xs.append(X[ok])
            Ys.append((g - M)[ok].to(torch.float32))
        slab.close()
    X, Y = torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous()
    return X, Y, {"samples": int(X.shape[0]), "dropped": dropped, "seconds": time.perf_counter() - t0}


def train(ctx: Context, X, Y, hidden: int = 256, epochs: int = 20, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Train the MLP on standardised features and scaled targets with the
    library's own kernels; the standardisation is folded into the first layer
    afterwards, so inference takes the raw feature map."""
    import torch

    y_scale = float(torch.sqrt((Y.double() ** 2).mean()).item()) or 1.0
    T = (Y / y_scale).contiguous()
    mu = X.double().mean(0)
    sd = X.double().std(0)
    floor = 1e-3 * float(sd.max().item())
    sd = torch.where(sd > floor, sd, torch.ones_like(sd))
    Xn = ((X.double() - mu) / sd).to(torch.float32).contiguous()
    mlp = MLP(ctx, X.shape[1], hidden, Y.shape[1], seed=seed)
    mlp.set_output_scale(y_scale)
    n = X.shape[0]
    batch = min(batch, n)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    history = []
    probe = min(n, 1024)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(X.device)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            mlp.train_step(Xn[idx].contiguous(), T[idx].contiguous(), lr)
        loss, _ = mlp.grad(Xn[:probe].contiguous(), T[:probe].contiguous())
        history.append(loss)
        if log:
            log(f"epoch {ep} loss {loss:.4e}")
    # fold x -> (x - mu) / sd into W1, b1
    p = mlp.get_params().astype(np.float64)
    I, H = X.shape[1], hidden
    W1 = p[: I * H].reshape(I, H)
    b1 = p[I * H: I * H + H]
    mu_n, sd_n = mu.cpu().numpy(), sd.cpu().numpy()
    b1 -= (mu_n / sd_n) @ W1
    W1 /= sd_n[:, None]
    mlp.set_params(p.astype(np.float32))
    return mlp, history, y_scale


def clone_network(mlp: MLP, ctx: Context, y_scale: float) -> MLP:
    """The same network on another context (the FP32-spectral one)."""
    other = MLP(ctx, mlp.n_in, mlp.hidden, mlp.n_out)
    other.set_params(mlp.get_params())
    other.set_output_scale(y_scale)
    return other


def fp32_switch(inst) -> float:
    """Residual at which a run leaves the FP32 spectral stage for FP64:
    max(1e-5, 2e-5/eps), far above the FP32 stage's own floor (measured 1e-7 to
    7e-7 on the heat slab at 32^3 for eps from 0.49 down to 0.0072; the outer
    residual holds Q/eps).  At this size, one cell per visit, a V-cycle costs
    about as much in FP32 as in FP64 and more near the floor, where the inner
    solves run to their cap, so the FP32 stage takes only the first, large
    reductions."""
    return max(1e-5, 2e-5 / inst["eps"])


def time_to_residual(plan, inst, tol: float = 1e-8, max_cycles: int = 300, max_seconds: float = 60.0,
                     return_field: bool = False):
    """MG-SGS-PFP V-cycles on one instance from its initial state until the outer
    residual is below tol.  plan = [(ctx, mlp or None, switch), ...]: V-cycles
    on each context (with its network attached, if any) until the residual is
    below that leg's switch value (a number, or a function of the instance) or
    stalls for 20 cycles, then the next leg from the same field.  Returns
    seconds, V-cycles, inner updates per visit, learned starts taken and
    per-leg counts (and the final field with return_field)."""
    import torch

    f = initial_field(plan[0][0], inst["nx"])
    hist, inner, visits, learned, legs = [], 0, 0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ctx, mlp, switch in plan:
        if callable(switch):
            switch = switch(inst)
        slab = Slab(ctx, [inst], f)
        if mlp is not None:
            slab.attach_warmstart(mlp)
        if not hist:
            hist.append(slab.residual()[0])
        start, best, best_at = len(hist), hist[-1], len(hist)
        while hist[-1] >= switch and len(hist) <= max_cycles and time.perf_counter() - t0 < max_seconds:
            r, st = slab.vcycle(1, tol=tol, **MG)
            hist.append(r[0])
            inner += st["inner_iters"]
            visits += st["visits"]
            learned += st["learned"]
            if r[0] < 0.9 * best:
                best, best_at = r[0], len(hist)
            if not np.isfinite(r[0]) or (switch > tol and len(hist) - best_at > 20):
                break
        legs.append({"precision": "fp64" if ctx.params.precision == 0 else "fp32", "learned": mlp is not None,
                     "vcycles": len(hist) - start, "residual_at_end": hist[-1]})
        slab.close()
    torch.cuda.synchronize()
    out = {"seconds": time.perf_counter() - t0, "vcycles": len(hist) - 1, "final_residual": hist[-1],
           "reached": hist[-1] < tol, "inner_per_visit": inner / max(visits, 1), "visits": visits,
           "learned_taken": learned, "legs": legs}
    if return_field:
        out["f"] = f
    return out


# ------------------------------------------------------------------ 2D cavities
# Family (lid-driven cavities on [0, 1]^2, walls T = 1 at rest except the lid
# y = 1): lid speed ~ U(0.3, 0.7), eps log-uniform in [0.01, 0.3]; instance i
# draws from numpy.random.default_rng([seed, i]); initial state the unit
# Maxwellian at rest of total mass 1.

MG2 = dict(coarsest=4, nu1=1, nu2=1, coarse_iters=20)


def cavity_instance(seed: int, i: int, n: int):
    rng = np.random.default_rng([seed, i])
    lid = float(rng.uniform(0.3, 0.7))
    eps = float(np.exp(rng.uniform(np.log(0.01), np.log(0.3))))
    return dict(nx=n, ny=n, eps=eps, lid=lid)


def cavity_walls(lid: float):
    return ((1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (0.0, 0.0)), (1.0, (lid, 0.0)))


def cavity_field(ctx: Context, nx: int, ny: int):
    """Uniform unit Maxwellian at rest of total mass 1 on [0, 1]^2 (input data)."""
    import torch

    N, L = ctx.params.N, ctx.params.L
    dv = 2.0 * L / N
    x = (np.arange(N) - N // 2 + 1) * dv
    V = np.stack(np.meshgrid(x, x, indexing="ij"), -1).reshape(-1, 2)
    m = np.exp(-(V * V).sum(1) / 2.0) / (2.0 * np.pi)
    f0 = np.repeat(m[None], nx * ny, axis=0)
    f0 *= 1.0 / (dv * dv * f0.sum() / (nx * ny))
    return torch.from_numpy(f0).to(f"cuda:{ctx.params.device}").contiguous()


def cavity_dataset(ctx: Context, instances, n_snap: int = 3):
    """Features X [n, K + 5] (float32) and targets f_next - M[f] [n, K] (float32):
    for the states f after V-cycles 0 .. n_snap - 1 of every instance, the
    features of f's transport part and Maxwellian, and the state after the next
    V-cycle.  Returns (X, Y, info)."""
    import torch

    Xs, Ys, t0 = [], [], time.perf_counter()
    for d in instances:
        f = cavity_field(ctx, d["nx"], d["ny"])
        cav = Cavity(ctx, d["nx"], d["ny"], d["eps"], cavity_walls(d["lid"]), f)
        eps = torch.full((d["nx"] * d["ny"],), d["eps"], dtype=torch.float64, device=f.device)
        for _ in range(n_snap):
            T = cav.inflow()
            theta, M, _ = ctx.maxwellian(f)
            X = ctx.features(T, theta, eps, 1.0 / d["nx"])
            cav.vcycle(1, tol=1e-8, **MG2)
            ok = torch.isfinite(f).all(1)
            Xs.append(X[ok])
            Ys.append((f - M)[ok].to(torch.float32))
        cav.close()
    X, Y = torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous()
    return X, Y, {"samples": int(X.shape[0]), "seconds": time.perf_counter() - t0}


def cavity_time_to_residual(plan, inst, tol: float = 1e-5, max_cycles: int = 200, max_seconds: float = 120.0,
                            coarsest: int = 4):
    """MG-SGS-PFP V-cycles on one cavity from the uniform state until the outer
    residual is below tol; plan as in time_to_residual.  Returns seconds,
    V-cycles, inner updates per visit, learned starts taken and per-leg counts."""
    import torch

    f = cavity_field(plan[0][0], inst["nx"], inst["ny"])
    hist, inner, visits, learned, legs = [], 0, 0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ctx, mlp, switch in plan:
        if callable(switch):
            switch = switch(inst)
        cav = Cavity(ctx, inst["nx"], inst["ny"], inst["eps"], cavity_walls(inst["lid"]), f)
        if mlp is not None:
            cav.attach_warmstart(mlp)
        if not hist:
            hist.append(cav.residual())
        start, best, best_at = len(hist), hist[-1], len(hist)
        while hist[-1] >= switch and len(hist) <= max_cycles and time.perf_counter() - t0 < max_seconds:
            r, st = cav.vcycle(1, tol=tol, coarsest=coarsest, nu1=1, nu2=1, coarse_iters=20)
            hist.append(r)
            inner += st["inner_iters"]
            visits += st["visits"]
            learned += st["learned"]
            if r < 0.9 * best:
                best, best_at = r, len(hist)
            if not np.isfinite(r) or (switch > tol and len(hist) - best_at > 10):
                break
        legs.append({"precision": "fp64" if ctx.params.precision == 0 else "fp32", "learned": mlp is not None,
                     "vcycles": len(hist) - start, "residual_at_end": hist[-1]})
        cav.close()
    torch.cuda.synchronize()
    return {"seconds": time.perf_counter() - t0, "vcycles": len(hist) - 1, "final_residual": hist[-1],
            "reached": hist[-1] < tol, "inner_per_visit": inner / max(visits, 1), "visits": visits,
            "learned_taken": learned, "legs": legs}
