"""Data generation, training and evaluation of the learned warm start.

Every step runs in libbz through the C ABI: the cell solves that produce the
training targets (bz_cell_fixed_point to a tight tolerance), the discrete
Maxwellians, the feature map, the MLP forward/backward/Adam kernels, and the
learned cell update.  This module only moves tensors between those calls.

Target of one cell: (g* - M[f_old]) / y_scale, where g* solves the inner
problem of eq. inner_eqn for the cell's transport inflow and BGK-penalty
source, and y_scale is the RMS of g* - M[f_old] over the training set.
"""
from __future__ import annotations

import time

import numpy as np

import synth

from . import Context, MLP


def inflow_of(fl, fr, N, L, dx, dev):
    """Transport inflow of eq. r from the two neighbours (first order)."""
    import torch

    v1 = torch.tensor((np.arange(N) - N // 2 + 1) * (2 * L / N), dtype=torch.float64, device=dev)
    v1 = v1.view(N, 1, 1).expand(N, N, N).reshape(-1)
    return ((-torch.clamp(v1, min=0) * fl + torch.clamp(v1, max=0) * fr) / dx).contiguous()


def make_dataset(ctx: Context, n_inst: int, cells_per_inst: int, dx: float, seed: int = 7, start: int = 0,
                 tol: float = 1e-10):
    """Features X [n, K+6] (float32), raw targets g* - M[f_old] [n, K] (float32) and
    the inputs (f_old, inflow, eps) on the device, restricted to the cells whose
    plain solve converged (strong-shock cells can fail the existence test and
    then diverge under the plain fallback iteration; they are left out)."""
    import torch

    dev = torch.device(f"cuda:{ctx.params.device}")
    N, L = ctx.params.N, ctx.params.L
    fl, fo, fr, eps = synth.warmstart_cells(n_inst, cells_per_inst, N, L, seed=seed, start=start)
    fo_t = torch.from_numpy(fo).to(dev)
    inflow = inflow_of(torch.from_numpy(fl).to(dev), torch.from_numpy(fr).to(dev), N, L, dx, dev)
    eps_t = torch.from_numpy(eps).to(dev)
    g, st = ctx.cell_fixed_point(fo_t, inflow, eps_t, dx, tol=tol, max_iter=400)
    stats = ctx.decode_stats(st)
    keep = torch.from_numpy(stats["status"] == 0).to(dev) & torch.isfinite(g).all(1)
    fo_t, inflow, eps_t, g = fo_t[keep].contiguous(), inflow[keep].contiguous(), eps_t[keep].contiguous(), g[keep]
    theta, M, _ = ctx.maxwellian(fo_t)
    X = ctx.features(inflow, theta, eps_t, dx)
    Y = (g - M).to(torch.float32)
    return X, Y, (fo_t, inflow, eps_t), stats


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
    return mlp, history


def compare(ctx: Context, mlp: MLP, f_old, inflow, eps, dx, tol=1e-8, max_iter=100, reps=3):
    """Inner iterations and wall time of the plain and learned cell updates on
    the same cells, and the largest difference of their converged answers."""
    import torch

    out = {}
    for name in ("plain", "learned"):
        fn = (lambda: ctx.cell_fixed_point(f_old, inflow, eps, dx, tol=tol, max_iter=max_iter)) if name == "plain" \
            else (lambda: ctx.cell_fixed_point_learned(mlp, f_old, inflow, eps, dx, tol=tol, max_iter=max_iter))
        g, st = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g, st = fn()
        torch.cuda.synchronize()
        s = ctx.decode_stats(st)
        out[name] = {"seconds": (time.perf_counter() - t0) / reps, "mean_iterations": float(s["iterations"].mean()),
                     "max_iterations": int(s["iterations"].max()), "learned_kept": int(s["learned"].sum()),
                     "unconverged": int((s["status"] != 0).sum()), "g": g}
    diff = (out["plain"]["g"] - out["learned"]["g"]).abs().max().item()
    scale = out["plain"]["g"].abs().max().item()
    for v in out.values():
        v.pop("g")
    out["max_rel_diff"] = diff / scale
    return out
