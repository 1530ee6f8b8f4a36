"""The launch-plan tuner (bz_tune) and every candidate plan: each keeps oracle
parity of the collision term (the plans change how the pipeline is launched,
not what it computes), the tuner keeps the fastest candidate and later
contexts of the same discretisation start from it."""
import numpy as np
import pytest

import synth
from oracle import collision as OQ
from oracle.grid import Spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return bz


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("waves", [8, 4, 2])
@pytest.mark.parametrize("chunk,acc", [(0, 0), (7, 2)])
def test_every_plan_keeps_parity(bz, prec, waves, chunk, acc):
    # 32^3, a small rule, 3 radial nodes; 10 cells in chunks of 7 (a ragged last
    # chunk) with the nodes folded two at a time (a ragged last group), or one
    # chunk with all nodes held
    N, L, nt, nph, nr, B = 32, 8.0, 4, 6, 3, 10
    print(f"plan waves={waves} chunk={chunk} acc={acc} precision={prec}", flush=True)
    sp = Spec(d=3, N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr)
    f = synth.mixture_batch(B, N, L, seed=71)
    ctx = bz.Context(N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr, precision=prec)
    ctx.set_plan(waves, chunk, acc)
    assert ctx.get_plan() == {"pair_waves": waves, "chunk_cells": chunk, "acc_nodes": acc}
    Q = ctx.eval_Q(torch.from_numpy(f).to("cuda:0"), corrected=True).cpu().numpy()
    tol = 1e-12 if prec == 0 else 2e-6
    for i in (0, 6, 7, 9):
        ref = OQ.q_corrected(sp, f[i])
        _, loss = OQ.q_fsm(sp, f[i], parts=True)
        err = np.abs(Q[i] - ref).max() / max(np.abs(ref).max(), np.abs(loss).max())
        assert err < tol, (i, err)


@pytest.mark.parametrize("prec", [0, 1])
def test_held_nodes_do_not_change_the_result(bz, prec):
    # the column pass sums the radial nodes in node order whatever the number
    # held, so one node per pass and all nodes per pass give the same bits
    N, L, nt, nph, nr, B = 32, 8.0, 4, 6, 5, 6
    print(f"held nodes, precision={prec}", flush=True)
    f = torch.from_numpy(synth.mixture_batch(B, N, L, seed=73)).to("cuda:0")
    out = []
    for acc in (1, 2, 0):
        ctx = bz.Context(N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr, precision=prec)
        ctx.set_plan(4, 0, acc)
        out.append(ctx.eval_Q(f, corrected=True).cpu())
    assert torch.equal(out[0], out[1]) and torch.equal(out[0], out[2])


def test_tuner_keeps_and_caches_the_fastest_plan(bz):
    N, L, nt, nph, nr, B = 32, 8.0, 4, 8, 3, 96
    f = torch.from_numpy(synth.mixture_batch(B, N, L, seed=72)).to("cuda:0")
    ctx = bz.Context(N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr)
    rep = ctx.tune(f, corrected=True)
    print(rep, flush=True)
    ms = [m for _, m in rep["candidates"]]
    assert len(ms) == 9 and all(m > 0 for m in ms)
    assert ms[rep["best"]] == min(ms)
    assert ctx.get_plan() == rep["plan"]
    again = bz.Context(N=N, L=L, n_theta=nt, n_phi=nph, n_rho=nr)
    assert again.get_plan() == rep["plan"]
    with pytest.raises(bz.BZError):
        ctx.set_plan(3, 0)
