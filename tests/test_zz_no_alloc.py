"""The allocation-free collision entry point (bz_eval_Q_noalloc) against
bz_eval_Q through the C ABI: two calls in a row on each context, the second
with a smaller batch, chunked and unchunked, 3D and 2D velocities; and the
refusal of a context whose one-cell workspace exceeds the static scratch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2409_01910_amd as bz

    bz.load_library()
    return torch.device("cuda:0")


# (d, N, L, n_theta, n_phi, n_rho, precision, batches, flags): 32^3 with n_theta = 8
# and n_rho = 2 needs 7.7 MB per cell in FP64 (corrected), so 40 cells run in 5
# chunks of 8
CASES = [
    (3, 16, 8.0, 4, 8, 8, 0, (37, 6), dict(corrected=True, conserve="mass")),
    (3, 32, 8.0, 8, 16, 2, 0, (40, 3), dict(corrected=True, conserve="mass")),
    (3, 32, 8.0, 2, 4, 2, 1, (23, 4), dict(corrected=True, conserve="all")),
    (3, 32, 8.0, 2, 4, 2, 2, (21, 5), dict(corrected=True, conserve="mass")),
    (3, 8, 6.0, 2, 4, 3, 0, (9, 2), dict(corrected=False)),
    (2, 48, 8.0, 0, 16, 6, 0, (30, 7), dict(corrected=True, conserve="mass")),
    (2, 32, 8.0, 0, 16, 6, 1, (12, 5), dict(corrected=True)),
]


@pytest.mark.parametrize("case", CASES)
def test_noalloc_matches_eval_q_on_two_calls(dev, case):
    import paper_2409_01910_amd as bz

    d, N, L, nt, nph, nr, prec, batches, kw = case
    print(f"noalloc d={d} N={N} M={nt}x{nph} n_rho={nr} prec={prec} batches={batches} {kw}", flush=True)
    ctx = bz.Context(N=N, L=L, n_theta=max(nt, 2), n_phi=nph, n_rho=nr, precision=prec, d=d)
    for B in batches:
        f = torch.from_numpy(synth.mixture_batch(B, N, L, d=d, seed=B)).to(dev)
        ref = ctx.eval_Q(f, **kw)
        out = torch.full_like(f, float("nan"))
        got = ctx.eval_Q_noalloc(f, out, **kw)
        torch.cuda.synchronize()
        scale = ref.abs().max().item()
        err = (got - ref).abs().max().item() / scale
        print(f"  B={B} max rel diff {err:.3e}", flush=True)
        assert torch.isfinite(got).all().item()
        assert err <= 1e-12
        if kw.get("corrected"):
            th_ref = torch.empty((B, d + 2), dtype=torch.float64, device=dev)
            th_got = torch.empty_like(th_ref)
            ctx.eval_Q(f, theta=th_ref, **kw)
            ctx.eval_Q_noalloc(f, out, theta=th_got, **kw)
            assert torch.equal(th_ref, th_got)


def test_noalloc_refuses_a_cell_beyond_the_scratch(dev):
    import paper_2409_01910_amd as bz

    # 32^3 FP64 corrected with 64 polar and 64 radial nodes: 71.6 MB for one cell > 64 MiB
    ctx = bz.Context(N=32, L=8.0, n_theta=64, n_phi=4, n_rho=64)
    f = torch.from_numpy(synth.mixture_batch(1, 32, 8.0, seed=3)).to(dev)
    out = torch.empty_like(f)
    with pytest.raises(bz.BZError, match="bytes of scratch"):
        ctx.eval_Q_noalloc(f, out, corrected=True)
    # the plain form needs less and runs
    ctx.eval_Q_noalloc(f, out, corrected=False)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all().item()


def test_noalloc_empty_batch(dev):
    import paper_2409_01910_amd as bz

    ctx = bz.Context(N=8, L=4.0, n_theta=2, n_phi=4, n_rho=2)
    f = torch.empty((0, 512), dtype=torch.float64, device=dev)
    assert ctx.eval_Q_noalloc(f, torch.empty_like(f)).numel() == 0
