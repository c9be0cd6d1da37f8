"""The FFT autotuner: every launch variant it may pick (compile-time length
kernels, runtime plans over radix schedules and thread counts, the four-lane xy
kernels at every thread count, the GEMM tiles of the back-projection and
of the block rotation) computes the same result as the oracle or as the
definition, and it installs exactly one winner per pass."""
import numpy as np
import pytest

from paper_1907_06821_amd import synth
from tests._helpers import gpu_context, oracle_for, random_block, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["cube", "cube48", "tiny", "skew"])
def test_every_fft_candidate_matches_oracle(torch_cuda, which):
    import torch
    import paper_1907_06821_amd as pw
    if which == "cube":
        prob = synth.batched_problems(4, seed=3)[2]          # one of the uneven cubes (40^3)
    elif which == "cube48":
        prob = synth.batched_problems(4, seed=3)[1]          # 48^3: the four-lane xy kernel (M = 12)
    elif which == "tiny":
        prob = synth.config(1)                               # 16^3: the four-lane xy kernel (M = 4)
    else:
        prob = synth.small_nonlocal_problem()                # 12 x 15 x 20 grid: xy runtime plans only
    op = oracle_for(prob)
    nb = 4
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    c = random_block(11, nb, op.npw)
    ref = op.apply(c, shift=prob.e_ref)
    # complex64 H psi takes its projector GEMMs in BF16 (about 1e-3 of the
    # nonlocal term): its FFT variants are compared with each other at FP32
    # rounding, and the tuned one with the oracle at the BF16 level
    for dtype, tol_ref, tol_var in ((pw.PW_C128, 1e-12, 1e-12), (pw.PW_C64, 2e-3, 3e-6)):
        recs = pw.autotune(ctx, nb, dtype=dtype, reps=2)
        if which in ("cube48", "tiny"):
            # four-lane kernel at 128, 192, 256 and 512 threads; complex128 also with V(r)
            # loaded ahead (sched 1)
            n4 = 8 if dtype == pw.PW_C128 else 4
            assert sum(r["pass_"] == 1 and r["kind"] == 3 for r in recs) == n4
        for p in range(3):
            mine = [r for r in recs if r["pass_"] == p]
            assert len(mine) >= 2
            assert sum(r["chosen"] for r in mine) == 1
            assert all(r["ms"] > 0 for r in mine)
        tdt = "complex128" if dtype == pw.PW_C128 else "complex64"
        base = pw.hpsi(ctx, to_dev(c, tdt), shift=prob.e_ref).cpu().numpy()
        assert rel_err(base, ref) < tol_ref                  # the tuned choice
        if dtype == pw.PW_C128:
            assert sum(r["pass_"] == 5 and r["chosen"] for r in recs) == 1
        for r in recs:
            pw.fft_choose(ctx, r, dtype=dtype)
            got = pw.hpsi(ctx, to_dev(c, tdt), shift=prob.e_ref).cpu().numpy()
            err_ = rel_err(got, ref if dtype == pw.PW_C128 else base)
            assert err_ < tol_var, (r, err_)
            if r["pass_"] == 5:                              # block rotation: Gram/Cholesky orthonormalisation
                q = pw.orthonormalize(ctx, to_dev(c)).cpu().numpy()
                assert np.abs(q.conj() @ q.T - np.eye(nb)).max() < 1e-13, r
                # Psi = L^H Q with L^H upper triangular: the spans agree band by band
                coef = q.conj() @ c.T
                assert np.abs(np.tril(coef, -1)).max() < 1e-12 * np.abs(coef).max(), r
                assert rel_err(coef.T @ q, c) < 1e-13, r
            pw.fft_choose(ctx, {"pass_": r["pass_"], "kind": 0, "radix": r["radix"]}, dtype=dtype)
        with pytest.raises(pw.PwError):
            pw.fft_choose(ctx, {"pass_": 1, "kind": 2, "nthr": 100, "sched": 0}, dtype=dtype)


def test_gemm_tiles_at_136_bands(torch_cuda):
    """Every back-projection and block-rotation tile at 136 bands (row tiles of
    16, 32, 64, 128 and 144 with a ragged last tile): H psi against the oracle and the
    Gram/Cholesky orthonormalisation against its definition."""
    import paper_1907_06821_amd as pw
    prob = synth.batched_problems(4, seed=3)[1]              # 48^3 cube
    op = oracle_for(prob)
    nb = 136
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128)
    assert op.npw > nb
    c = random_block(12, nb, op.npw)
    ref = op.apply(c, shift=prob.e_ref)
    recs = [r for r in pw.autotune(ctx, nb, dtype=pw.PW_C128, reps=1) if r["pass_"] in (4, 5)]
    assert len(recs) == 28
    for r in recs:
        pw.fft_choose(ctx, r)
        if r["pass_"] == 4:
            got = pw.hpsi(ctx, to_dev(c), shift=prob.e_ref).cpu().numpy()
            assert rel_err(got, ref) < 1e-12, r
        else:
            q = pw.orthonormalize(ctx, to_dev(c)).cpu().numpy()
            assert np.abs(q.conj() @ q.T - np.eye(nb)).max() < 1e-12, r
            coef = q.conj() @ c.T
            assert np.abs(np.tril(coef, -1)).max() < 1e-11 * np.abs(coef).max(), r
            assert rel_err(coef.T @ q, c) < 1e-12, r
        pw.fft_choose(ctx, {"pass_": r["pass_"], "kind": 0, "radix": r["radix"]})


@pytest.mark.parametrize("nb", [96, 128])
def test_gram_single_tile(torch_cuda, nb):
    """Square band-by-band products of 65..128 bands take one 128 x 128 NT tile:
    the Gram/Cholesky orthonormalisation against its definition."""
    import paper_1907_06821_amd as pw
    prob = synth.batched_problems(4, seed=3)[1]              # 48^3 cube
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128)
    c = random_block(13, nb, ctx.npw)
    q = pw.orthonormalize(ctx, to_dev(c)).cpu().numpy()
    assert np.abs(q.conj() @ q.T - np.eye(nb)).max() < 1e-12
    coef = q.conj() @ c.T
    assert np.abs(np.tril(coef, -1)).max() < 1e-11 * np.abs(coef).max()
    assert rel_err(coef.T @ q, c) < 1e-12


@pytest.mark.parametrize("nb", [1, 5, 16, 17, 32, 33])
def test_narrow_tiles_few_bands(torch_cuda, nb):
    """A few bands against a tall projector table (520 projectors): the 16- and
    32-wide NT tiles (128-row tiles of the table) and the 16- and 32-row NN tiles,
    with ragged edges; H psi against the oracle, and the Gram/Cholesky
    orthonormalisation (64 x 16 and 64 x 32 NT tiles) against its definition."""
    import paper_1907_06821_amd as pw
    prob = synth.cubic_random_problem(10.0, (40, 40, 40), 8.0, 130, 0.3, nb, seed=2)
    op = oracle_for(prob)
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128)
    assert ctx.nproj == 520
    c = random_block(14, nb, op.npw)
    got = pw.hpsi(ctx, to_dev(c), shift=prob.e_ref).cpu().numpy()
    assert rel_err(got, op.apply(c, shift=prob.e_ref)) < 1e-12
    q = pw.orthonormalize(ctx, to_dev(c)).cpu().numpy()
    assert np.abs(q.conj() @ q.T - np.eye(nb)).max() < 1e-12
    coef = q.conj() @ c.T
    assert np.abs(np.tril(coef, -1)).max() < 1e-11 * np.abs(coef).max()
    assert rel_err(coef.T @ q, c) < 1e-12
