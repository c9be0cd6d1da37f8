"""GPU parity of the H psi path (FFT passes, kinetic epilogue, projector GEMMs)
against the FP64 CPU oracle.  All inputs are seeded synthetic problems."""
import dataclasses
import math

import numpy as np
import pytest

from paper_1907_06821_amd import synth
from tests._helpers import gpu_context, oracle_for, rel_err, to_dev, random_block

pytestmark = pytest.mark.gpu


def _direct_to_grid(miller, grid, coef):
    """f(r_j) = sum_G c(G) exp(+2 pi i sum_a n_a j_a / N_a), written out (tiny grids only)."""
    n0, n1, n2 = grid
    j0, j1, j2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    out = np.zeros((coef.shape[0], n0, n1, n2), dtype=np.complex128)
    for g, (a, b, c) in enumerate(miller):
        ph = np.exp(2j * math.pi * ((a * j0 % n0) / n0 + (b * j1 % n1) / n1 + (c * j2 % n2) / n2))
        out += coef[:, g, None, None, None] * ph[None]
    return out


def test_wave_to_grid_matches_direct_sum(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem()
    op = oracle_for(prob)
    ctx = gpu_context(prob, max_bands=3)
    c = random_block(1, 3, op.npw)
    got = pw.wave_to_grid(ctx, to_dev(c)).cpu().numpy()
    ref = _direct_to_grid(op.miller, prob.grid, c)
    err_ = rel_err(got, ref)
    assert err_ < 1e-13, err_
    # complex64 path
    ctx32 = gpu_context(prob, 3, pw.PW_PREP_C128 | pw.PW_PREP_C64)
    got32 = pw.wave_to_grid(ctx32, to_dev(c, "complex64")).cpu().numpy()
    err_ = rel_err(got32, ref)
    assert err_ < 2e-6, err_


def test_grid_to_wave_matches_direct_sum(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem()
    op = oracle_for(prob)
    ctx = gpu_context(prob, max_bands=2)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2,) + prob.grid) + 1j * rng.standard_normal((2,) + prob.grid)
    got = pw.grid_to_wave(ctx, to_dev(f)).cpu().numpy()
    n = np.prod(prob.grid)
    n0, n1, n2 = prob.grid
    j0, j1, j2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    ref = np.empty((2, op.npw), dtype=np.complex128)
    for g, (a, b, c) in enumerate(op.miller):
        ph = np.exp(-2j * math.pi * ((a * j0 % n0) / n0 + (b * j1 % n1) / n1 + (c * j2 % n2) / n2))
        ref[:, g] = np.sum(f * ph[None], axis=(1, 2, 3)) / n
    err_ = rel_err(got, ref)
    assert err_ < 1e-13, err_


def test_parseval_and_roundtrip_wire(torch_cuda):
    """sum_j |psi(r_j)|^2 = N sum_G |c(G)|^2 and grid -> wave inverts wave -> grid."""
    import paper_1907_06821_amd as pw
    prob = synth.config(2)
    ctx = gpu_context(prob, max_bands=4)
    c = random_block(2, 4, ctx.npw)
    g = pw.wave_to_grid(ctx, to_dev(c))
    n = np.prod(prob.grid)
    lhs = (g.abs() ** 2).sum(dim=(1, 2, 3)).cpu().numpy()
    rhs = n * np.sum(np.abs(c) ** 2, axis=1)
    assert np.max(np.abs(lhs / rhs - 1)) < 1e-13
    back = pw.grid_to_wave(ctx, g).cpu().numpy()
    err_ = rel_err(back, c)
    assert err_ < 1e-14, err_


def test_hpsi_local_equals_dense_tiny(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.config(1)
    op = oracle_for(prob)
    h = op.dense()
    ctx = gpu_context(prob, max_bands=8)
    c = random_block(3, 8, op.npw)
    got = pw.hpsi(ctx, to_dev(c)).cpu().numpy()
    ref = c @ h.T
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(h)) * math.sqrt(op.npw)
    err_ = rel_err(got, ref)
    assert err_ < 1e-13, err_


@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.11, -0.23, 0.07)])
def test_hpsi_nonlocal_equals_dense_small(torch_cuda, kpt):
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem(kpt=kpt)
    op = oracle_for(prob)
    h = op.dense()
    ctx = gpu_context(prob, max_bands=5)
    c = random_block(4, 5, op.npw)
    for shift in (0.0, 0.37):
        got = pw.hpsi(ctx, to_dev(c), shift=shift).cpu().numpy()
        ref = c @ h.T - shift * c
        err_ = rel_err(got, ref)
        assert err_ < 1e-13, err_


def test_hpsi_chunks_and_strides(torch_cuda):
    """nb above max_bands loops over chunks; ld > npw views are honoured."""
    import torch
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem()
    op = oracle_for(prob)
    h = op.dense()
    ctx = gpu_context(prob, max_bands=2)
    c = random_block(5, 7, op.npw)
    big = torch.zeros((7, op.npw + 13), dtype=torch.complex128, device="cuda")
    big[:, :op.npw] = to_dev(c)
    out = torch.full((7, op.npw + 5), 7.0, dtype=torch.complex128, device="cuda")
    pw.hpsi(ctx, big[:, :op.npw], out=out[:, :op.npw])
    got = out[:, :op.npw].cpu().numpy()
    err_ = rel_err(got, c @ h.T)
    assert err_ < 1e-13, err_
    assert torch.all(out[:, op.npw:] == 7.0)
    # zero bands is a no-op
    pw.hpsi(ctx, big[:0, :op.npw], out=out[:0, :op.npw])


@pytest.mark.parametrize("nb", [128, 136])
def test_hpsi_wire256_sampled_bands(torch_cuda, nb):
    """Full wire cell (48x48x192 grid, 1024 projectors) in the benchmark's launch
    shape (128 bands, or 136 with buffer bands, at once); sampled bands checked
    against the oracle's matrix-free H psi."""
    import paper_1907_06821_amd as pw
    prob = synth.config(2)
    op = oracle_for(prob)
    ctx = gpu_context(prob, max_bands=nb)
    c = random_block(6, nb, op.npw)
    got = pw.hpsi(ctx, to_dev(c), shift=prob.e_ref).cpu().numpy()
    for b in (0, 57, nb - 1):
        ref = op.apply(c[b:b + 1], shift=prob.e_ref)[0]
        err_ = rel_err(got[b], ref)
        assert err_ < 1e-12, err_


def test_hermiticity_wire256(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.config(2)
    ctx = gpu_context(prob, max_bands=2)
    x = to_dev(random_block(7, 2, ctx.npw))
    hx = pw.hpsi(ctx, x).cpu().numpy()
    xc = x.cpu().numpy()
    a = np.vdot(xc[0], hx[1])     # <x0 | H x1>
    b = np.vdot(xc[1], hx[0])     # <x1 | H x0>
    assert abs(a - np.conj(b)) <= 1e-12 * abs(a)


def test_hpsi_c64_error_bound(torch_cuda):
    """complex64 FFT/pointwise + BF16 projector GEMMs vs the FP64 oracle.
    Bound from the arithmetic: FP32 FFT error ~ 1e-6 of the local part, BF16
    rounding (unit roundoff 2^-8) of beta and of the projections ~ 2 u of the
    nonlocal part."""
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem()
    op = oracle_for(prob)
    ctx = gpu_context(prob, max_bands=6, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    c = random_block(8, 6, op.npw)
    got = pw.hpsi(ctx, to_dev(c, "complex64"), shift=0.2).cpu().numpy()
    ref = op.apply(c, shift=0.2)
    nl = (c @ op.beta.conj().T * op.dproj[None, :]) @ op.beta
    u = 2.0 ** -8
    for b in range(6):
        err = np.linalg.norm(got[b] - ref[b])
        bound = 4 * u * np.linalg.norm(nl[b]) + 2e-6 * np.linalg.norm(ref[b])
        assert err <= bound, (b, err, bound)


@pytest.mark.parametrize("nb", [128, 136, 150, 300])
def test_orthonormalize_matches_oracle(torch_cuda, nb):
    import paper_1907_06821_amd as pw
    from oracle.eigen import cholesky_orthonormalize
    prob = synth.config(2)
    ctx = gpu_context(prob, max_bands=nb)
    c = random_block(9, nb, ctx.npw)
    t = to_dev(c)
    pw.orthonormalize(ctx, t)
    got = t.cpu().numpy()
    s = got.conj() @ got.T
    assert np.max(np.abs(s - np.eye(nb))) < 1e-12
    ref = cholesky_orthonormalize(c)
    err_ = rel_err(got, ref)
    assert err_ < 1e-11, err_


def test_orthonormalize_dependent_bands_fails(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem()
    ctx = gpu_context(prob, max_bands=4)
    c = random_block(10, 4, ctx.npw)
    c[3] = c[1]
    with pytest.raises(pw.PwError) as e:
        pw.orthonormalize(ctx, to_dev(c))
    assert e.value.status == pw.PW_ENOTPD


def test_bad_arguments_rejected(torch_cuda):
    import paper_1907_06821_amd as pw
    import ctypes as C
    prob = synth.small_nonlocal_problem()
    ctx = gpu_context(prob, max_bands=2)
    x = to_dev(random_block(11, 2, ctx.npw))
    lib = pw.lib()
    st = lib.pw_hpsi(ctx.handle, pw.PW_C128, 2, C.c_void_p(x.data_ptr()), ctx.npw - 1, C.c_void_p(x.data_ptr()),
                     ctx.npw, 0.0, None)
    assert st == pw.PW_EINVAL
    st = lib.pw_hpsi(ctx.handle, pw.PW_C64, 2, C.c_void_p(x.data_ptr()), ctx.npw, C.c_void_p(x.data_ptr()),
                     ctx.npw, 0.0, None)
    assert st in (pw.PW_EUNSUPPORTED, pw.PW_EINVAL)
    # a grid too small for the sphere is refused at context creation
    with pytest.raises(pw.PwError) as e:
        pw.Context((8, 8, 8), (10.0, 10.0, 10.0), 6.0, np.zeros((8, 8, 8)))
    assert e.value.status == pw.PW_EINVAL


def test_hpsi_wire2000_sampled_bands(torch_cuda):
    """The 2000-atom wire (96x96x384 grid, 8000 projectors, 387,091 plane waves)
    with 512 bands in one call, complex128 and complex64 (BF16 projector GEMMs):
    sampled bands against the oracle's matrix-free H psi, whose projector rows
    are built atom by atom."""
    import torch
    import paper_1907_06821_amd as pw
    prob = synth.config(3)
    op = oracle_for(prob)
    assert op.lazy
    nb = 512
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    c = random_block(7, nb, op.npw)
    x = to_dev(c)
    y = pw.hpsi(ctx, x, shift=prob.e_ref)
    y32 = pw.hpsi(ctx, x.to(torch.complex64), shift=prob.e_ref)
    bands = [0, 301, nb - 1]
    ref = op.apply(c[bands], shift=prob.e_ref)
    got = y[bands].cpu().numpy()
    got32 = y32[bands].cpu().numpy()
    for i in range(len(bands)):
        assert rel_err(got[i], ref[i]) < 1e-12
        assert rel_err(got32[i], ref[i]) < 2e-3


@pytest.mark.parametrize("which,nb", [("wire256", 16), ("cube", 16), ("wire256", 160), ("cube", 150)])
def test_c64_only_context_builds_the_same_tables(torch_cuda, which, nb):
    """A complex64-only context builds its BF16 projector planes from FP64 rows
    64 atoms at a time (the FP64 table never exists whole); its complex64 H psi
    equals that of a context that built the whole FP64 table first, bit for bit
    (wire256: four chunks; the cube: a partial last chunk), with row-major planes
    (16 bands) and with 16-row panels (contexts of 150 and 160 bands)."""
    import paper_1907_06821_amd as pw
    if which == "wire256":
        prob = synth.config(2)
    else:
        prob = max(synth.batched_problems(8, seed=2), key=lambda p: p.natom)
        assert 64 < prob.natom < 128
    full = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    only = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C64)
    c = to_dev(synth.start_vectors(3, nb, full.npw), "complex64")
    a = pw.hpsi(full, c, shift=prob.e_ref).cpu().numpy()
    b = pw.hpsi(only, c, shift=prob.e_ref).cpu().numpy()
    assert np.array_equal(a, b)
    assert only.info()["device_bytes"] < full.info()["device_bytes"]


def test_bf16_wide_variants_agree(torch_cuda):
    """Every launch variant of the BF16 projector GEMMs for more than 144 bands
    (pass 6 of the autotuner) on the 2000-atom wire with 512 bands: the complex64
    H psi of each is within the BF16 bound of the complex128 one (4 u of the
    nonlocal part plus single precision FFT rounding), and the autotuner installs
    exactly one."""
    import torch
    import paper_1907_06821_amd as pw
    prob = synth.config(3)
    nb = 512
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    loc = pw.Context.from_problem(dataclasses.replace(prob, pos=prob.pos[:0], depth=prob.depth[:0],
                                                      dproj=prob.dproj[:0]), max_bands=nb, flags=pw.PW_PREP_C128)
    x = to_dev(random_block(13, nb, ctx.npw))
    ref = pw.hpsi(ctx, x, shift=prob.e_ref)
    nl = ref - pw.hpsi(loc, x, shift=prob.e_ref)
    bound = 4 * 2.0 ** -8 * torch.linalg.vector_norm(nl, dim=1) + 1e-5 * torch.linalg.vector_norm(ref, dim=1)
    x32 = x.to(torch.complex64)
    recs = [r for r in pw.autotune(ctx, 64, dtype=pw.PW_C64, reps=1) if r["pass_"] == 6]
    assert len(recs) == 4 and sum(r["chosen"] for r in recs) == 1
    for r in recs:
        pw.fft_choose(ctx, r, dtype=pw.PW_C64)
        got = pw.hpsi(ctx, x32, shift=prob.e_ref).to(torch.complex128)
        err = torch.linalg.vector_norm(got - ref, dim=1)
        assert bool(torch.all(err <= bound)), (r["sched"], float((err / bound).max()))


@pytest.mark.parametrize("ecut,natom,tail", [(10.4, 3, 1), (9.0, 3, 2), (8.0, 20, 3)])
def test_bf16_ring_short_splits(torch_cuda, ecut, natom, tail):
    """The LDS-DMA ring kernels (launch variants 0-3) where a workgroup's K range
    holds only one, two or three 32-deep stages (the last projection split; the
    back-projection over 12 or 80 projectors, two or four stages): 160 bands,
    every variant within the BF16 bound of complex128."""
    import torch
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem(grid=(24, 24, 30), ecut=ecut, natom=natom, nbands=160)
    nb = 160
    ctx = gpu_context(prob, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64)
    # the split of the projection's plane-wave range (128-row tiles, about 512
    # workgroups, at least four stages a split): its last split holds `tail` stages
    ldg = (ctx.npw + 63) // 64 * 64
    ns = max(1, min(512, ldg // 128))
    kchunk = ((ldg + ns - 1) // ns + 31) // 32 * 32
    assert (ldg - (math.ceil(ldg / kchunk) - 1) * kchunk) // 32 == tail
    loc = pw.Context.from_problem(dataclasses.replace(prob, pos=prob.pos[:0], depth=prob.depth[:0],
                                                      dproj=prob.dproj[:0]), max_bands=nb, flags=pw.PW_PREP_C128)
    x = to_dev(random_block(17, nb, ctx.npw))
    ref = pw.hpsi(ctx, x, shift=prob.e_ref)
    nl = ref - pw.hpsi(loc, x, shift=prob.e_ref)
    bound = 4 * 2.0 ** -8 * torch.linalg.vector_norm(nl, dim=1) + 1e-5 * torch.linalg.vector_norm(ref, dim=1)
    x32 = x.to(torch.complex64)
    for v in range(4):
        pw.fft_choose(ctx, dict(pass_=6, kind=3, sched=v), dtype=pw.PW_C64)
        got = pw.hpsi(ctx, x32, shift=prob.e_ref)
        err = torch.linalg.vector_norm(got.to(torch.complex128) - ref, dim=1)
        assert bool(torch.all(err <= bound)), (v, float((err / bound).max()))
