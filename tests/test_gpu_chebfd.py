"""GPU Chebyshev filter diagonalisation against the oracle: the filtered block
element by element, ChebFD steps against the oracle's steps and the dense
eigenpairs in the window, the Lanczos spectral bounds against the dense
spectrum, error paths, and sampled residuals on the wire cell."""
import numpy as np
import pytest

from paper_1907_06821_amd import synth
from oracle.chebfd import chebfd_step, chebyshev_filter, window_coefficients
from tests._helpers import gpu_context, oracle_for, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _bounds(h, pad=0.3):
    lam = np.linalg.eigvalsh(h)
    return lam, lam[0] - pad, lam[-1] + pad


@pytest.mark.parametrize("which,degree", [("tiny", 0), ("tiny", 1), ("tiny", 150), ("nl", 90)])
def test_filter_matches_oracle(torch_cuda, which, degree):
    import paper_1907_06821_amd as pw
    if which == "tiny":
        prob = synth.config(1)
    else:
        prob = synth.small_nonlocal_problem(kpt=(0.11, -0.23, 0.07))
    op = oracle_for(prob)
    lam, emin, emax = _bounds(op.dense())
    e, w = 0.55, 0.3
    nb = 5
    c = synth.start_vectors(3, nb, op.npw)
    ctx = gpu_context(prob, max_bands=nb)
    got = pw.cheb_filter(ctx, to_dev(c), e, w, degree, emin, emax).cpu().numpy()
    ref = chebyshev_filter(op.apply, c, window_coefficients(e, w, emin, emax, degree), emin, emax)
    assert rel_err(got, ref) < 1e-11


def test_chebfd_steps_match_oracle_and_dense(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.config(1)
    op = oracle_for(prob)
    lam, emin, emax = _bounds(op.dense(), 0.2)
    e, w, degree = 0.5, 0.25, 300
    inside = lam[np.abs(lam - e) <= w]
    nb = len(inside) + 6
    v0 = synth.start_vectors(1, nb, op.npw)
    ctx = gpu_context(prob, max_bands=nb)
    t = to_dev(v0)
    eig1, res1 = pw.chebfd_step(ctx, t, e, w, degree, emin, emax)
    oeps, ov, ores = chebfd_step(op.apply, v0, e, w, emin, emax, degree)
    assert np.max(np.abs(eig1 - oeps)) < 1e-10
    assert np.max(np.abs(res1 - ores)) < 1e-9 * max(1.0, np.max(ores))
    hist = [np.max(res1[np.abs(eig1 - e) <= w])]
    for _ in range(3):
        eig, res = pw.chebfd_step(ctx, t, e, w, degree, emin, emax)
        hist.append(np.max(res[np.abs(eig - e) <= w]))
    sel = np.abs(eig - e) <= w
    assert sel.sum() == len(inside)
    assert np.max(np.abs(eig[sel] - inside)) < 1e-9
    assert hist[-1] < 1e-7 and hist[-1] < 1e-2 * hist[0]
    v = t.cpu().numpy()
    assert np.max(np.abs(v.conj() @ v.T - np.eye(nb))) < 1e-12
    direct = np.linalg.norm(op.apply(v) - eig[:, None] * v, axis=1)
    assert np.max(np.abs(direct - res)) < 1e-10


@pytest.mark.parametrize("which", ["tiny", "nl"])
def test_spectral_bounds_enclose_the_spectrum(torch_cuda, which):
    import paper_1907_06821_amd as pw
    prob = synth.config(1) if which == "tiny" else synth.small_nonlocal_problem(kpt=(0.11, -0.23, 0.07))
    op = oracle_for(prob)
    lam = np.linalg.eigvalsh(op.dense())
    ctx = gpu_context(prob, max_bands=2)
    v0 = to_dev(synth.start_vectors(5, 1, op.npw)[0])
    lo, hi = pw.spectral_bounds(ctx, v0, steps=60)
    assert lo <= lam[0] and hi >= lam[-1], (lo, hi, lam[0], lam[-1])
    assert hi - lo < 1.3 * (lam[-1] - lam[0])


def test_chebfd_errors(torch_cuda):
    import paper_1907_06821_amd as pw
    prob = synth.config(1)
    op = oracle_for(prob)
    lam, emin, emax = _bounds(op.dense())
    ctx = gpu_context(prob, max_bands=4)
    c = to_dev(synth.start_vectors(1, 4, op.npw))
    bad = [dict(degree=-1), dict(emin=emax, emax=emin), dict(w=0.0), dict(e=emax + 5.0)]
    for b in bad:
        kw = dict(e=0.5, w=0.2, degree=10, emin=emin, emax=emax)
        kw.update(b)
        with pytest.raises(pw.PwError) as ex:
            pw.cheb_filter(ctx, c, kw["e"], kw["w"], kw["degree"], kw["emin"], kw["emax"])
        assert ex.value.status == pw.PW_EINVAL, b
    # bounds that cut the spectrum: the recurrence overflows and the step says so
    with pytest.raises(pw.PwError) as ex:
        pw.chebfd_step(ctx, c, 0.5, 0.2, 3000, emin, 0.5 * (emin + emax))
    assert ex.value.status in (pw.PW_ENAN, pw.PW_ENOTPD)


def test_chebfd_wire256_sampled_residuals(torch_cuda):
    """One step on the 256-atom wire (24 bands, bounds from the library's
    Lanczos): orthonormal output, and the oracle's own H psi reproduces the
    residuals of two sampled bands."""
    import paper_1907_06821_amd as pw
    import torch
    prob = synth.config(2)
    ctx = gpu_context(prob, max_bands=24)
    v0 = to_dev(synth.start_vectors(2, 1, ctx.npw, seed=7)[0])
    lo, hi = pw.spectral_bounds(ctx, v0, steps=40)
    # the lowest eigenvalue from an independent folded solve far below the spectrum
    low = to_dev(synth.start_vectors(2, 4, ctx.npw, seed=8))
    leig, lres, lst = pw.folded_cg_solve(ctx, -5.0, low, tol=1e-6, maxit=4000, check_every=20, precond=1)
    assert lst["converged"] and lo <= leig[0] and leig[0] - lo < 0.1 * (hi - lo), (lo, leig[0])
    # the top: Rayleigh quotients of the highest-energy plane waves bound the largest eigenvalue from below
    kin = ctx.kinetic()
    top = np.argsort(kin)[-8:]
    e = np.zeros((8, ctx.npw), dtype=np.complex128)
    e[np.arange(8), top] = 1.0
    he = pw.hpsi(ctx, to_dev(e)).cpu().numpy()
    rq = np.real(he[np.arange(8), top])
    assert hi >= rq.max() and hi < rq.max() + 0.1 * (hi - lo), (hi, rq.max())
    t = to_dev(synth.start_vectors(2, 24, ctx.npw, seed=3))
    eig, res = pw.chebfd_step(ctx, t, prob.e_ref, 0.05, 120, lo, hi)
    assert np.all(np.diff(eig) >= 0) and np.all(np.isfinite(res))
    v = t.cpu().numpy()
    assert np.max(np.abs(v.conj() @ v.T - np.eye(24))) < 1e-12
    op = oracle_for(prob)
    for b in (0, 17):
        r = np.linalg.norm(op.apply(v[b:b + 1])[0] - eig[b] * v[b])
        assert abs(r - res[b]) < 1e-9 * max(1.0, res[b]), (b, r, res[b])


def test_chebfd_single_vector(torch_cuda):
    """nb = 1: the step returns the Rayleigh quotient of the filtered, normalised
    vector and its residual, as the oracle's step does."""
    import paper_1907_06821_amd as pw
    prob = synth.small_nonlocal_problem(kpt=(0.11, -0.23, 0.07))
    op = oracle_for(prob)
    lam, emin, emax = _bounds(op.dense())
    v0 = synth.start_vectors(4, 1, op.npw)
    ctx = gpu_context(prob, max_bands=1)
    t = to_dev(v0)
    eig, res = pw.chebfd_step(ctx, t, 0.6, 0.3, 60, emin, emax)
    oeps, ov, ores = chebfd_step(op.apply, v0, 0.6, 0.3, emin, emax, 60)
    assert abs(eig[0] - oeps[0]) < 1e-12 and abs(res[0] - ores[0]) < 1e-11
    v = t.cpu().numpy()
    assert abs(abs(np.vdot(ov[0], v[0])) - 1.0) < 1e-12
