"""Pins of the oracle's folded linear solve against what the mathematics fixes:
the eigen-expansion against an LU solve of the original equation, M' against
the exact inverse of (H - E)^2 when every eigenstate is supplied, its action on
and off the eigenstate span, finite termination of CG, and PCG against the
spectral solution.  CPU only."""
import numpy as np
import pytest

from paper_1907_06821_amd import synth
from oracle import hamiltonian as oh
from oracle.eigen import nearest_eigenpairs
from oracle.linsolve import folded_pcg, mprime, spectral_solution
from oracle.precond import paper_m


def _problem():
    prob = synth.small_nonlocal_problem(kpt=(0.11, -0.23, 0.07))
    op = oh.Operator.from_problem(prob)
    return prob, op, op.dense()


def _sources(op, prob, nrhs, seed=0):
    return synth.boundary_sources(7, nrhs, op.miller, prob.cell, kpt=prob.kpt, seed=seed)


def test_spectral_solution_equals_lu_solve():
    prob, op, h = _problem()
    e = 0.37
    w = _sources(op, prob, 3)
    x = spectral_solution(h, e, w)
    ref = np.linalg.solve(h - e * np.eye(h.shape[0]), w.T).T
    assert np.max(np.abs(x - ref)) < 1e-10 * np.max(np.abs(ref))
    assert np.max(np.linalg.norm(x @ h.T - e * x - w, axis=1)) < 1e-10


def test_mprime_with_every_eigenstate_is_the_exact_inverse():
    """phi = all eigenvectors, Delta = 0: M' = (H - E)^-2 whatever M is."""
    prob, op, h = _problem()
    e = 0.41
    eps, u = np.linalg.eigh(h)
    phi = np.ascontiguousarray(u.T)
    v = synth.start_vectors(99, 2, op.npw, seed=3)
    av = (v @ h.T - e * v) @ h.T - e * (v @ h.T - e * v)
    mdiag = paper_m(op.kin, e, 1.0)
    got = mprime(av, mdiag, e, phi, eps, np.zeros_like(eps))
    assert np.max(np.abs(got - v)) < 1e-9 * np.max(np.abs(v))


def test_mprime_on_and_off_the_eigenstate_span():
    prob, op, h = _problem()
    e = 0.5
    eps, phi, _, _ = nearest_eigenpairs(h, e, 5)
    delta = np.array([1e-3, 2e-2, 0.0, 5e-2, 1e-4])
    mdiag = paper_m(op.kin, e, 0.7)
    # on the span: phi_i / ((eps_i - E)^2 + Delta_i^2)
    got = mprime(phi, mdiag, e, phi, eps, delta)
    want = phi / ((eps - e) ** 2 + delta ** 2)[:, None]
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    # off the span: (1 - P) M v for v orthogonal to every phi_i
    v = synth.start_vectors(99, 3, op.npw, seed=5)
    v = v - (v @ phi.conj().T) @ phi
    mv = mdiag[None, :] * v
    want = mv - (mv @ phi.conj().T) @ phi
    # (the leftover <phi_i|v> ~ 1e-16 is amplified by 1/d_i up to ~1e4)
    assert np.max(np.abs(mprime(v, mdiag, e, phi, eps, delta) - want)) < 1e-10 * np.max(np.abs(mv))
    # no eigenstates: M' is M
    assert np.array_equal(mprime(v, mdiag, e), mdiag[None, :] * v)


def test_mprime_is_hermitian_positive_definite():
    prob, op, h = _problem()
    e = 0.5
    eps, phi, _, _ = nearest_eigenpairs(h, e, 4)
    delta = np.full(4, 1e-2)
    mdiag = paper_m(op.kin, e, 1.0)
    dense = mprime(np.eye(op.npw), mdiag, e, phi, eps, delta).T     # column j = M' e_j
    assert np.max(np.abs(dense - dense.conj().T)) < 1e-12 * np.max(np.abs(dense))
    assert np.linalg.eigvalsh(0.5 * (dense + dense.conj().T)).min() > 0


def test_cg_terminates_within_the_dimension():
    """Exact-arithmetic CG ends in at most n steps; on a well-conditioned 24 x 24
    Hermitian H with E in a spectral gap it reaches 1e-10 by then."""
    rng = np.random.default_rng(11)
    n = 24
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.concatenate([np.linspace(-2.0, -0.5, n // 2), np.linspace(0.5, 2.0, n // 2)])
    h = (q * lam) @ q.conj().T
    w = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    r = folded_pcg(lambda b: b @ h.T, 0.0, w, np.zeros_like(w), np.ones(n), tol=1e-10, maxit=n,
                   check_every=1)
    assert r["converged"] and r["iters"] <= n
    assert np.max(np.abs(r["psi"] - np.linalg.solve(h, w.T).T)) < 1e-9


def test_exact_preconditioner_converges_in_one_step():
    prob, op, h = _problem()
    e = 0.33
    eps, u = np.linalg.eigh(h)
    w = _sources(op, prob, 2, seed=1)
    r = folded_pcg(lambda b: b @ h.T, e, w, np.zeros_like(w), paper_m(op.kin, e, 1.0),
                   np.ascontiguousarray(u.T), eps, np.zeros_like(eps), tol=1e-9, maxit=5, check_every=1)
    assert r["iters"] == 1 and r["converged"]
    assert np.max(r["resid"]) < 1e-9


@pytest.mark.parametrize("use_eigs", [False, True])
def test_pcg_reaches_the_spectral_solution(use_eigs):
    prob = synth.config(1)
    op = oh.Operator.from_problem(prob)
    h = op.dense()
    e = prob.e_ref
    w = _sources(op, prob, 3, seed=2)
    ref = spectral_solution(h, e, w)
    mdiag = paper_m(op.kin, e, 1.0)
    kw = {}
    if use_eigs:
        eps, phi, _, _ = nearest_eigenpairs(h, e, 8)
        kw = dict(phi=phi, eps=eps, delta=np.full(8, 1e-9))
    hist = []
    r = folded_pcg(op.apply, e, w, np.zeros_like(w), mdiag, tol=1e-9, maxit=4000, check_every=10,
                   history=hist, **kw)
    assert r["converged"]
    # the error in psi is at most the residual over the smallest |eps - E|
    gap = np.min(np.abs(np.linalg.eigvalsh(h) - e))
    assert np.max(np.linalg.norm(r["psi"] - ref, axis=1)) < 2e-9 / gap
    direct = np.linalg.norm(r["psi"] @ h.T - e * r["psi"] - w, axis=1)
    assert np.allclose(r["resid"], direct, rtol=1e-6, atol=1e-14)
    if use_eigs:
        plain = folded_pcg(op.apply, e, w, np.zeros_like(w), mdiag, tol=1e-9, maxit=4000, check_every=10)
        assert r["iters"] < plain["iters"]


def test_boundary_sources_sit_near_the_boundary():
    prob = synth.config(1)
    op = oh.Operator.from_problem(prob)
    w = synth.boundary_sources(1, 2, op.miller, prob.cell, slab=0.1)
    assert np.allclose(np.linalg.norm(w, axis=1), 1.0)
    n = prob.grid
    g = np.zeros((2,) + tuple(n), dtype=np.complex128)
    idx = tuple(np.mod(op.miller, n).T)
    for l in range(2):
        g[l][idx] = w[l]
    f = np.fft.ifftn(g, axes=(1, 2, 3))
    dens = np.sum(np.abs(f) ** 2, axis=(1, 2))                   # [2][n2] along z
    z = np.arange(n[2]) / n[2]
    near = np.minimum(z, 1 - z) <= 0.25
    assert np.all(dens[:, near].sum(axis=1) / dens.sum(axis=1) > 0.9)
