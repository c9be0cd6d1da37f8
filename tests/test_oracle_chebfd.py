"""Pins of the oracle's Chebyshev filter diagonalisation: window coefficients
against Gauss-Chebyshev quadrature, positivity of the Jackson kernel, the filter
on exact eigenvectors against the scalar polynomial, and ChebFD steps reaching
the dense eigenpairs in the window.  CPU only."""
import numpy as np
from numpy.polynomial import chebyshev as npc

from paper_1907_06821_amd import synth
from oracle import hamiltonian as oh
from oracle.chebfd import chebfd_step, chebyshev_filter, jackson_damping, window_coefficients


def test_window_coefficients_equal_quadrature():
    """mu_k = (2 - delta_k0)/N sum_j f(x_j) T_k(x_j) at the Chebyshev nodes; the
    indicator's jumps limit the quadrature to O(1/N)."""
    emin, emax, e, w = -3.0, 13.0, 0.4, 0.7
    mu = window_coefficients(e, w, emin, emax, 60, jackson=False)
    n = 400000
    x = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    en = 0.5 * (emax + emin) + 0.5 * (emax - emin) * x
    f = ((en >= e - w) & (en <= e + w)).astype(float)
    k = np.arange(61)
    t = np.cos(np.outer(k, np.arccos(x)))
    quad = (t @ f) / n * np.where(k == 0, 1.0, 2.0)
    assert np.max(np.abs(mu - quad)) < 2e-5


def test_jackson_kernel_is_positive():
    """The Jackson-damped expansion of a delta function is non-negative."""
    for m in (8, 31, 200):
        g = jackson_damping(m)
        assert abs(g[0] - 1.0) < 1e-15 and np.all(np.diff(g) < 0) and abs(g[-1]) < 1e-2
        x = np.linspace(-1, 1, 2001)
        for x0 in (-0.9, 0.0, 0.37):
            kern = npc.chebval(x, g * np.where(np.arange(m + 1) == 0, 1.0, 2.0) * npc.chebval(x0, np.eye(m + 1)))
            assert kern.min() > -1e-10 * kern.max()


def test_filter_on_eigenvectors_is_the_scalar_polynomial():
    prob = synth.small_nonlocal_problem(kpt=(0.11, -0.23, 0.07))
    op = oh.Operator.from_problem(prob)
    h = op.dense()
    lam, u = np.linalg.eigh(h)
    emin, emax = lam[0] - 0.5, lam[-1] + 0.5
    coef = window_coefficients(0.6, 0.3, emin, emax, 120)
    v = np.ascontiguousarray(u[:, ::37].T)
    got = chebyshev_filter(lambda b: b @ h.T, v, coef, emin, emax)
    x = (lam[::37] - 0.5 * (emax + emin)) / (0.5 * (emax - emin))
    want = npc.chebval(x, coef)[:, None] * v
    assert np.max(np.abs(got - want)) < 1e-12
    # inside the window the filter is close to 1, far outside close to 0
    xs = (np.array([0.6, 3.0]) - 0.5 * (emax + emin)) / (0.5 * (emax - emin))
    p = npc.chebval(xs, coef)
    assert p[0] > 0.95 and abs(p[1]) < 1e-3


def test_chebfd_steps_reach_the_window_eigenpairs():
    prob = synth.config(1)
    op = oh.Operator.from_problem(prob)
    h = op.dense()
    lam = np.linalg.eigvalsh(h)
    e, w = 0.5, 0.25
    inside = lam[np.abs(lam - e) <= w]
    nb = len(inside) + 6
    emin, emax = lam[0] - 0.2, lam[-1] + 0.2
    v = synth.start_vectors(1, nb, op.npw)
    res_hist = []
    for _ in range(4):
        eps, v, res = chebfd_step(op.apply, v, e, w, emin, emax, 300)
        sel = np.abs(eps - e) <= w
        res_hist.append(res[sel].max())
    assert sel.sum() == len(inside)
    assert np.max(np.abs(eps[sel] - inside)) < 1e-9
    assert res_hist[-1] < 1e-7 and res_hist[-1] < 1e-2 * res_hist[0]
