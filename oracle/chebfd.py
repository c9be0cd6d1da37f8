"""Chebyshev filter diagonalisation of an energy window (oracle, CPU, FP64).

Test infrastructure: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the library never does.

The paper obtains the eigenstates near E with ChebFD (Sec. II.B, ChebFD
paragraph): a polynomial p(H), a linear combination of Chebyshev polynomials,
imitates a window function around E; applied to a block of random vectors it
keeps the eigencomponents inside the window and suppresses the rest, and a
subspace diagonalisation of <phi_i|H|phi_j> then gives approximate eigenstates;
the step is repeated, each repetition lowering the error (its Fig. on ChebFD).
The paper gives no formulas; the textbook ones are used:

  spectrum map     x = (H - c) / h with c = (emax + emin) / 2, h = (emax - emin) / 2,
                   so that [emin, emax] (which must hold the spectrum) maps to [-1, 1]
  window           the indicator of [E - w, E + w], mapped to [a, b] (clipped to [-1, 1])
  coefficients     of that indicator in Chebyshev polynomials of the first kind,
                   mu_0 = (arccos a - arccos b) / pi,
                   mu_k = 2 (sin(k arccos a) - sin(k arccos b)) / (k pi),  k >= 1
  damping          Jackson's kernel for degree M (kernel polynomial method,
                   Weisse, Wellein, Alvermann, Fehske, Rev. Mod. Phys. 78, 275 (2006)):
                   g_k = ((M - k + 1) cos(k q) + sin(k q) cot q) / (M + 1), q = pi / (M + 1)
  filter           p(H) v = sum_{k=0..M} g_k mu_k T_k(x) v with the recurrence
                   T_0 v = v, T_1 v = x v, T_{k+1} v = 2 x T_k v - T_{k-1} v
  one ChebFD step  Phi <- p(H) Phi; Cholesky orthonormalisation; Rayleigh-Ritz in H
                   (eigenvalues ascending); residuals Delta_i = ||H phi_i - eps_i phi_i||
"""
from __future__ import annotations

import numpy as np

from .eigen import cholesky_orthonormalize, rayleigh_ritz


def window_coefficients(e_ref, half_width, emin, emax, degree, jackson=True):
    """g_k mu_k, k = 0..degree, of the window [E - w, E + w] on the spectrum map of
    [emin, emax]."""
    c = 0.5 * (emax + emin)
    h = 0.5 * (emax - emin)
    a = min(1.0, max(-1.0, (e_ref - half_width - c) / h))
    b = min(1.0, max(-1.0, (e_ref + half_width - c) / h))
    ta, tb = np.arccos(a), np.arccos(b)
    k = np.arange(degree + 1, dtype=np.float64)
    mu = np.empty(degree + 1)
    mu[0] = (ta - tb) / np.pi
    mu[1:] = 2.0 * (np.sin(k[1:] * ta) - np.sin(k[1:] * tb)) / (k[1:] * np.pi)
    if jackson:
        mu = mu * jackson_damping(degree)
    return mu


def jackson_damping(degree):
    """Jackson's damping factors g_0..g_M (Weisse et al. 2006)."""
    m = degree
    q = np.pi / (m + 1)
    k = np.arange(m + 1, dtype=np.float64)
    return ((m - k + 1) * np.cos(k * q) + np.sin(k * q) / np.tan(q)) / (m + 1)


def chebyshev_filter(apply_h, block, coef, emin, emax):
    """p(H) block = sum_k coef_k T_k((H - c)/h) block for a band-major block."""
    c = 0.5 * (emax + emin)
    h = 0.5 * (emax - emin)
    u_prev = np.array(block, dtype=np.complex128)
    y = coef[0] * u_prev
    if len(coef) == 1:
        return y
    u = (apply_h(u_prev) - c * u_prev) / h
    y = y + coef[1] * u
    for k in range(2, len(coef)):
        u_next = 2.0 * (apply_h(u) - c * u) / h - u_prev
        y = y + coef[k] * u_next
        u_prev, u = u, u_next
    return y


def chebfd_step(apply_h, block, e_ref, half_width, emin, emax, degree):
    """One ChebFD step: filter, orthonormalise, Rayleigh-Ritz in H.
    Returns (eps ascending, Ritz vectors [nb, npw], residuals Delta_i)."""
    coef = window_coefficients(e_ref, half_width, emin, emax, degree)
    y = chebyshev_filter(apply_h, block, coef, emin, emax)
    q = cholesky_orthonormalize(y)
    eps, v, hv = rayleigh_ritz(q, apply_h(q))
    resid = np.linalg.norm(hv - eps[:, None] * v, axis=1)
    return eps, v, resid
