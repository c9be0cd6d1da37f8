"""Eigenpairs nearest a reference energy, residuals and orthonormalisation (oracle).

The paper needs a limited number of eigenstates of H around a given energy E
(Sec. II.B, paragraph on methods for a few states near E, which names the
folded-spectrum method).  Their quality is measured by the eigen-residual
Delta_i = || H phi_i - eps_i phi_i || (definition under the preconditioner M'
equation, Sec. II.B).

Folding: the eigenvalues of A = (H - E)^2 are (lambda - E)^2 with the same
eigenvectors, and A is positive semi-definite (Sec. II.B, folded equation), so
the N states nearest E are the N lowest states of A.
"""
from __future__ import annotations

import numpy as np


def nearest_eigenpairs(h, e_ref, n):
    """Dense Hermitian eigensolve, then the n eigenpairs with the smallest
    |lambda - E_ref| (ties broken by lambda).  Returned ascending in lambda.

    Returns (lam [n], vecs [n, npw] band-major, all_lam [npw], gap_ratio) where
    gap_ratio = (|lam_(n+1) - E| - |lam_(n) - E|) -- the distance, in folded
    order, between the last kept and the first rejected state.  A tiny value
    means the nth state is not unique."""
    w, u = np.linalg.eigh(h)
    key = np.lexsort((w, np.abs(w - e_ref)))
    pick = key[:n]
    pick = pick[np.argsort(w[pick], kind="stable")]
    if len(key) > n:
        gap = abs(w[key[n]] - e_ref) - abs(w[key[n - 1]] - e_ref)
    else:
        gap = np.inf
    return w[pick], np.ascontiguousarray(u[:, pick].T), w, gap


def residuals(hop, vecs, lam):
    """Delta_i = ||H v_i - lam_i v_i||_2 / ||v_i|| for a band-major block."""
    hv = hop(vecs)
    r = hv - lam[:, None] * vecs
    return np.linalg.norm(r, axis=1) / np.linalg.norm(vecs, axis=1)


def cholesky_orthonormalize(block):
    """Psi <- Psi L^{-H} with S = Psi^H Psi = L L^H (band-major: rows are bands).

    Written with the band-major convention: S_ij = <psi_i|psi_j>, and the new
    band b is sum_j conj(Linv[b, j]) psi_j."""
    s = block.conj() @ block.T
    ell = np.linalg.cholesky(s)
    linv = np.linalg.inv(ell)
    return linv.conj() @ block


def rayleigh_ritz(block, hblock):
    """Subspace diagonalisation of <psi_i|H|psi_j> for an orthonormal block:
    returns (theta ascending, rotated block, rotated H block)."""
    m = block.conj() @ hblock.T
    m = 0.5 * (m + m.conj().T)
    theta, q = np.linalg.eigh(m)
    # new band b = sum_j q[j, b] psi_j
    return theta, q.T @ block, q.T @ hblock


def principal_cosines(u_ref, v):
    """Singular values of U_ref^H V for two orthonormal band-major blocks: the
    cosines of the principal angles between the subspaces."""
    return np.linalg.svd(u_ref.conj() @ v.T, compute_uv=False)
