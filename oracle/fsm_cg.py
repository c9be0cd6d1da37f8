"""Folded-spectrum preconditioned conjugate gradients (oracle, CPU, FP64).

Target: the N eigenpairs of H nearest E (Sec. II.B names the folded-spectrum
method for a few eigenstates near E).  Folding with A = (H - E)^2, which is
positive semi-definite (Sec. II.B, folded equation), turns them into the N
lowest states of A; the block minimises tr(Psi^H A Psi) over orthonormal Psi
by preconditioned CG, the same PCG machinery the paper applies to the folded
linear equation (Sec. II.B, functional F), with a G-diagonal preconditioner
(Sec. II.B, M(G)).  Convergence is judged by the eigen-residual
Delta_i = ||H psi_i - theta_i psi_i|| (Sec. II.B, definition of Delta_i;
1e-6 is the accuracy the paper's Sec. II.B results call for).

One iteration, all bands at once (band-major blocks [N, npw]):
  1. mu_i = <psi_i|A|psi_i> = ||Y_i||^2 with Y = (H - E) Psi, AX = (H - E) Y
  2. gradient g_i = A psi_i - mu_i psi_i
  3. z_i = K_i o g_i (diagonal preconditioner)
  4. Polak-Ribiere (non-negative) conjugation p_i = -z_i + beta_i p_i
  5. p_i made orthogonal to every psi_j
  6. YP = (H - E) P, AP = (H - E) YP           (the two H applications)
  7. per band, the exact minimum of the Rayleigh quotient of A on span{psi_i, p_i}
  8. Psi, Y, AX updated with the same 2x2 combination
  9. Cholesky re-orthonormalisation, applied to Psi, Y and AX alike
 10. every `check_every` steps: recompute Y, AX exactly; Rayleigh-Ritz in A
     (bands ordered by folded value; P and the previous gradient turn with
     them); residuals Delta_i from a Rayleigh-Ritz in H taken on copies.
 11. at the end: Rayleigh-Ritz in H, eigenvalues ascending.
A Rayleigh-Ritz in H inside the loop is avoided on purpose: on an unconverged
block it can pair a state above E with one below E at the same folded value and
stall the minimisation.
"""
from __future__ import annotations

import time

import numpy as np

from .precond import tpa2, band_kinetic, paper_m


def _dots(a, b):
    """Per-band <a_i|b_i> (complex)."""
    return np.sum(a.conj() * b, axis=1)


def _chol_transform(x):
    s = x.conj() @ x.T
    ell = np.linalg.cholesky(s)
    return np.linalg.inv(ell).conj()            # new = T @ old


def _line_coeffs(a11, a12, a22):
    """Lowest eigenvector (alpha, beta) of [[a11, a12], [conj(a12), a22]] (real
    diagonals), normalised, computed without cancellation."""
    d = 0.5 * (a22 - a11)
    r = np.sqrt(d * d + np.abs(a12) ** 2)
    alpha = np.where(d >= 0, d + r, a12)
    beta = np.where(d >= 0, -np.conj(a12), d - r)
    nrm = np.sqrt(np.abs(alpha) ** 2 + np.abs(beta) ** 2)
    nrm = np.where(nrm > 0, nrm, 1.0)
    alpha = np.where(r > 0, alpha / nrm, 1.0)
    beta = np.where(r > 0, beta / nrm, 0.0)
    return alpha, beta


def fsm_cg(apply_h, e_ref, psi0, kin, tol=1e-6, maxit=5000, precond="tpa", delta_e=1.0,
           check_every=10, mlp=None, history=None):
    """Run the folded-spectrum PCG.

    apply_h(block) -> H @ block for a band-major block.
    precond: "tpa" (folded Teter-Payne-Allan), "paper" (M(G)), "none", or a
    callable (block, kin) -> weights [N, npw].
    Returns dict(theta, psi, resid, iters, n_hpsi, converged, seconds)."""
    t0 = time.perf_counter()
    e = float(e_ref)
    x = np.array(psi0, dtype=np.complex128)
    nb = x.shape[0]
    kin = np.asarray(kin)
    n_hpsi = 0

    def fold(v):
        nonlocal n_hpsi
        y = apply_h(v) - e * v
        ay = apply_h(y) - e * y
        n_hpsi += 2 * v.shape[0]
        return y, ay

    def weights(block):
        if callable(precond):
            return precond(block, kin)
        if precond == "tpa":
            return tpa2(kin, band_kinetic(block, kin))
        if precond == "paper":
            return np.broadcast_to(paper_m(kin, e, delta_e)[None, :], block.shape)
        if precond == "none":
            return np.ones(block.shape)
        raise ValueError(precond)

    x = _chol_transform(x) @ x
    y, ax = fold(x)
    m = y.conj() @ y.T
    _, qa = np.linalg.eigh(0.5 * (m + m.conj().T))
    x, y, ax = qa.T @ x, qa.T @ y, qa.T @ ax
    p = np.zeros_like(x)
    gz_old = None
    g_old = None
    theta = None
    resid = None
    converged = False
    it = 0
    for it in range(1, maxit + 1):
        mu = np.real(_dots(y, y))
        g = ax - mu[:, None] * x
        z = weights(x) * g
        gz = np.real(_dots(g, z))
        if gz_old is None:
            beta = np.zeros(nb)
        else:
            beta = np.maximum(0.0, (gz - np.real(_dots(g_old, z))) / np.where(gz_old > 0, gz_old, 1.0))
        p = -z + beta[:, None] * p
        p = p - (p @ x.conj().T) @ x                   # p_i -= sum_j <psi_j|p_i> psi_j
        gz_old, g_old = gz, g
        yp, ap = fold(p)
        pn = np.sqrt(np.real(_dots(p, p)))
        pn = np.where(pn > 0, pn, 1.0)
        a11 = mu
        a12 = _dots(y, yp) / pn
        a22 = np.real(_dots(yp, yp)) / pn ** 2
        alpha, bet = _line_coeffs(a11, a12, a22)
        bet = bet / pn
        x = alpha[:, None] * x + bet[:, None] * p
        y = alpha[:, None] * y + bet[:, None] * yp
        ax = alpha[:, None] * ax + bet[:, None] * ap
        t = _chol_transform(x)
        x, y, ax = t @ x, t @ y, t @ ax
        if it % check_every == 0 or it == maxit:
            y, ax = fold(x)
            m = y.conj() @ y.T                       # <psi_i|A|psi_j>
            _, qa = np.linalg.eigh(0.5 * (m + m.conj().T))
            x, y, ax, p, g_old = qa.T @ x, qa.T @ y, qa.T @ ax, qa.T @ p, qa.T @ g_old
            gz_old = np.real(_dots(g_old, weights(x) * g_old))
            theta, q, resid = _h_rayleigh_ritz(x, y, e)
            if history is not None:
                history.append((it, float(resid.max())))
            if resid.max() <= tol:
                converged = True
                break
    # final Rayleigh-Ritz in H: ascending energies, residuals from an exact H psi
    y_final = apply_h(x) - e * x
    n_hpsi += nb
    theta_f, q, resid_f = _h_rayleigh_ritz(x, y_final, e)
    x = q.T @ x
    return dict(theta=theta_f, psi=x, resid=resid_f, iters=it, n_hpsi=n_hpsi,
                converged=converged, seconds=time.perf_counter() - t0)


def _h_rayleigh_ritz(x, y, e):
    """Rayleigh-Ritz in H for an orthonormal block with Y = (H - E) X.
    Returns theta ascending, the rotation q (new_b = sum_j q[j, b] x_j) and the
    residual norms ||H x'_b - theta_b x'_b||."""
    m = x.conj() @ y.T
    m = 0.5 * (m + m.conj().T)
    w, q = np.linalg.eigh(m)
    xr = q.T @ x
    yr = q.T @ y
    r = yr - w[:, None] * xr                   # (H - E)x' - (theta - E)x'
    resid = np.linalg.norm(r, axis=1)
    return w + e, q, resid
