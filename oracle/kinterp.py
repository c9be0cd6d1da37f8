"""Wave-function interpolation between two k-points (oracle, CPU, FP64).

Test infrastructure: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the library never does.

Sec. II.C (wave-function interpolation): with orthonormal eigenstates
psi_i(k1), psi_i(k2) and energies eps_i(k1), eps_i(k2) of two nearby k-points,
the Hamiltonian in between is taken linear in k, H(k) ~ alpha H(k1) +
(1 - alpha) H(k2) with alpha = (k - k2) / (k1 - k2).  In the basis psi_i(k1)

  H_ij(k) = alpha eps_i(k1) delta_ij + (1 - alpha) sum_m conj(U_im) U_jm eps_m(k2),

U the unitary matrix made by Gram-Schmidt from the overlaps
S_ij = <psi_j(k2)|psi_i(k1)> (the rows of S orthonormalised in order).
Diagonalising H(k) gives eps(k) and coefficient vectors c; the interpolated
state, continuous at both ends, is

  psi(k) = alpha sum_j c_j psi_j(k1) + (1 - alpha) sum_{j,l} c_j U_jl psi_l(k2).

Plane-wave coefficients at different k live on different cutoff spheres; they
are compared on common Miller triples, a coefficient missing from a sphere
being zero.
"""
from __future__ import annotations

import numpy as np


def basis_map(miller_from, miller_to):
    """For each Miller triple of miller_to, its row in miller_from, or -1."""
    index = {tuple(int(v) for v in m): i for i, m in enumerate(np.asarray(miller_from))}
    return np.array([index.get(tuple(int(v) for v in m), -1) for m in np.asarray(miller_to)], dtype=np.int64)


def to_basis(block, miller_from, miller_to):
    """Coefficients of a band-major block re-indexed onto another sphere."""
    idx = basis_map(miller_from, miller_to)
    out = np.zeros((block.shape[0], len(idx)), dtype=np.complex128)
    keep = idx >= 0
    out[:, keep] = block[:, idx[keep]]
    return out


def gram_schmidt_rows(s):
    """Classical Gram-Schmidt of the rows of s, in order: row i minus its
    components along the already orthonormalised rows, then normalised."""
    s = np.asarray(s, dtype=np.complex128)
    u = np.zeros_like(s)
    for i in range(s.shape[0]):
        v = s[i].copy()
        for a in range(i):
            v = v - np.vdot(u[a], s[i]) * u[a]
        u[i] = v / np.linalg.norm(v)
    return u


def interpolate(alpha, eps1, psi1, miller1, eps2, psi2, miller2, miller_k):
    """Energies (ascending) and states (on miller_k) at the k with the given alpha.
    Returns (eps, psi_k, U, S)."""
    p2 = to_basis(psi2, miller2, miller1)
    s = psi1 @ p2.conj().T                              # s[i, j] = <psi_j(k2)|psi_i(k1)>
    u = gram_schmidt_rows(s)
    eps1 = np.asarray(eps1, dtype=np.float64)
    eps2 = np.asarray(eps2, dtype=np.float64)
    hk = alpha * np.diag(eps1) + (1.0 - alpha) * (u.conj() * eps2[None, :]) @ u.T
    hk = 0.5 * (hk + hk.conj().T)
    eps, c = np.linalg.eigh(hk)
    coef = c.T                                          # row b: coefficients of state b
    psik = alpha * coef @ to_basis(psi1, miller1, miller_k) + \
        (1.0 - alpha) * (coef @ u) @ to_basis(psi2, miller2, miller_k)
    return eps, psik, u, s
