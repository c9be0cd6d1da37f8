"""Eigenpairs nearest E by shift-invert, and their completeness by Sylvester inertia (oracle).

The paper needs the eigenstates of H nearest a transport energy E (Sec. II.B,
paragraph on methods for a few states near E).  For a cell whose dense H fits
in host memory but is too large for a full eigendecomposition (the 256-atom
wire: 48,369 plane waves, a 37 GB matrix), the oracle takes two library routes
that do not involve the folded-spectrum method at all:

  * Sylvester's law of inertia: for a Hermitian M = H - sigma I factored as
    M = P L D L^H P^T (Bunch-Kaufman, D block diagonal with 1x1 and 2x2
    Hermitian blocks), the number of eigenvalues of H below sigma equals the
    number of negative eigenvalues of D.  Two such counts bracket how many
    eigenvalues lie in a window [E - r, E + r).
  * Lanczos (ARPACK) on the inverse (H - E I)^{-1}: its eigenvalues of largest
    magnitude are 1/(lambda - E) for the lambda nearest E, with the same
    eigenvectors.  Each Lanczos step is one solve with the LDL^H factors.

The factorisation is a library primitive (LAPACK's Hermitian indefinite
factorisation through torch.linalg.ldl_factor_ex, in place); the dense matrix
is the definition H_{GG'} of oracle.hamiltonian written into a preallocated
array a block of rows at a time.  Rayleigh quotients and residuals of the
returned vectors come from the matrix-free H psi (numpy FFT), a route
independent of the dense matrix.

Test infrastructure: used by tests/ and the scripts under tests/golden/ only.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import potential_fourier


def work_matrix(n):
    """An [n, n] complex128 torch CPU tensor in column-major order: LAPACK's
    factorisation then works on it in place (a row-major one is copied first)."""
    import torch
    return torch.empty_strided((n, n), (1, n), dtype=torch.complex128)


def dense_shifted_into(out, miller, kin, vgrid, beta=None, dproj=None, sigma=0.0, rows=512):
    """Write H - sigma I (the dense matrix of oracle.hamiltonian.dense_hamiltonian)
    into `out`, an [npw, npw] complex128 array (numpy, or a torch CPU tensor of
    either memory order), `rows` rows at a time so that no npw x npw temporary
    is formed.  A column-major torch tensor receives the conjugate transpose of
    each row block as a block of columns (H is Hermitian), a contiguous write."""
    miller = np.asarray(miller)
    grid = np.asarray(np.asarray(vgrid).shape)
    vt = potential_fourier(vgrid).ravel()
    npw = miller.shape[0]
    kin = np.asarray(kin, dtype=np.float64)
    bt = None
    if beta is not None and beta.shape[0]:
        bt = beta.T * np.asarray(dproj, dtype=np.float64)[None, :]    # [npw, nproj] beta_p(G) D_p
        bconj = beta.conj()                                           # [nproj, npw]
    for r0 in range(0, npw, rows):
        r1 = min(npw, r0 + rows)
        d = (miller[r0:r1, None, :] - miller[None, :, :]) % grid[None, None, :]
        blk = vt[(d[..., 0] * grid[1] + d[..., 1]) * grid[2] + d[..., 2]]
        idx = np.arange(r0, r1)
        blk[idx - r0, idx] += kin[r0:r1] - sigma
        if bt is not None:
            blk += bt[r0:r1] @ bconj
        if isinstance(out, np.ndarray):
            out[r0:r1] = blk
        elif out.stride(0) == 1:
            import torch
            out[:, r0:r1] = torch.from_numpy(np.ascontiguousarray(blk.conj().T))
        else:
            import torch
            out[r0:r1] = torch.from_numpy(blk)
    return out


def ldl_inplace(m):
    """Bunch-Kaufman LDL^H of the Hermitian torch CPU tensor m, in place.
    Returns (m holding the compact factors, pivots) as LAPACK's Hermitian
    indefinite factorisation defines them."""
    import torch
    n = m.shape[0]
    piv = torch.empty(n, dtype=torch.int32)
    info = torch.empty((), dtype=torch.int32)
    torch.linalg.ldl_factor_ex(m, hermitian=True, out=(m, piv, info))
    if int(info) < 0:
        raise RuntimeError(f"LDL^H factorisation failed (info {int(info)})")
    return m, piv


def negative_count(ld, piv):
    """Number of negative eigenvalues of the block-diagonal D of a compact LDL^H
    factorisation (ld, piv as ldl_inplace returns them): 1x1 blocks where the
    pivot is positive, 2x2 Hermitian blocks where two consecutive pivots are
    negative.  By Sylvester's law of inertia this is the number of negative
    eigenvalues of the factored matrix."""
    import torch
    p = piv.numpy()
    n = p.shape[0]
    diag = torch.diagonal(ld).real.numpy().copy()
    sub = torch.diagonal(ld, offset=-1).numpy().copy()
    sup = torch.diagonal(ld, offset=1).numpy().copy()
    neg = 0
    k = 0
    while k < n:
        if p[k] > 0:
            neg += int(diag[k] < 0.0)
            k += 1
        else:
            # 2x2 block [[a, b], [conj b, c]]: the off-diagonal sits on one side of the
            # diagonal depending on the storage triangle; the other side holds zero
            b = sub[k] if abs(sub[k]) >= abs(sup[k]) else np.conj(sup[k])
            w = np.linalg.eigvalsh(np.array([[diag[k], b], [np.conj(b), diag[k + 1]]]))
            neg += int(np.sum(w < 0.0))
            k += 2
    return neg


def count_below(op, sigma, work=None):
    """Number of eigenvalues of the operator's dense H strictly below sigma
    (Sylvester inertia of H - sigma I).  `work`: optional preallocated torch
    complex128 [npw, npw] array (work_matrix) that is overwritten."""
    m = work if work is not None else work_matrix(op.npw)
    dense_shifted_into(m, op.miller, op.kin, op.vgrid, op.beta, op.dproj, sigma)
    ld, piv = ldl_inplace(m)
    return negative_count(ld, piv)


def nearest_by_shift_invert(op, e_ref, k, work=None, tol=1e-13, ncv=None, v0_seed=0, log=None):
    """The k eigenpairs of H nearest e_ref by Lanczos on (H - e_ref I)^{-1}.

    Returns a dict with lam [k] ascending (Rayleigh quotients of the Lanczos
    vectors with the matrix-free H psi), vecs [k, npw] band-major, resid [k]
    (||H v - lam v|| with the matrix-free H psi), below (eigenvalues below
    e_ref by inertia) and the Lanczos values 1/(lambda - E)."""
    import torch
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = op.npw
    m = work if work is not None else work_matrix(n)
    dense_shifted_into(m, op.miller, op.kin, op.vgrid, op.beta, op.dproj, e_ref)
    if log:
        log("dense H - E I built")
    ld, piv = ldl_inplace(m)
    below = negative_count(ld, piv)
    if log:
        log(f"factorised: {below} eigenvalues below E")
    nsolve = [0]

    def solve(x):
        b = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(n, -1)))
        nsolve[0] += 1
        return torch.linalg.ldl_solve(ld, piv, b, hermitian=True).numpy().reshape(np.shape(x))

    opinv = LinearOperator((n, n), matvec=solve, dtype=np.complex128)
    v0 = np.random.default_rng(v0_seed).standard_normal(n) + 0j
    mu, vec = eigsh(opinv, k=k, which="LM", tol=tol, ncv=ncv or min(n, 2 * k + 32), v0=v0)
    if log:
        log(f"Lanczos done after {nsolve[0]} solves")
    vecs = np.ascontiguousarray(vec.T)
    vecs /= np.linalg.norm(vecs, axis=1)[:, None]
    hv = op.apply(vecs)
    lam = np.real(np.sum(vecs.conj() * hv, axis=1))
    resid = np.linalg.norm(hv - lam[:, None] * vecs, axis=1)
    order = np.argsort(lam, kind="stable")
    return {"lam": lam[order], "vecs": vecs[order], "resid": resid[order], "below": below,
            "lanczos_inv": np.asarray(mu)[order], "solves": nsolve[0]}
