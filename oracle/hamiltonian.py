"""Plane-wave Kohn-Sham Hamiltonian (oracle): dense matrix and matrix-free H psi.

The paper solves H psi = E psi in a plane-wave basis with norm-conserving
Kleinman-Bylander pseudopotentials (Sec. II; the folded equation of
Sec. II.B applies H twice).  On the sphere basis {G} of the cell the matrix is

    H_{G G'} = (1/2)|G+k|^2 delta_{G G'} + Vt(G - G') + sum_p beta_p(G) D_p conj(beta_p(G'))

with the local potential given by its samples V(r_j) on the FFT grid
r_j = (j0 L0/N0, j1 L1/N1, j2 L2/N2) and

    Vt(q) = (1/N) sum_j V(r_j) exp(-i q . r_j),      N = N0 N1 N2,

q taken modulo the grid.  The KB projectors (synthetic stand-ins for the
paper's pseudopotentials) are, for atom a at R_a and q = G + k,

    beta_{a,j}(G) = N_s Y_j(q) exp(-|q|^2 s^2 / 2) exp(-i q . R_a) / sqrt(Omega)

with N_s = sqrt(8 pi^(3/2) s^3) (unit norm in the continuum), Y_s = 1 and
Y_{p,m} = sqrt(3) q_m / |q| (0 at q = 0), per atom in the order s, px, py, pz.
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------------------
# local potential
# ----------------------------------------------------------------------------

def gaussian_wells(cell, grid, pos, depth, width):
    """V(r_j) = sum_a A_a exp(-|r_j - R_a|^2 / w^2), distances by per-axis
    minimum image, evaluated point by point with the full 3-vector distance."""
    cell = np.asarray(cell, dtype=np.float64)
    n = [int(x) for x in grid]
    j0, j1, j2 = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    r = np.stack([j0 * cell[0] / n[0], j1 * cell[1] / n[1], j2 * cell[2] / n[2]], axis=-1)
    v = np.zeros(tuple(n))
    for a in range(np.asarray(pos).shape[0]):
        d = r - np.asarray(pos[a])[None, None, None, :]
        d = d - cell * np.round(d / cell)
        v += float(depth[a]) * np.exp(-np.sum(d * d, axis=-1) / (width * width))
    return v


def _dft_matrix(n, sign):
    """Dense 1D DFT matrix exp(sign * 2 pi i q j / n), angles reduced exactly
    as integers (q j mod n) before the trigonometric call."""
    q = np.arange(n)
    m = np.outer(q, q) % n
    ang = 2.0 * math.pi * m / n
    return np.cos(ang) + sign * 1j * np.sin(ang)


def potential_fourier(vgrid):
    """Vt(q) = (1/N) sum_j V(r_j) exp(-2 pi i sum_i q_i j_i / N_i) for every
    q on the grid, by direct separable summation (no FFT)."""
    v = np.asarray(vgrid, dtype=np.complex128)
    n0, n1, n2 = v.shape
    v = np.tensordot(_dft_matrix(n0, -1), v, axes=(1, 0))
    v = np.tensordot(_dft_matrix(n1, -1), v, axes=(1, 1)).transpose(1, 0, 2)
    v = np.tensordot(_dft_matrix(n2, -1), v, axes=(1, 2)).transpose(1, 2, 0)
    return v / (n0 * n1 * n2)


# ----------------------------------------------------------------------------
# nonlocal projectors
# ----------------------------------------------------------------------------

def projectors(miller, cell, pos, sigma, nl=4, kpt=(0.0, 0.0, 0.0), atoms=None):
    """beta_{a,j}(G) as a [natom*nl, npw] complex array (rows s, px, py, pz per atom).

    `atoms` optionally restricts the rows to a subset of atom indices."""
    cell = np.asarray(cell, dtype=np.float64)
    omega = float(np.prod(cell))
    q = 2.0 * math.pi * np.asarray(miller, dtype=np.float64) / cell[None, :] + np.asarray(kpt)[None, :]
    qn = np.sqrt(np.sum(q * q, axis=1))
    radial = math.sqrt(8.0 * math.pi ** 1.5 * sigma ** 3) * np.exp(-0.5 * (qn * sigma) ** 2) / math.sqrt(omega)
    ang = [np.ones_like(qn)]
    if nl == 4:
        safe = np.where(qn > 0.0, qn, 1.0)
        for m in range(3):
            ang.append(np.where(qn > 0.0, math.sqrt(3.0) * q[:, m] / safe, 0.0))
    elif nl != 1:
        raise ValueError("nl must be 1 (s) or 4 (s + p)")
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    idx = range(pos.shape[0]) if atoms is None else atoms
    rows = []
    for a in idx:
        phase = np.exp(-1j * (q @ pos[a]))
        for j in range(nl):
            rows.append(radial * ang[j] * phase)
    if not rows:
        return np.zeros((0, q.shape[0]), dtype=np.complex128)
    return np.array(rows)


# ----------------------------------------------------------------------------
# Hamiltonian
# ----------------------------------------------------------------------------

def dense_hamiltonian(miller, kin, vgrid, beta=None, dproj=None):
    """The full [npw, npw] FP64 matrix H_{GG'} defined in the module docstring."""
    miller = np.asarray(miller)
    grid = np.asarray(vgrid).shape
    vt = potential_fourier(vgrid)
    d = (miller[:, None, :] - miller[None, :, :]) % np.asarray(grid)[None, None, :]
    h = vt[d[..., 0], d[..., 1], d[..., 2]]
    h[np.diag_indices_from(h)] += kin
    if beta is not None and beta.shape[0]:
        h += (beta.T * np.asarray(dproj)[None, :]) @ beta.conj()
    return h


def hpsi(block, miller, kin, vgrid, beta=None, dproj=None, shift=0.0):
    """(H - shift) applied to a [nb, npw] coefficient block without forming H.

    Local part: place c(G) on the grid at n mod N, go to real space with the
    unnormalised exp(+iG.r) sum, multiply by V(r_j), come back with
    (1/N) exp(-iG.r) and keep the sphere.  Kinetic part: (1/2)|G+k|^2 c(G).
    Nonlocal part: sum_p beta_p D_p <beta_p|c>."""
    block = np.atleast_2d(np.asarray(block, dtype=np.complex128))
    vgrid = np.asarray(vgrid)
    n = vgrid.shape
    ntot = n[0] * n[1] * n[2]
    m = np.asarray(miller) % np.asarray(n)[None, :]
    out = np.empty_like(block)
    for b in range(block.shape[0]):
        g = np.zeros(n, dtype=np.complex128)
        g[m[:, 0], m[:, 1], m[:, 2]] = block[b]
        r = np.fft.ifftn(g) * ntot
        r *= vgrid
        back = np.fft.fftn(r) / ntot
        out[b] = back[m[:, 0], m[:, 1], m[:, 2]]
    out += (np.asarray(kin)[None, :] - shift) * block
    if beta is not None and beta.shape[0]:
        proj = block @ beta.conj().T          # [nb, nproj] = <beta_p | c_b>
        out += (proj * np.asarray(dproj)[None, :]) @ beta
    return out


class Operator:
    """Everything the oracle derives for one problem: basis, V, projectors.

    Built from a synthetic problem's raw inputs (cell, grid, ecut, kpt, atom
    centres, well depths/width, projector width, D)."""

    # projector tables larger than this many entries are not stored: apply()
    # then builds them a few atoms at a time (the same rows, summed by atom)
    MAX_TABLE = 200_000_000

    def __init__(self, cell, grid, ecut, vgrid, pos=None, sigma=0.8, nl=0, dproj=None,
                 kpt=(0.0, 0.0, 0.0)):
        from .basis import plane_wave_basis, fits_grid
        self.cell = tuple(float(x) for x in cell)
        self.grid = tuple(int(x) for x in grid)
        self.ecut = float(ecut)
        self.kpt = tuple(float(x) for x in kpt)
        self.miller, self.kin = plane_wave_basis(self.cell, self.ecut, self.kpt)
        if not fits_grid(self.miller, self.grid):
            raise ValueError("cutoff sphere does not fit the FFT grid")
        self.vgrid = np.asarray(vgrid, dtype=np.float64)
        self.nl = int(nl)
        self.pos = None if pos is None else np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        self.sigma = float(sigma)
        self.lazy = False
        if self.nl and pos is not None and len(pos):
            self.dproj = np.asarray(dproj, dtype=np.float64)
            self.lazy = len(self.pos) * self.nl * self.miller.shape[0] > self.MAX_TABLE
            self.beta = None if self.lazy else projectors(self.miller, self.cell, pos, sigma, nl, self.kpt)
        else:
            self.beta = None
            self.dproj = None

    @classmethod
    def from_problem(cls, prob, vgrid=None):
        v = prob.vgrid() if vgrid is None else vgrid
        return cls(prob.cell, prob.grid, prob.ecut, v, prob.pos, prob.sigma, prob.nl, prob.dproj,
                   prob.kpt)

    @property
    def npw(self):
        return self.miller.shape[0]

    def dense(self):
        if self.lazy:
            raise ValueError("no dense H for a cell whose projector table is not stored")
        return dense_hamiltonian(self.miller, self.kin, self.vgrid, self.beta, self.dproj)

    def apply(self, block, shift=0.0, atom_chunk=100):
        if not self.lazy:
            return hpsi(block, self.miller, self.kin, self.vgrid, self.beta, self.dproj, shift)
        block = np.atleast_2d(np.asarray(block, dtype=np.complex128))
        out = hpsi(block, self.miller, self.kin, self.vgrid, None, None, shift)
        for a0 in range(0, len(self.pos), atom_chunk):
            atoms = range(a0, min(a0 + atom_chunk, len(self.pos)))
            beta = projectors(self.miller, self.cell, self.pos, self.sigma, self.nl, self.kpt, atoms=atoms)
            d = self.dproj[a0 * self.nl:(a0 + len(atoms)) * self.nl]
            out += ((block @ beta.conj().T) * d[None, :]) @ beta
        return out


def matrix_elements(op, rows, cols, vt=None):
    """H_{G G'} for G in rows and G' in cols (index arrays into op.miller): the
    definition in the module docstring evaluated only there.  The projector rows
    are built at the needed plane waves alone, so this stays cheap for cells whose
    full projector table is never stored.  vt: optional precomputed
    potential_fourier(op.vgrid)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    grid = np.asarray(op.grid)
    if vt is None:
        vt = potential_fourier(op.vgrid)
    m = np.asarray(op.miller)
    d = (m[rows][:, None, :] - m[cols][None, :, :]) % grid[None, None, :]
    h = vt[d[..., 0], d[..., 1], d[..., 2]].astype(np.complex128)
    h += (rows[:, None] == cols[None, :]) * np.asarray(op.kin)[rows][:, None]
    if op.nl and op.pos is not None and len(op.pos):
        br = projectors(m[rows], op.cell, op.pos, op.sigma, op.nl, op.kpt)     # [nproj, |rows|]
        bc = projectors(m[cols], op.cell, op.pos, op.sigma, op.nl, op.kpt)     # [nproj, |cols|]
        h += (br.T * op.dproj[None, :]) @ bc.conj()
    return h
