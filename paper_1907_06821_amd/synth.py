"""Seeded synthetic inputs for the folded-spectrum eigensolve.

This module builds the *inputs* of a plane-wave problem: the cell and grid, the
atom centres, the local-potential samples V(r_j) on the FFT grid, the
Kleinman-Bylander strengths D and random start vectors.  It holds none of the
method's arithmetic (no basis, no kinetic energies, no FFT, no projectors, no
Hamiltonian): the library and the CPU oracle each compute those from these
inputs on their own.

The paper's systems are copper nanowires of ~4000 atoms with 1 nm radius
electrodes and a 40 Ry cutoff (Sec. II, first paragraphs).  Their coordinates
and pseudopotentials are not available, so the workloads here are synthetic
stand-ins of the same shape: an fcc wire cut to a cylinder along z, each atom
carrying a Gaussian local well and four Gaussian Kleinman-Bylander projectors
(s + three p).

The sources w of the folded linear equation are sums of Gaussian blobs placed
near the cell's z boundary (the paper's w is nonzero only near the boundary,
far from the central region, Sec. II.A), given by their closed-form
plane-wave coefficients at Miller triples the caller supplies.

Seeds: ``numpy.random.default_rng([cfg_id, purpose])`` with purpose
0 = positions, 1 = D strengths, 2 = start vectors, 3 = vacancies,
4 = per-problem draws, 5 = network initialisation, 6 = linear-equation sources.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "config", "cubic_random_problem", "fcc_wire_sites",
    "gaussian_potential_grid", "start_vectors", "boundary_sources", "CONFIG_NAMES",
]

FCC_A = 6.82  # fcc lattice constant (bohr) of the copper-like wire


@dataclass
class Problem:
    """One synthetic plane-wave eigenproblem (inputs only).

    cell   : orthorhombic cell lengths (bohr), axis 2 = z (wire axis)
    grid   : FFT grid (n0, n1, n2)
    ecut   : kinetic cutoff, Ha: plane waves with (1/2)|G+k|^2 <= ecut
    kpt    : Bloch vector (Cartesian, 1/bohr)
    pos    : [natom, 3] atom centres (bohr)
    depth  : [natom] Gaussian well depth A_a (Ha, negative = attractive)
    width  : Gaussian width w: V_a(r) = A_a exp(-|r - R_a|^2 / w^2)
    nl     : projectors per atom (0 = local only, 4 = s + px, py, pz)
    sigma  : Gaussian width of the projector form factor exp(-|q|^2 sigma^2/2)
    dproj  : [natom * nl] KB strengths D_p (Ha), order per atom: s, px, py, pz
    e_ref  : reference energy (Ha)
    nbands : number of states wanted nearest e_ref
    """

    name: str
    cell: tuple
    grid: tuple
    ecut: float
    pos: np.ndarray
    depth: np.ndarray
    width: float
    nl: int
    sigma: float
    dproj: np.ndarray
    e_ref: float
    nbands: int
    kpt: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def natom(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nproj(self) -> int:
        return self.natom * self.nl

    def vgrid(self) -> np.ndarray:
        """V(r_j) on the grid, float64 [n0][n1][n2] C order."""
        return gaussian_potential_grid(self.cell, self.grid, self.pos, self.depth, self.width)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def fcc_wire_sites(cell, nsites, a=FCC_A):
    """The `nsites` fcc sites nearest the wire axis (x, y) = (L0/2, L1/2).

    The lattice is strained along z to a_z = L2 / round(L2 / a) so that the
    wire is seamless across the periodic boundary.  One site sits on the axis.
    Sites are ranked by (squared radius in units of (a/2)^2, z, y, x) with
    integer keys, so exact ties are broken reproducibly.
    """
    lx, ly, lz = cell
    nz = int(round(lz / a))
    az = lz / nz
    # half-lattice integer coordinates: fcc = all (i, j, k) with i + j + k even
    rmax = int(math.ceil(min(lx, ly) / a)) + 1
    cand = []
    for k in range(2 * nz):
        for j in range(-2 * rmax, 2 * rmax + 1):
            for i in range(-2 * rmax, 2 * rmax + 1):
                if (i + j + k) % 2:
                    continue
                cand.append((i * i + j * j, k, j, i))
    cand.sort()
    if len(cand) < nsites:
        raise ValueError("cell too small for the requested number of sites")
    out = np.empty((nsites, 3))
    for s, (_, k, j, i) in enumerate(cand[:nsites]):
        out[s] = (lx / 2 + i * a / 2, ly / 2 + j * a / 2, k * az / 2)
    # keep every site inside the cell with the lateral size checked
    if np.any(out[:, 0] < 0) or np.any(out[:, 0] >= lx) or np.any(out[:, 1] < 0) or np.any(out[:, 1] >= ly):
        raise ValueError("wire does not fit laterally in the cell")
    return out


def gaussian_potential_grid(cell, grid, pos, depth, width):
    """V(r_j) = sum_a A_a exp(-|r_j - R_a|^2_mi / w^2) on the grid.

    r_j = (j0 L0/n0, j1 L1/n1, j2 L2/n2); |.|_mi is the per-axis minimum-image
    distance.  The Gaussian factorises over the three axes, so the sum is taken
    as a product of per-axis factors contracted over atoms.
    """
    cell = np.asarray(cell, dtype=np.float64)
    n0, n1, n2 = (int(x) for x in grid)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    depth = np.asarray(depth, dtype=np.float64).reshape(-1)
    facs = []
    for ax, n in enumerate((n0, n1, n2)):
        r = np.arange(n) * (cell[ax] / n)
        d = r[None, :] - pos[:, ax][:, None]
        d -= cell[ax] * np.round(d / cell[ax])
        facs.append(np.exp(-(d * d) / (width * width)))
    if pos.shape[0] == 0:
        return np.zeros((n0, n1, n2))
    fx, fy, fz = facs
    fxy = (depth[:, None, None] * fx[:, :, None] * fy[:, None, :]).reshape(pos.shape[0], n0 * n1)
    v = fxy.T @ fz
    return np.ascontiguousarray(v.reshape(n0, n1, n2))


def start_vectors(cfg_id, nbands, npw, seed=0):
    """Random complex start block [nbands][npw], entries (x + iy)/sqrt(2), x, y ~ N(0, 1)."""
    rng = np.random.default_rng([cfg_id, 2, seed])
    x = rng.standard_normal((nbands, npw))
    y = rng.standard_normal((nbands, npw))
    return (x + 1j * y) / math.sqrt(2.0)


def boundary_sources(cfg_id, nrhs, miller, cell, kpt=(0.0, 0.0, 0.0), seed=0, nblob=8, width=1.0,
                     slab=0.1):
    """Right-hand sides w [nrhs][npw] of the folded linear equation, one unit-norm
    row per source: w_l(G) proportional to sum_k a_lk exp(-|q|^2 width^2 / 2 - i q.R_lk),
    q = 2 pi n / L + k, the plane-wave coefficients of Gaussian blobs of the given
    width centred at R_lk.  Blob centres: x, y uniform over the cell, z within
    slab * L_z of the plane z = 0 (the cell boundary along the wire); a_lk complex
    normal.  miller [npw][3] in the caller's coefficient order."""
    rng = np.random.default_rng([cfg_id, 6, seed])
    m = np.asarray(miller, dtype=np.float64).reshape(-1, 3)
    cell = np.asarray(cell, dtype=np.float64)
    q = 2.0 * np.pi * m / cell[None, :] + np.asarray(kpt, dtype=np.float64)[None, :]
    env = np.exp(-0.5 * width * width * np.sum(q * q, axis=1))
    out = np.empty((nrhs, m.shape[0]), dtype=np.complex128)
    for l in range(nrhs):
        r = rng.uniform(0.0, 1.0, size=(nblob, 3)) * cell[None, :]
        r[:, 2] = rng.uniform(-slab, slab, size=nblob) * cell[2]
        a = (rng.standard_normal(nblob) + 1j * rng.standard_normal(nblob)) / math.sqrt(2.0)
        w = (np.exp(-1j * (q @ r.T)) @ a) * env
        out[l] = w / np.linalg.norm(w)
    return out


def _kb_strengths(cfg_id, natom, nl, seed=0):
    if nl == 0:
        return np.zeros(0)
    rng = np.random.default_rng([cfg_id, 1, seed])
    ds = rng.uniform(0.5, 2.0, size=natom)
    dp = rng.uniform(0.5, 2.0, size=natom)
    d = np.empty((natom, nl))
    d[:, 0] = ds
    d[:, 1:] = dp[:, None]
    return d.reshape(-1)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

CONFIG_NAMES = ("tiny", "wire256", "wire2000", "batched", "wire4000")


def config(cfg, seed=0, free_electron=False, nbands=None, e_ref=None):
    """Build a named workload.

    1 / "tiny"      : 10^3 bohr cube, 16^3 grid, Ecut 6 Ha, 8 Gaussian wells
                      (depth -2 Ha, width 1 bohr) at uniform random centres,
                      local only, E_ref 0.5 Ha, 8 states.
    2 / "wire256"   : 20x20x80 bohr, 48x48x192, Ecut 10 Ha, 256-atom fcc wire,
                      wells -3 Ha / 1.2 bohr, 4 KB projectors (sigma 0.8 bohr),
                      D in U[0.5, 2] Ha, E_ref 0.3 Ha, 128 states.
    3 / "wire2000"  : 40x40x160, 96x96x384, Ecut 10 Ha, 2000 atoms, 512 states.
    5 / "wire4000"  : 50x50x200, 128x128x512, Ecut 10 Ha, 4040 sites minus 40
                      seeded vacancies, 1024 states.
    """
    if isinstance(cfg, str):
        cfg = {"tiny": 1, "wire256": 2, "wire2000": 3, "batched": 4, "wire4000": 5}[cfg]
    if cfg == 1:
        cell = (10.0, 10.0, 10.0)
        rng = np.random.default_rng([1, 0, seed])
        pos = rng.uniform(0.0, 1.0, size=(8, 3)) * np.asarray(cell)
        depth = np.full(8, -2.0)
        if free_electron:
            pos = pos[:0]
            depth = depth[:0]
        return Problem("tiny", cell, (16, 16, 16), 6.0, pos, depth, 1.0, 0, 0.8,
                       np.zeros(0), 0.5 if e_ref is None else e_ref, nbands or 8, seed=seed)
    if cfg in (2, 3, 5):
        cell, grid, nat, nb, nsites = {
            2: ((20.0, 20.0, 80.0), (48, 48, 192), 256, 128, 256),
            3: ((40.0, 40.0, 160.0), (96, 96, 384), 2000, 512, 2000),
            5: ((50.0, 50.0, 200.0), (128, 128, 512), 4000, 1024, 4040),
        }[cfg]
        pos = fcc_wire_sites(cell, nsites)
        if nsites > nat:
            rng = np.random.default_rng([cfg, 3, seed])
            drop = rng.choice(nsites, size=nsites - nat, replace=False)
            pos = np.delete(pos, np.sort(drop), axis=0)
        depth = np.full(nat, -3.0)
        d = _kb_strengths(cfg, nat, 4, seed)
        name = {2: "wire256", 3: "wire2000", 5: "wire4000"}[cfg]
        if free_electron:
            pos, depth, d = pos[:0], depth[:0], d[:0]
        return Problem(name, cell, grid, 10.0, pos, depth, 1.2, 4, 0.8, d,
                       0.3 if e_ref is None else e_ref, nbands or nb, seed=seed)
    raise ValueError(f"unknown config {cfg!r}; use batched_problems() for config 4")


def cubic_random_problem(side, grid, ecut, natom, e_ref, nbands, nl=4, seed=0, cfg_id=4,
                         depth=-3.0, width=1.2, sigma=0.8):
    """A cube of side `side` with `natom` Gaussian wells at uniform random centres."""
    rng = np.random.default_rng([cfg_id, 0, seed])
    pos = rng.uniform(0.0, side, size=(natom, 3))
    d = _kb_strengths(cfg_id, natom, nl, seed)
    return Problem(f"cube{side:g}_{natom}", (float(side),) * 3, tuple(grid), float(ecut), pos,
                   np.full(natom, depth), width, nl, sigma, d, float(e_ref), int(nbands), seed=seed)


def batched_problems(nprob=64, seed=0):
    """The uneven batch: cubes of side {8,10,12,14} bohr on {32,40,48,64}^3 grids,
    Ecut 8 Ha, 16..96 atoms with 4 projectors, E_ref ~ U[-0.5, 1.0] Ha, 16 states."""
    rng = np.random.default_rng([4, 4, seed])
    sides = (8.0, 10.0, 12.0, 14.0)
    grids = (32, 40, 48, 64)
    out = []
    for p in range(nprob):
        s = int(rng.integers(0, 4))
        nat = int(rng.integers(16, 97))
        e = float(rng.uniform(-0.5, 1.0))
        out.append(cubic_random_problem(sides[s], (grids[s],) * 3, 8.0, nat, e, 16,
                                        seed=seed * 1000 + p))
    return out


def small_nonlocal_problem(seed=0, grid=(12, 15, 20), cell=(7.0, 8.0, 9.0), ecut=4.0, natom=3,
                           nbands=6, e_ref=0.5, kpt=(0.0, 0.0, 0.0)):
    """A tiny orthorhombic cell with Gaussian wells and 4 KB projectors per atom.

    Grid sizes are chosen to exercise radices 2, 3, 4 and 5."""
    rng = np.random.default_rng([7, 0, seed])
    pos = rng.uniform(0.0, 1.0, size=(natom, 3)) * np.asarray(cell)
    d = _kb_strengths(7, natom, 4, seed)
    return Problem("small_nl", tuple(cell), tuple(grid), float(ecut), pos, np.full(natom, -2.5), 1.1,
                   4, 0.8, d, e_ref, nbands, kpt=tuple(kpt), seed=seed)


def mlp_init(seed=0, hidden=64):
    """Initial draws of the 3-hidden-hidden-1 preconditioner network, flat float64
    in the layout W1[h][3], b1[h], W2[h][h], b2[h], W3[h], b3: Glorot-uniform
    weights, zero biases, the last layer scaled by 0.1 so that the network starts
    near f = 0 (the plain preconditioner).  Seeds default_rng([5, seed])."""
    rng = np.random.default_rng([5, seed])

    def glorot(o, i):
        lim = math.sqrt(6.0 / (o + i))
        return rng.uniform(-lim, lim, size=(o, i))

    return np.concatenate([glorot(hidden, 3).ravel(), np.zeros(hidden), glorot(hidden, hidden).ravel(),
                           np.zeros(hidden), 0.1 * glorot(1, hidden).ravel(), np.zeros(1)])
