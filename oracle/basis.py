"""Plane-wave basis on the cutoff sphere (oracle).

The paper expands wave functions in plane waves up to a kinetic cutoff
(Sec. II, computational details: 40 Ry).  For an orthorhombic cell of lengths
L_i the reciprocal vectors are G = 2 pi (n0/L0, n1/L1, n2/L2) for integer
Miller triples n, and the basis is every n with (1/2)|G + k|^2 <= Ecut (Ha).

Order: lexicographic in the signed triple (n0, n1, n2).  Within one z-column
(fixed n0, n1) the kept n2 form one contiguous run of consecutive integers.
"""
from __future__ import annotations

import math

import numpy as np


def kinetic(miller, cell, kpt=(0.0, 0.0, 0.0)):
    """(1/2)|G + k|^2 in Ha for each Miller triple."""
    miller = np.asarray(miller, dtype=np.float64)
    q = 2.0 * math.pi * miller / np.asarray(cell, dtype=np.float64)[None, :] + np.asarray(kpt)[None, :]
    return 0.5 * np.sum(q * q, axis=1)


def plane_wave_basis(cell, ecut, kpt=(0.0, 0.0, 0.0)):
    """Miller triples with (1/2)|G+k|^2 <= ecut, lexicographically ordered.

    Returns (miller int64 [npw, 3], kinetic float64 [npw]).
    """
    gmax = math.sqrt(2.0 * ecut)
    ranges = []
    for L, k in zip(cell, kpt):
        nmax = int(math.ceil((gmax + abs(k)) * L / (2.0 * math.pi))) + 1
        ranges.append(np.arange(-nmax, nmax + 1))
    n0, n1, n2 = np.meshgrid(*ranges, indexing="ij")
    cand = np.stack([n0.ravel(), n1.ravel(), n2.ravel()], axis=1)
    t = kinetic(cand, cell, kpt)
    keep = cand[t <= ecut]
    # meshgrid with indexing="ij" already enumerates lexicographically; sort anyway
    order = np.lexsort((keep[:, 2], keep[:, 1], keep[:, 0]))
    keep = keep[order].astype(np.int64)
    return keep, kinetic(keep, cell, kpt)


def cutoff_margin(cell, ecut, kpt=(0.0, 0.0, 0.0)):
    """Smallest |(1/2)|G+k|^2 - ecut| over all G: how far the nearest plane wave
    sits from the sphere boundary.  Used to show that "<=" vs "<" and rounding
    cannot change the basis."""
    gmax = math.sqrt(2.0 * ecut)
    ranges = []
    for L, k in zip(cell, kpt):
        nmax = int(math.ceil((gmax + abs(k)) * L / (2.0 * math.pi))) + 2
        ranges.append(np.arange(-nmax, nmax + 1))
    n0, n1, n2 = np.meshgrid(*ranges, indexing="ij")
    cand = np.stack([n0.ravel(), n1.ravel(), n2.ravel()], axis=1)
    return float(np.min(np.abs(kinetic(cand, cell, kpt) - ecut)))


def fits_grid(miller, grid):
    """True when distinct Miller triples land on distinct grid points, i.e.
    2 max|n_i| + 1 <= N_i on every axis (no wrap-around collisions)."""
    m = np.max(np.abs(np.asarray(miller)), axis=0)
    return bool(np.all(2 * m + 1 <= np.asarray(grid)))


def shells(kin, tol=1e-9):
    """Shell index of every plane wave: sort (1/2)|G+k|^2 ascending and open a new
    shell wherever two consecutive values differ by more than `tol` Ha.
    Returns (shell_id int64 [npw], shell_T [nshell] = smallest T in each shell)."""
    kin = np.asarray(kin, dtype=np.float64)
    order = np.argsort(kin, kind="stable")
    ts = kin[order]
    new = np.empty(ts.shape[0], dtype=bool)
    if ts.shape[0]:
        new[0] = True
        new[1:] = np.diff(ts) > tol
    sid_sorted = np.cumsum(new) - 1
    sid = np.empty_like(sid_sorted)
    sid[order] = sid_sorted
    return sid.astype(np.int64), ts[new]
