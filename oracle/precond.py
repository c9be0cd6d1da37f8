"""Diagonal G-space preconditioners for the folded operator (oracle).

paper_M : the paper's G-space diagonal preconditioner (Sec. II.B, definition
          under the M' equation): M(G) = 1 / ((G^2 - E)^2 + dE^2).  The paper
          writes G^2 in Rydberg units; in Hartree the kinetic energy of a plane
          wave is T_G = (1/2)|G+k|^2, so M(G) = 1 / ((T_G - E)^2 + dE^2).
tpa2    : Teter-Payne-Allan's kinetic preconditioner (Phys. Rev. B 40, 12255,
          1989), K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4)
          with x = T_G / T_i and T_i = <psi_i| -(1/2) nabla^2 |psi_i>, squared
          because the folded operator grows as T_G^2 at high G.
"""
from __future__ import annotations

import numpy as np


def tpa(x):
    x = np.asarray(x, dtype=np.float64)
    num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x))
    return num / (num + 16.0 * x ** 4)


def band_kinetic(block, kin):
    """T_i = sum_G T_G |c_i(G)|^2 / sum_G |c_i(G)|^2 for each band."""
    p = np.abs(block) ** 2
    return (p @ np.asarray(kin)) / np.sum(p, axis=1)


def tpa2(kin, tband):
    """[nb, npw] folded TPA weights K(T_G / T_i)^2."""
    x = np.asarray(kin)[None, :] / np.asarray(tband)[:, None]
    return tpa(x) ** 2


def paper_m(kin, e_ref, delta_e):
    """[npw] weights 1 / ((T_G - E)^2 + dE^2)."""
    k = np.asarray(kin)
    return 1.0 / ((k - e_ref) ** 2 + delta_e ** 2)
