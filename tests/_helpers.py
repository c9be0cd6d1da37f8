"""Shared test plumbing: pair an oracle operator with a library context built
from the same synthetic problem (the two share only the raw inputs)."""
from __future__ import annotations

import numpy as np

from paper_1907_06821_amd import synth
from oracle.hamiltonian import Operator


def oracle_for(prob, vgrid=None):
    return Operator.from_problem(prob, vgrid=vgrid)


def gpu_context(prob, max_bands=None, flags=None, vgrid=None):
    import paper_1907_06821_amd as pw
    if flags is None:
        flags = pw.PW_PREP_C128
    return pw.Context.from_problem(prob, max_bands=max_bands, flags=flags, vgrid=vgrid)


def to_dev(a, dtype="complex128"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).astype(dtype))
    return t.to("cuda")


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_block(seed, nb, npw):
    return synth.start_vectors(99, nb, npw, seed=seed)
