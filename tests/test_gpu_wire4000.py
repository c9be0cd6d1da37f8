"""H psi on the 4000-atom wire (50 x 50 x 200 bohr, 128 x 128 x 512 grid, Ecut
10 Ha, 755,605 plane waves, 16,000 projectors): 128-point xy planes and
512-point z columns take launch variants no smaller cell reaches, and its
complex128 projector table (193 GB) is never stored: complex128 H psi
generates the rows per call (PW_PREP_C128_OTF).

* Sixteen of the wire's atoms: every output coefficient of four dense random
  bands against the oracle's H psi, for complex128 with a stored table, with
  generated rows (one chunk, and chunks of 5 atoms with a ragged last one), and
  complex64 + BF16.
* The whole cell, 1024 bands in one call as the benchmark runs it: each band
  holds three plane waves, so the oracle can evaluate the exact matrix elements
  H_{GG'} of sampled output rows (oracle.hamiltonian.matrix_elements).
  complex128 (generated rows) must match them to 1e-12; complex64 + BF16 must
  stay within the bound of its arithmetic against the complex128 result.

Bound of complex64 + BF16: rounding to BF16 (unit roundoff u = 2^-8) of the
table, of the bands and of the projections gives at most about 4 u of the
nonlocal part; a single precision FFT pair on 2^23 points about 1e-5 of the
whole (unit roundoff 6e-8 times log2 N = 23 per transform, two transforms and
the product with V).
"""
import dataclasses

import numpy as np
import pytest

from paper_1907_06821_amd import synth
from tests._helpers import gpu_context, oracle_for, rel_err, to_dev

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8


def _few_atom_wire(natom=16):
    p = synth.config(5)
    return dataclasses.replace(p, pos=p.pos[:natom], depth=p.depth[:natom], dproj=p.dproj[:natom * p.nl])


@pytest.mark.parametrize("mode", ["c128", "c128_otf", "c128_otf_chunks", "c64"])
def test_hpsi_wire4000_grid_against_oracle(torch_cuda, mode):
    import paper_1907_06821_amd as pw
    prob = _few_atom_wire()
    op = oracle_for(prob)
    assert op.npw == 755605 and tuple(prob.grid) == (128, 128, 512)
    nb = 4
    flags = {"c128": pw.PW_PREP_C128, "c128_otf": pw.PW_PREP_C128_OTF, "c128_otf_chunks": pw.PW_PREP_C128_OTF,
             "c64": pw.PW_PREP_C64}[mode]
    ctx = gpu_context(prob, max_bands=nb, flags=flags)
    if mode == "c128_otf_chunks":
        ctx.set_otf_atoms(5)
    dtype = "complex64" if mode == "c64" else "complex128"
    c = synth.start_vectors(5, nb, op.npw, seed=3)
    got = pw.hpsi(ctx, to_dev(c, dtype), shift=prob.e_ref).cpu().numpy()
    ref = op.apply(c, shift=prob.e_ref)
    if mode != "c64":
        for b in range(nb):
            assert rel_err(got[b], ref[b]) < 1e-12
        return
    nl = (c @ op.beta.conj().T * op.dproj[None, :]) @ op.beta
    for b in range(nb):
        err = np.linalg.norm(got[b] - ref[b])
        bound = 4 * U_BF16 * np.linalg.norm(nl[b]) + 1e-5 * np.linalg.norm(ref[b])
        assert err <= bound, (b, err, bound)


def test_hpsi_wire4000_full_cell_sparse_bands(torch_cuda):
    import torch
    import paper_1907_06821_amd as pw
    from oracle.hamiltonian import matrix_elements, potential_fourier
    prob = synth.config(5)
    nb, nnz = prob.nbands, 3
    assert nb == 1024 and prob.natom == 4000
    op = oracle_for(prob)
    npw = op.npw
    rng = np.random.default_rng([5, 9])
    idx = np.stack([rng.choice(npw, size=nnz, replace=False) for _ in range(nb)])
    amp = (rng.standard_normal((nb, nnz)) + 1j * rng.standard_normal((nb, nnz))) / np.sqrt(2.0)
    x = torch.zeros((nb, npw), dtype=torch.complex128, device="cuda")
    x[torch.arange(nb, device="cuda")[:, None], torch.from_numpy(idx).to("cuda")] = torch.from_numpy(amp).to("cuda")
    shift = prob.e_ref
    vg = op.vgrid
    ctx = pw.Context.from_problem(prob, max_bands=nb, flags=pw.PW_PREP_C64 | pw.PW_PREP_C128_OTF, vgrid=vg)
    y = pw.hpsi(ctx, x, shift=shift)
    y32 = pw.hpsi(ctx, x.to(torch.complex64), shift=shift)
    # complex128 against the exact matrix elements of sampled rows of sampled bands
    vt = potential_fourier(op.vgrid)
    for b in (0, 517, nb - 1):
        rows = np.concatenate([idx[b], rng.choice(npw, size=253, replace=False)])
        h = matrix_elements(op, rows, idx[b], vt=vt)
        ref = h @ amp[b]
        ref[:nnz] -= shift * amp[b]
        got = y[b, torch.from_numpy(rows).to("cuda")].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), b
    # complex64 + BF16 against complex128, the nonlocal part from a context without atoms
    loc = pw.Context.from_problem(dataclasses.replace(prob, pos=prob.pos[:0], depth=prob.depth[:0],
                                                      dproj=prob.dproj[:0]), max_bands=nb,
                                  flags=pw.PW_PREP_C128, vgrid=vg)
    yl = pw.hpsi(loc, x, shift=shift)
    for b in range(0, nb, 31):
        ref = y[b]
        err = float(torch.linalg.vector_norm(y32[b].to(torch.complex128) - ref))
        nl = float(torch.linalg.vector_norm(ref - yl[b]))
        bound = 4 * U_BF16 * nl + 1e-5 * float(torch.linalg.vector_norm(ref))
        assert err <= bound, (b, err, bound)
