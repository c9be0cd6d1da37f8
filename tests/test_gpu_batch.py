"""Batched solves of uneven cubic problems (fused launches over all problems
with a device mask, recorded graphs replayed each problem's in turn, or all as
one graph) against the same problems solved one by one: the same kernels in the
same order, so every check's residuals and the final eigenpairs agree bit for
bit."""
import numpy as np
import pytest

from paper_1907_06821_amd import synth

pytestmark = pytest.mark.gpu


def _compare(ind, eigs, ress, sts, status, psis, min_hist=6):
    import torch
    for i in range(len(ind)):
        e, r, st, psi = ind[i]
        assert sts[i]["iters"] == st["iters"], i
        assert sts[i]["n_hpsi"] == st["n_hpsi"], i
        assert status[i] == st["status"], i
        assert len(st["hist"]) >= min_hist
        assert np.array_equal(sts[i]["hist"], st["hist"]), i
        assert np.array_equal(eigs[i], e) and np.array_equal(ress[i], r), i
        assert torch.equal(psis[i], psi), i


@pytest.mark.parametrize("launch", [2, 1, 0])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_individual_solves(torch_cuda, precision, launch):
    import torch
    import paper_1907_06821_amd as pw
    probs = synth.batched_problems(6, seed=1)
    nb, nconv = 12, 8
    ctxs = [pw.Context.from_problem(p, max_bands=nb, flags=pw.PW_PREP_C128 | pw.PW_PREP_C64) for p in probs]
    starts = [torch.from_numpy(synth.start_vectors(4, nb, c.npw, seed=i)).to("cuda") for i, c in enumerate(ctxs)]
    kw = dict(tol=1e-7, maxit=130, check_every=20, precision=precision, precond=1, nconv=nconv)
    ind = []
    for c, p, s in zip(ctxs, probs, starts):
        psi = s.clone()
        e, r, st = pw.folded_cg_solve(c, p.e_ref, psi, raise_on_noconv=False, hist_len=16, **kw)
        ind.append((e, r, st, psi))
    psis = [s.clone() for s in starts]
    eigs, ress, sts, status = pw.batch_solve(ctxs, [p.e_ref for p in probs], psis, hist_len=16,
                                             raise_on_noconv=False, batch_launch=launch, **kw)
    # mode 2 fuses the FP64 solves; mixed precision falls back to mode 1
    assert all(s_["fused"] == (launch == 2 and precision == 0) for s_ in sts)
    _compare(ind, eigs, ress, sts, status, psis)     # several replays of the recorded rounds


@pytest.mark.parametrize("cells", ["one", "uneven"])
def test_fused_batch_equals_individual_solves_at_136_bands(torch_cuda, cells):
    """128 wanted + 8 buffer bands: the FP64 projector GEMMs of 129-144 bands run as the
    first 128 bands and the rest, in the fused batch's job lists as in a single solve, so
    the fused batch stays bit for bit each problem's own solve ("one": three starts on one
    cell).  Cells whose projector counts take different GEMM tiles ("uneven") cannot share
    one projection launch: the batch falls back to its recorded rounds, still bit for bit."""
    import torch
    import paper_1907_06821_amd as pw
    probs = synth.batched_problems(3, seed=2)
    if cells == "one":
        probs = [probs[0]] * 3
    nb, nconv = 136, 128
    ctxs = [pw.Context.from_problem(p, max_bands=nb) for p in probs]
    assert all(c.npw >= nb and c.nproj > 0 for c in ctxs)
    starts = [torch.from_numpy(synth.start_vectors(4, nb, c.npw, seed=i)).to("cuda") for i, c in enumerate(ctxs)]
    kw = dict(tol=1e-9, maxit=40, check_every=20, precision=0, precond=1, nconv=nconv)
    ind = []
    for c, p, s in zip(ctxs, probs, starts):
        psi = s.clone()
        e, r, st = pw.folded_cg_solve(c, p.e_ref, psi, raise_on_noconv=False, hist_len=16, **kw)
        ind.append((e, r, st, psi))
    psis = [s.clone() for s in starts]
    eigs, ress, sts, status = pw.batch_solve(ctxs, [p.e_ref for p in probs], psis, hist_len=16,
                                             raise_on_noconv=False, batch_launch=2, **kw)
    if cells == "one":
        assert all(s_["fused"] for s_ in sts)
    print("projector counts", [c.nproj for c in ctxs], "fused", [s_["fused"] for s_ in sts])
    _compare(ind, eigs, ress, sts, status, psis, min_hist=2)


@pytest.mark.parametrize("fault", [0, 2])
def test_fused_batch_with_finishing_problems(torch_cuda, fault):
    """Problems of the fused batch that converge at different checks drop out
    through the device mask while the others go on; with fault = 2 every problem
    restarts at its second check (host-forced loss of the Gram factorisation).
    Each problem's path is bit for bit that of its own solve."""
    import torch
    import paper_1907_06821_amd as pw
    probs = synth.batched_problems(8, seed=3)
    nb, nconv = 12, 8
    ctxs = [pw.Context.from_problem(p, max_bands=nb) for p in probs]
    starts = [torch.from_numpy(synth.start_vectors(4, nb, c.npw, seed=20 + i)).to("cuda") for i, c in enumerate(ctxs)]
    kw = dict(tol=1e-6, maxit=2000, check_every=20, precision=0, precond=1, nconv=nconv, fault_check=fault)
    ind = []
    for c, p, s in zip(ctxs, probs, starts):
        psi = s.clone()
        e, r, st = pw.folded_cg_solve(c, p.e_ref, psi, raise_on_noconv=False, hist_len=128, **kw)
        ind.append((e, r, st, psi))
    iters = sorted({st["iters"] for _, _, st, _ in ind})
    assert len(iters) >= 2, iters                     # some problems finish at a check, others go on
    psis = [s.clone() for s in starts]
    eigs, ress, sts, status = pw.batch_solve(ctxs, [p.e_ref for p in probs], psis, hist_len=128,
                                             raise_on_noconv=False, **kw)
    assert all(s_["fused"] for s_ in sts)
    if fault:
        assert all(s_["recoveries"] == 1 for s_ in sts)
    _compare(ind, eigs, ress, sts, status, psis, min_hist=2)


def test_batch_rejects_shared_contexts(torch_cuda):
    import torch
    import paper_1907_06821_amd as pw
    p = synth.batched_problems(1, seed=2)[0]
    c = pw.Context.from_problem(p, max_bands=8)
    psi = torch.from_numpy(synth.start_vectors(4, 8, c.npw)).to("cuda")
    with pytest.raises(pw.PwError):
        pw.batch_solve([c, c], [p.e_ref, p.e_ref], [psi, psi.clone()], maxit=20)
