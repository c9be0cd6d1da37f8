"""Pins of the shift-invert / inertia oracle (oracle.shift_invert).

The inertia count is checked against the eigenvalues of a dense eigensolve
(numpy) on the tiny cell, on a small cell with projectors and at a k-point, and
on random Hermitian matrices with a weak diagonal (so that Bunch-Kaufman takes
many 2x2 pivots); a diagonal matrix gives the count by inspection.  The
shift-invert eigenpairs are checked against the dense nearest eigenpairs.
"""
import numpy as np
import pytest

from paper_1907_06821_amd import synth
from oracle.eigen import nearest_eigenpairs
from oracle.hamiltonian import Operator
from oracle.shift_invert import (count_below, dense_shifted_into, ldl_inplace, nearest_by_shift_invert,
                                 negative_count)

torch = pytest.importorskip("torch")


def _problems():
    return [synth.config(1), synth.small_nonlocal_problem(nbands=6, e_ref=0.8),
            synth.small_nonlocal_problem(nbands=5, e_ref=0.6, kpt=(0.11, -0.07, 0.05))]


@pytest.mark.parametrize("k", range(3))
def test_dense_rows_match_dense_hamiltonian(k):
    op = Operator.from_problem(_problems()[k])
    h = op.dense()
    m = np.empty_like(h)
    dense_shifted_into(m, op.miller, op.kin, op.vgrid, op.beta, op.dproj, 0.37, rows=37)
    assert np.abs(m - (h - 0.37 * np.eye(op.npw))).max() < 1e-14


@pytest.mark.parametrize("k", range(3))
def test_inertia_counts_match_dense_spectrum(k):
    op = Operator.from_problem(_problems()[k])
    w = np.linalg.eigvalsh(op.dense())
    # shifts between eigenvalues (not on one): midpoints of a spread of gaps
    mids = 0.5 * (w[:-1] + w[1:])
    for s in list(mids[:: max(1, len(mids) // 9)]) + [w[0] - 1.0, w[-1] + 1.0]:
        assert count_below(op, float(s)) == int(np.sum(w < s))


def test_inertia_with_two_by_two_pivots():
    rng = np.random.default_rng(3)
    for n in (7, 60, 201):
        a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        a = a + a.conj().T
        a[np.diag_indices(n)] *= 1e-3
        ld, piv = ldl_inplace(torch.from_numpy(a.copy()))
        assert int((piv < 0).sum()) > 0
        assert negative_count(ld, piv) == int(np.sum(np.linalg.eigvalsh(a) < 0.0))


def test_inertia_of_diagonal_matrix():
    d = np.array([3.0, -1.0, 0.5, -2.0, -7.0, 4.0, 1e-9, -1e-9])
    ld, piv = ldl_inplace(torch.from_numpy(np.diag(d).astype(np.complex128)))
    assert negative_count(ld, piv) == 4


@pytest.mark.parametrize("k", range(3))
def test_shift_invert_matches_dense_nearest(k):
    prob = _problems()[k]
    op = Operator.from_problem(prob)
    lam, vec, _, gap = nearest_eigenpairs(op.dense(), prob.e_ref, prob.nbands)
    assert gap > 1e-6
    r = nearest_by_shift_invert(op, prob.e_ref, prob.nbands)
    assert np.abs(r["lam"] - lam).max() < 1e-11
    assert r["resid"].max() < 1e-10
    # same subspace
    s = np.linalg.svd(vec.conj() @ r["vecs"].T, compute_uv=False)
    assert s.min() > 1 - 1e-10
    assert r["below"] == int(np.sum(np.linalg.eigvalsh(op.dense()) < prob.e_ref))
