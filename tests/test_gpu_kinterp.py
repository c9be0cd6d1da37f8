"""GPU wave-function interpolation between k-points against the oracle: energies
and states with a complete basis on a shared sphere (exact linear interpolation
of H), with a truncated basis on different spheres, the k1 end point, and
errors."""
import numpy as np
import pytest

from paper_1907_06821_amd import synth
from oracle.kinterp import interpolate
from tests._helpers import gpu_context, oracle_for, to_dev

pytestmark = pytest.mark.gpu


def _pair(k1, k2, kk, n=None):
    probs = [synth.small_nonlocal_problem(kpt=(k, -0.23, 0.07)) for k in (k1, k2, kk)]
    ops = [oracle_for(p) for p in probs]
    ctxs = [gpu_context(p, max_bands=4) for p in probs]
    e1, v1 = np.linalg.eigh(ops[0].dense())
    e2, v2 = np.linalg.eigh(ops[1].dense())
    n = n or len(e1)
    return ops, ctxs, e1[:n], np.ascontiguousarray(v1[:, :n].T), e2[:n], np.ascontiguousarray(v2[:, :n].T)


def _phase_aligned(a, b):
    ph = np.sum(b.conj() * a, axis=1)
    return a * (np.abs(ph) / ph)[:, None]


def test_complete_basis_matches_linear_interpolation(torch_cuda):
    import paper_1907_06821_amd as pw
    ops, ctxs, e1, v1, e2, v2 = _pair(0.11, 0.115, 0.1125)
    assert np.array_equal(ops[0].miller, ops[1].miller)
    h1, h2 = ops[0].dense(), ops[1].dense()
    for alpha in (0.0, 0.4, 1.0):
        eps, psik = pw.kinterp(ctxs[0], ctxs[1], ctxs[0], alpha, to_dev(v1), e1, to_dev(v2), e2)
        hmix = alpha * h1 + (1 - alpha) * h2
        assert np.max(np.abs(eps - np.linalg.eigvalsh(hmix))) < 1e-10
        p = psik.cpu().numpy()
        assert np.max(np.linalg.norm(p @ hmix.T - eps[:, None] * p, axis=1)) < 1e-9


def test_truncated_basis_matches_oracle(torch_cuda):
    import paper_1907_06821_amd as pw
    ops, ctxs, e1, v1, e2, v2 = _pair(0.11, 0.21, 0.16, n=10)
    assert not np.array_equal(ops[0].miller, ops[1].miller)
    for alpha in (0.25, 0.5):
        eps, psik = pw.kinterp(ctxs[0], ctxs[1], ctxs[2], alpha, to_dev(v1), e1, to_dev(v2), e2)
        oeps, opsi, _, _ = interpolate(alpha, e1, v1, ops[0].miller, e2, v2, ops[1].miller, ops[2].miller)
        assert np.max(np.abs(eps - oeps)) < 1e-11
        assert np.min(np.diff(oeps)) > 1e-6                      # non-degenerate: states unique up to phase
        p = psik.cpu().numpy()
        assert np.max(np.abs(_phase_aligned(p, opsi) - opsi)) < 1e-10
    eps, _ = pw.kinterp(ctxs[0], ctxs[1], ctxs[2], 1.0, to_dev(v1), e1, to_dev(v2), e2, states=False)
    assert np.max(np.abs(eps - e1)) < 1e-12


def test_kinterp_errors(torch_cuda):
    import paper_1907_06821_amd as pw
    ops, ctxs, e1, v1, e2, v2 = _pair(0.11, 0.21, 0.16, n=6)
    other = gpu_context(synth.config(1), max_bands=4)
    with pytest.raises(pw.PwError) as ex:                        # contexts of different cells
        pw.kinterp(ctxs[0], other, ctxs[2], 0.5, to_dev(v1), e1, to_dev(synth.start_vectors(1, 6, other.npw)), e2)
    assert ex.value.status == pw.PW_EINVAL
    with pytest.raises(pw.PwError) as ex:                        # k2 states all zero: no Gram-Schmidt
        pw.kinterp(ctxs[0], ctxs[1], ctxs[2], 0.5, to_dev(v1), e1, to_dev(np.zeros_like(v2)), e2)
    assert ex.value.status == pw.PW_ENOTPD


def test_single_state_closed_form(torch_cuda):
    """n = 1: U = S/|S| has modulus one, so eps(k) = alpha eps1 + (1 - alpha) eps2,
    and the state is alpha psi1 + (1 - alpha) U psi2."""
    import paper_1907_06821_amd as pw
    ops, ctxs, e1, v1, e2, v2 = _pair(0.11, 0.21, 0.16, n=1)
    for alpha in (0.3, 0.8):
        eps, psik = pw.kinterp(ctxs[0], ctxs[1], ctxs[0], alpha, to_dev(v1), e1, to_dev(v2), e2)
        assert abs(eps[0] - (alpha * e1[0] + (1 - alpha) * e2[0])) < 1e-13
        from oracle.kinterp import to_basis
        p2 = to_basis(v2, ops[1].miller, ops[0].miller)
        s = np.vdot(p2[0], v1[0])
        want = alpha * v1[0] + (1 - alpha) * (s / abs(s)) * p2[0]
        got = psik.cpu().numpy()[0]
        ph = np.vdot(want, got)
        assert np.max(np.abs(got * (abs(ph) / ph) - want)) < 1e-12
