"""Pins of the oracle's wave-function interpolation: Gram-Schmidt against a
library QR, the end points, and with a complete basis on a shared sphere the
interpolated Hamiltonian equals alpha H(k1) + (1 - alpha) H(k2) exactly (its
eigenvalues, and its eigenvectors as interpolated states); with a truncated
basis the error shrinks with the k spacing.  CPU only."""
import numpy as np

from paper_1907_06821_amd import synth
from oracle import hamiltonian as oh
from oracle.basis import plane_wave_basis
from oracle.kinterp import basis_map, gram_schmidt_rows, interpolate, to_basis


def _op(kpt):
    return oh.Operator.from_problem(synth.small_nonlocal_problem(kpt=kpt))


def test_gram_schmidt_equals_qr():
    rng = np.random.default_rng(3)
    s = rng.standard_normal((7, 7)) + 1j * rng.standard_normal((7, 7))
    u = gram_schmidt_rows(s)
    assert np.max(np.abs(u.conj() @ u.T - np.eye(7))) < 1e-13
    q, r = np.linalg.qr(s.T)                      # columns of s.T are the rows of s
    ph = np.diag(r) / np.abs(np.diag(r))
    assert np.max(np.abs(u - (q * ph[None, :]).T)) < 1e-12
    # a unitary matrix is left unchanged
    assert np.max(np.abs(gram_schmidt_rows(u) - u)) < 1e-13


def test_basis_map_round_trip():
    m1, _ = plane_wave_basis((7.0, 8.0, 9.0), 4.0, (0.11, -0.23, 0.07))
    m2, _ = plane_wave_basis((7.0, 8.0, 9.0), 4.0, (0.31, -0.23, 0.07))
    x = synth.start_vectors(99, 2, len(m1))
    y = to_basis(to_basis(x, m1, m2), m2, m1)
    keep = basis_map(m2, m1) >= 0
    assert np.array_equal(y[:, keep], x[:, keep]) and np.all(y[:, ~keep] == 0)
    assert 0 < (~keep).sum() < 0.2 * len(m1)


def test_end_point_k1_returns_its_energies():
    o1, o2 = _op((0.11, -0.23, 0.07)), _op((0.16, -0.23, 0.07))
    e1, v1 = np.linalg.eigh(o1.dense())
    e2, v2 = np.linalg.eigh(o2.dense())
    n = 12
    eps, _, _, _ = interpolate(1.0, e1[:n], v1[:, :n].T, o1.miller, e2[:n], v2[:, :n].T, o2.miller, o1.miller)
    assert np.max(np.abs(eps - e1[:n])) < 1e-13


def test_complete_basis_is_exact_linear_interpolation():
    """k1, k2 close enough to share the sphere: with every eigenstate, U = S is
    unitary and H(k) = alpha H(k1) + (1 - alpha) H(k2) exactly."""
    o1, o2 = _op((0.11, -0.23, 0.07)), _op((0.115, -0.23, 0.07))
    assert np.array_equal(o1.miller, o2.miller)
    h1, h2 = o1.dense(), o2.dense()
    e1, v1 = np.linalg.eigh(h1)
    e2, v2 = np.linalg.eigh(h2)
    for alpha in (0.0, 0.3, 0.75):
        eps, psik, u, s = interpolate(alpha, e1, v1.T, o1.miller, e2, v2.T, o2.miller, o1.miller)
        hmix = alpha * h1 + (1 - alpha) * h2
        assert np.max(np.abs(u - s)) < 1e-10
        assert np.max(np.abs(eps - np.linalg.eigvalsh(hmix))) < 1e-10
        r = psik @ hmix.T - eps[:, None] * psik
        assert np.max(np.linalg.norm(r, axis=1)) < 1e-9


def test_truncated_basis_error_shrinks_with_spacing():
    """The 10 lowest states at k1 and k2 interpolated to the midpoint: the error
    against the exact energies there falls as the spacing shrinks."""
    errs = []
    for dk in (0.2, 0.1, 0.05):
        k0 = 0.11
        o1, o2, om = _op((k0, -0.23, 0.07)), _op((k0 + dk, -0.23, 0.07)), _op((k0 + 0.5 * dk, -0.23, 0.07))
        e1, v1 = np.linalg.eigh(o1.dense())
        e2, v2 = np.linalg.eigh(o2.dense())
        n = 10
        eps, _, _, _ = interpolate(0.5, e1[:n], v1[:, :n].T, o1.miller, e2[:n], v2[:, :n].T, o2.miller, om.miller)
        errs.append(np.max(np.abs(eps[:6] - np.linalg.eigvalsh(om.dense())[:6])))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 5e-3, errs
