"""GPU parity of the small dense FP64 kernels (Jacobi eigensolver for the
Rayleigh-Ritz step, Cholesky + inverse for the Gram step) against numpy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _herm(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, _ = np.linalg.qr(x)
    w = np.sort(rng.uniform(-1, 1, n)) * spread
    return (q * w) @ q.conj().T, w


@pytest.mark.parametrize("n", [1, 2, 7, 33, 64, 128, 136, 137, 160, 300, 1024])
def test_dense_eigh_random(torch_cuda, n):
    import torch
    import paper_1907_06821_amd as pw
    a, w_ref = _herm(n, n)
    t = torch.from_numpy(a).to("cuda")
    w, r, sweeps = pw.dense_eigh(t, key=0)
    w = w.cpu().numpy()
    r = r.cpu().numpy()
    print(f"n={n} sweeps={sweeps}")
    assert np.max(np.abs(w - w_ref)) < 1e-13 * max(1, n)
    # rows of R are eigenvectors: R A R^H = diag(w) (band-major convention R . A^T)
    v = r.T                                   # columns are eigenvectors
    assert np.max(np.abs(a @ v - v * w[None, :])) < 1e-11
    assert np.max(np.abs(v.conj().T @ v - np.eye(n))) < 1e-12
    assert sweeps <= 12


def test_dense_eigh_near_diagonal(torch_cuda):
    """A nearly converged Rayleigh-Ritz matrix (what late solver checks see): small
    eigenvalues to absolute 1e-15 and eigenvectors to 1e-12."""
    import torch
    import paper_1907_06821_amd as pw
    n = 128
    rng = np.random.default_rng(3)
    d = np.diag(np.linspace(1e-6, 1e-2, n)).astype(complex)
    e = 1e-9 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    a = d + e + e.conj().T
    w, r, sweeps = pw.dense_eigh(torch.from_numpy(a).to("cuda"))
    print("near-diagonal QL iterations", sweeps)
    assert np.max(np.abs(w.cpu().numpy() - np.linalg.eigvalsh(a))) < 1e-15
    v = r.cpu().numpy().T
    assert np.max(np.abs(a @ v - v * w.cpu().numpy()[None, :])) < 1e-15
    assert np.max(np.abs(v.conj().T @ v - np.eye(n))) < 1e-12
    assert 0 <= sweeps <= 10


@pytest.mark.parametrize("n", [136, 512])
def test_dense_eigh_folded_clusters(torch_cuda, n):
    """The spectrum a folded Rayleigh-Ritz matrix has: pairs (x - E)^2 of states
    either side of E nearly coincide, plus an exact degeneracy."""
    import torch
    import paper_1907_06821_amd as pw
    rng = np.random.default_rng(n + 1)
    x = np.sort(rng.uniform(-0.4, 0.4, n // 2))
    w_ref = np.sort(np.concatenate([x ** 2, (x + 1e-9) ** 2]))
    w_ref[5] = w_ref[4]                                  # an exact double eigenvalue
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    a = (q * w_ref) @ q.conj().T
    w, r, _ = pw.dense_eigh(torch.from_numpy(a).to("cuda"))
    w = w.cpu().numpy()
    v = r.cpu().numpy().T
    assert np.max(np.abs(w - w_ref)) < 1e-14
    assert np.max(np.abs(a @ v - v * w[None, :])) < 1e-13
    assert np.max(np.abs(v.conj().T @ v - np.eye(n))) < 1e-12


def test_dense_eigh_key_orders_by_distance(torch_cuda):
    import torch
    import paper_1907_06821_amd as pw
    a, w_ref = _herm(20, 5)
    w, r, _ = pw.dense_eigh(torch.from_numpy(a).to("cuda"), key=1, ref=0.1)
    w = w.cpu().numpy()
    assert np.all(np.diff(np.abs(w - 0.1)) >= 0)
    assert np.max(np.abs(np.sort(w) - w_ref)) < 1e-13


@pytest.mark.parametrize("n, split", [(128, 64), (300, 150), (1024, 512)])
def test_dense_eigh_decoupled_blocks(torch_cuda, n, split):
    """Degenerate tridiagonals: a block-diagonal matrix, whose reduction leaves an exact
    zero off-diagonal at the block boundary, where a tear of the divide and conquer
    falls (the merge across it has nothing to do), and a diagonal matrix with repeated
    entries (every off-diagonal zero, no merge at all).  One-workgroup path at 128,
    the launches over the GPU beyond 136."""
    import torch
    import paper_1907_06821_amd as pw
    a1, _ = _herm(split, n + 1)
    a2, _ = _herm(n - split, n + 2)
    a = np.zeros((n, n), complex)
    a[:split, :split] = a1
    a[split:, split:] = a2 + 0.25 * np.eye(n - split)
    rng = np.random.default_rng(n)
    d = np.repeat(rng.uniform(-1, 1, n // 4), 4)[:n]
    for m in (a, np.diag(d).astype(complex)):
        w, r, _ = pw.dense_eigh(torch.from_numpy(m).to("cuda"), key=0)
        w = w.cpu().numpy()
        v = r.cpu().numpy().T
        assert np.max(np.abs(w - np.linalg.eigvalsh(m))) < 1e-13 * max(1, n)
        assert np.max(np.abs(m @ v - v * w[None, :])) < 1e-11
        assert np.max(np.abs(v.conj().T @ v - np.eye(n))) < 1e-12


@pytest.mark.parametrize("n", [1, 5, 64, 128, 136, 137, 200, 256, 300, 1024])
def test_dense_chol_inv(torch_cuda, n):
    import torch
    import paper_1907_06821_amd as pw
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n + 20, n)) + 1j * rng.standard_normal((n + 20, n))
    s = x.conj().T @ x                        # Hermitian positive definite
    t = pw.dense_chol_inv(torch.from_numpy(s).to("cuda")).cpu().numpy()
    ell = np.linalg.cholesky(s)
    assert np.max(np.abs(t - np.linalg.inv(ell).conj())) < 1e-10 * np.linalg.cond(ell)
    # T S T^H... in band-major terms: (conj T) S (conj T)^H = Linv S Linv^H = I
    li = t.conj()
    assert np.max(np.abs(li @ s @ li.conj().T - np.eye(n))) < 1e-10


def test_dense_chol_inv_not_pd(torch_cuda):
    import torch
    import paper_1907_06821_amd as pw
    s = np.eye(4, dtype=complex)
    s[2, 2] = -1.0
    with pytest.raises(pw.PwError) as e:
        pw.dense_chol_inv(torch.from_numpy(s).to("cuda"))
    assert e.value.status == pw.PW_ENOTPD


@pytest.mark.parametrize("n, bad", [(4, 2), (300, 250), (1024, 700)])
def test_dense_chol_inv_not_pd_reports_the_pivot(torch_cuda, n, bad):
    """The leading bad x bad block is positive definite and pivot `bad` is not:
    the blocked factorisation (n > 136) reports the first failing pivot of the
    whole matrix, not of its diagonal block."""
    import torch
    import paper_1907_06821_amd as pw
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n + 20, n)) + 1j * rng.standard_normal((n + 20, n))
    s = x.conj().T @ x
    s[bad, bad] = -1e6
    with pytest.raises(pw.PwError) as e:
        pw.dense_chol_inv(torch.from_numpy(s).to("cuda"))
    assert e.value.status == pw.PW_ENOTPD
    assert f"pivot {bad}" in str(e.value)
