"""pw_dense_eigh_noalloc (work memory held by the library, no allocation per
call) against pw_dense_eigh on the same matrices: the same kernels on the same
inputs, so eigenvalues and eigenvectors agree bit for bit.  Two calls in a row,
the second smaller than the first (the array keeps the first call's contents),
through both eigensolver paths (n > 136: global memory; n <= 136: LDS), and
the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _hermitian(n, seed):
    rng = np.random.default_rng([41, seed])
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (a + a.conj().T)


@pytest.mark.parametrize("sizes", [(300, 100), (512, 7)])
def test_noalloc_eigh_equals_allocating_eigh(torch_cuda, sizes):
    import torch
    import paper_1907_06821_amd as pw
    for i, n in enumerate(sizes):
        a = _hermitian(n, 10 * n + i)
        t = torch.from_numpy(a).to("cuda")
        for key, ref in ((0, 0.0), (1, 0.3)):
            w1, r1, s1 = pw.dense_eigh(t, key=key, ref=ref)
            w2, r2, s2 = pw.dense_eigh(t, key=key, ref=ref, noalloc=True)
            assert torch.equal(w1, w2) and torch.equal(r1, r2) and s1 == s2
        ev = np.linalg.eigvalsh(a)
        assert np.max(np.abs(np.sort(w2.cpu().numpy()) - ev)) < 1e-12 * n * max(1.0, np.max(np.abs(ev)))


def test_noalloc_eigh_size_limit(torch_cuda):
    import torch
    import paper_1907_06821_amd as pw
    t = torch.from_numpy(_hermitian(513, 1)).to("cuda")
    with pytest.raises(pw.PwError) as e:
        pw.dense_eigh(t, noalloc=True)
    assert e.value.status == pw.PW_EINVAL
