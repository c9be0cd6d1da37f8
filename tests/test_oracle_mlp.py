"""CPU pins of the oracle's preconditioner network: gradient against central
finite differences, the loss against the cosine written on plain vectors,
closed-form cases of the loss and of Adam's first step, and the shell tables
(error direction, shell sums, metric weights) on inputs built so that the
answer is known."""
import numpy as np
import pytest

from paper_1907_06821_amd import synth
from oracle import mlp as om


def _random_tables(rng, k=2, ns=5, nb=3):
    xs = rng.uniform(0.0, 1.0, (k, ns, nb, 3))
    a = rng.standard_normal((k, ns, nb))
    b = rng.uniform(0.1, 1.0, (k, ns, nb))
    e = rng.uniform(0.5, 2.0, (k, nb))
    return xs, a, b, e


def test_init_layout_and_start_near_zero():
    theta = synth.mlp_init(0)
    assert theta.size == om.NPARAM == 4481
    w1, b1, w2, b2, w3, b3 = om.unpack(theta)
    assert np.all(b1 == 0) and np.all(b2 == 0) and b3 == 0
    assert np.max(np.abs(w3)) <= 0.1 * np.sqrt(6.0 / 65) + 1e-15
    f, _ = om.forward(theta, np.random.default_rng(0).uniform(0, 1, (50, 3)))
    assert np.max(np.abs(f)) < 0.5                       # starts close to the plain preconditioner


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = synth.mlp_init(1) + 0.05 * rng.standard_normal(om.NPARAM)
    xs, a, b, e = _random_tables(rng)
    loss, grad = om.loss_grad(theta, xs, a, b, e)
    assert loss == pytest.approx(om.loss(theta, xs, a, b, e), abs=1e-15)
    h = 1e-6
    fd = np.empty(om.NPARAM)
    for j in range(om.NPARAM):
        tp = theta.copy()
        tp[j] += h
        tm = theta.copy()
        tm[j] -= h
        fd[j] = (om.loss(tp, xs, a, b, e) - om.loss(tm, xs, a, b, e)) / (2 * h)
    assert np.max(np.abs(fd - grad)) < 1e-8 * max(1.0, np.max(np.abs(grad)))
    assert np.max(np.abs(grad)) > 1e-4                   # not trivially zero


def _orthonormal_split(rng, npw, nb):
    z = rng.standard_normal((npw, 2 * nb)) + 1j * rng.standard_normal((npw, 2 * nb))
    q, _ = np.linalg.qr(z)
    return q[:, :nb].T.copy(), q[:, nb:].T.copy()        # converged block, an orthogonal complement part


def _zero_output(theta):
    t = theta.copy()
    t[-om.H - 1:] = 0.0                                  # W3 = 0, b3 = 0  ->  f = 0
    return t


@pytest.mark.parametrize("weighted", [False, True])
def test_tables_and_loss_are_the_cosine_of_known_vectors(weighted):
    """x = C x* + o with o orthogonal to span(x*): the error direction is exactly o,
    and with f = 0 the loss is 1 - Re<K0 g, o> / (|K0 g| |o|) per band (in the
    diag(w) metric when weighted)."""
    rng = np.random.default_rng(4)
    npw, nb, nshell = 40, 3, 6
    xc, o = _orthonormal_split(rng, npw, nb)
    c = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
    xs = c @ xc + o
    g = rng.standard_normal((nb, npw)) + 1j * rng.standard_normal((nb, npw))
    k0 = rng.uniform(0.1, 1.0, (nb, npw))
    shell = np.sort(rng.integers(0, nshell, npw))
    wsh = rng.uniform(0.5, 3.0, nshell) if weighted else None
    a, b, e = om.harvest_tables(xs, xc, g, k0, shell, nshell, weight=wsh)
    wg = np.ones(npw) if wsh is None else wsh[shell]
    kg = k0 * g
    want = []
    for i in range(nb):
        ip = np.sum(wg * np.real(np.conj(o[i]) * kg[i]))
        want.append(1.0 - ip / (np.sqrt(np.sum(wg * np.abs(kg[i]) ** 2)) * np.sqrt(np.sum(wg * np.abs(o[i]) ** 2))))
    x = om.features(np.arange(nshell, dtype=float), np.ones(nb), 0.3, 10.0)
    theta = _zero_output(synth.mlp_init(2))
    got = om.loss(theta, x[None], a[None], b[None], e[None])
    assert got == pytest.approx(np.mean(want), abs=1e-13)
    # a constant network output rescales K uniformly and leaves every cosine alone
    t2 = theta.copy()
    t2[-1] = 0.7
    assert om.loss(t2, x[None], a[None], b[None], e[None]) == pytest.approx(got, abs=1e-13)


def test_perfect_direction_has_zero_loss_and_opposite_has_two():
    rng = np.random.default_rng(5)
    npw, nb, nshell = 30, 2, 4
    xc, o = _orthonormal_split(rng, npw, nb)
    k0 = rng.uniform(0.2, 1.0, (nb, npw))
    shell = np.sort(rng.integers(0, nshell, npw))
    x = om.features(np.arange(nshell, dtype=float), np.ones(nb), 0.3, 10.0)
    theta = _zero_output(synth.mlp_init(3))
    for sign, want in ((1.0, 0.0), (-1.0, 2.0)):
        g = sign * 2.5 * o / k0                          # K0 g = +-2.5 e
        a, b, e = om.harvest_tables(o, xc, g, k0, shell, nshell)
        assert om.loss(theta, x[None], a[None], b[None], e[None]) == pytest.approx(want, abs=1e-13)


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(6)
    theta = rng.standard_normal(50)
    grad = rng.standard_normal(50)
    new, m, v = om.adam_step(theta, grad, np.zeros(50), np.zeros(50), 1, 0.01)
    # bias-corrected m / sqrt(v) is g / |g| on the first step (eps = 1e-8 aside)
    assert np.all(np.abs(new - (theta - 0.01 * np.sign(grad))) <= 0.01 * 1e-8 / np.abs(grad) + 1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad ** 2)
