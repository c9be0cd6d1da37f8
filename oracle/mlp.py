"""The per-shell preconditioner network and its training loss (oracle, FP64).

Not in the paper: a learned stand-in for the diagonal preconditioner of the
folded PCG (the paper's diagonal preconditioner is M(G), Sec. II.B).  Written
from the definition below, in plain numpy FP64.

Network (3 -> 64 -> 64 -> 1, tanh), per |G+k| shell s and band i:
    x      = (T_s / Ecut, T_i / Ecut, E_ref / Ecut)
    h1     = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  r = W3 h2 + b3
    f_si   = 8 tanh(r / 8)                      (smooth clamp to [-8, 8])
Preconditioner: K_i(G) = K0_i(G) exp(f_{s(G), i}) with K0 the base diagonal
preconditioner (the library uses the paper's M(G); any K0 > 0 works here).

Loss (one snapshot): for band i with gradient g_i and error
e_i = (I - Psi* Psi*^H) psi_i (the part of psi_i outside the converged subspace;
the CG steps along -z_i, so the ideal preconditioned gradient points along e_i),
z_i = K_i o g_i and
    L_i = 1 - Re<z_i, e_i> / (||z_i|| ||e_i||).
With shell sums A_si = sum_{G in s} Re(conj(e_i) K0_i g_i), B_si = sum_{G in s}
|K0_i g_i|^2, E_i = ||e_i||^2 and w_si = exp(f_si):
    L_i = 1 - (sum_s w_si A_si) / (sqrt(sum_s w_si^2 B_si) sqrt(E_i)).
The training loss is the mean of L_i over bands and snapshots.

Weighted variant (used for training): the inner products and norms above are
taken in the metric diag(w_G), w_G = (T_G - E_ref)^2 + delta^2, the plane-wave
diagonal of (H - E_ref)^2 without the potential (an approximate A-norm).  w is
constant on a shell, so A_si, B_si and the shell parts of E_i are multiplied by
w_s and the loss formula is unchanged.

Parameter vector layout (4481 values): W1[64][3], b1[64], W2[64][64], b2[64],
W3[64], b3.
"""
from __future__ import annotations

import numpy as np

H = 64
NPARAM = H * 3 + H + H * H + H + H + 1


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    w1 = theta[o:o + 3 * H].reshape(H, 3); o += 3 * H
    b1 = theta[o:o + H]; o += H
    w2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return w1, b1, w2, b2, w3, b3


def init_params(seed=0):
    """Glorot-uniform weights, zero biases, last layer scaled by 0.1 (network
    starts close to f = 0, i.e. the base preconditioner K0)."""
    rng = np.random.default_rng([5, seed])
    def glorot(o, i):
        lim = np.sqrt(6.0 / (o + i))
        return rng.uniform(-lim, lim, size=(o, i))
    theta = np.concatenate([glorot(H, 3).ravel(), np.zeros(H), glorot(H, H).ravel(), np.zeros(H),
                            0.1 * glorot(1, H).ravel(), np.zeros(1)])
    assert theta.size == NPARAM
    return theta


def features(shell_t, tband, e_ref, ecut):
    """[nshell, nb, 3] inputs for every (shell, band)."""
    ns, nb = len(shell_t), len(tband)
    x = np.empty((ns, nb, 3))
    x[:, :, 0] = np.asarray(shell_t)[:, None] / ecut
    x[:, :, 1] = np.asarray(tband)[None, :] / ecut
    x[:, :, 2] = e_ref / ecut
    return x


def forward(theta, x):
    """f for inputs x[..., 3]; returns (f, cache)."""
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    h1 = np.tanh(x @ w1.T + b1)
    h2 = np.tanh(h1 @ w2.T + b2)
    r = h2 @ w3 + b3
    t = np.tanh(r / 8.0)
    return 8.0 * t, (x, h1, h2, t)


def loss(theta, xs, a, b, e):
    """Mean band loss over snapshots.  xs [K][ns][nb][3], a, b [K][ns][nb], e [K][nb]."""
    f, _ = forward(theta, xs)
    w = np.exp(f)
    u = np.sum(w * a, axis=1)                  # [K][nb]
    q = np.sum(w * w * b, axis=1)
    return float(np.mean(1.0 - u / (np.sqrt(q) * np.sqrt(e))))


def loss_grad(theta, xs, a, b, e):
    """(loss, dloss/dtheta) by the chain rule written out."""
    f, (x, h1, h2, t) = forward(theta, xs)
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    w = np.exp(f)
    u = np.sum(w * a, axis=1)
    q = np.sum(w * w * b, axis=1)
    n = np.sqrt(q)
    se = np.sqrt(e)
    nk = u.size                                # snapshots x bands
    l = float(np.mean(1.0 - u / (n * se)))
    # dL/dw_s = -A_s/(n sqrt E) + u w_s B_s/(n^3 sqrt E), all divided by nk
    dldw = (-a / (n * se)[:, None, :] + (u / (n ** 3 * se))[:, None, :] * w * b) / nk
    dldf = dldw * w
    dldr = (dldf * (1.0 - t * t)).reshape(-1)  # f = 8 tanh(r/8); samples flattened
    x, h1, h2 = x.reshape(-1, 3), h1.reshape(-1, H), h2.reshape(-1, H)
    g_w3 = dldr @ h2
    g_b3 = np.sum(dldr)
    d2 = dldr[:, None] * w3[None, :] * (1.0 - h2 * h2)
    g_w2 = d2.T @ h1
    g_b2 = np.sum(d2, axis=0)
    d1 = (d2 @ w2) * (1.0 - h1 * h1)
    g_w1 = d1.T @ x
    g_b1 = np.sum(d1, axis=0)
    grad = np.concatenate([g_w1.ravel(), g_b1, g_w2.ravel(), g_b2, g_w3, [g_b3]])
    return l, grad


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); step counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def harvest_tables(x_snap, x_conv, g, k0, shell, nshell, weight=None):
    """Shell tables of one snapshot.

    x_snap [nb][npw] current bands, x_conv [nb][npw] converged orthonormal block,
    g [nb][npw] gradients, k0 [nb][npw] base preconditioner weights, shell [npw],
    weight [nshell] optional metric weight per shell (w_s above).
    Returns A [nshell][nb], B [nshell][nb], E [nb]."""
    coef = x_snap @ x_conv.conj().T            # [i][j] = <x_conv_j | x_i>
    e = x_snap - coef @ x_conv                 # (I - P*) x_i
    kg = k0 * g
    nb = x_snap.shape[0]
    a = np.zeros((nshell, nb))
    b = np.zeros((nshell, nb))
    ra = np.real(np.conj(e) * kg)
    rb = np.abs(kg) ** 2
    wg = np.ones(len(shell)) if weight is None else np.asarray(weight)[shell]
    for i in range(nb):
        a[:, i] = np.bincount(shell, weights=wg * ra[i], minlength=nshell)
        b[:, i] = np.bincount(shell, weights=wg * rb[i], minlength=nshell)
    return a, b, np.sum(wg[None, :] * np.abs(e) ** 2, axis=1)
