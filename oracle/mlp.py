"""Reference for the learned per-element preconditioner (an addition to the
paper's method: the paper's preconditioners are BJ_ext / BJ^H_ext, Sec. 3.2.3).

The network approximates, element by element, the action of the inverse of
the Schur complement of the extended Jacobian (Eq. nonlinear_eqsys_Schur):
given a Krylov vector v = (v_w, v_sigma),

    r~  = v_w - bcoef R1'(w) v_sigma                     (Schur right-hand side)
    dw_e = s_e N(f_e / s_e ... )                          (per element, below)
    dsigma = v_sigma + R1'(w) dw                          (second block row)

Features of element e (2-D: self + 4 face neighbours; 3-D: self + 6):
    [r~ tiles of the patch / s_e,  w tiles of the patch,  a1dt, bcoef]
with s_e = RMS of the r~ patch (+1e-30), tile order (self, -x, +x, -y, +y,
-z, +z), each tile in the w[e][v][node] layout.  Output: dw_e / s_e.

MLP: n_in -> H -> H -> n_out, ReLU on the hidden layers, weights W[i][j]
from input i to output j, loss = mean over batch and outputs of (y - t)^2.
Adam (Kingma & Ba) with bias correction.  All FP64.

Parameter vector layout (shared with the library's ABI): W1 (n_in x H),
b1 (H), W2 (H x H), b2 (H), W3 (H x n_out), b3 (n_out), row-major.

Parity unpinned: the trained weights and the iteration savings have no
external reference; the forward/backward arithmetic is pinned by central
finite differences (tests/test_oracle_mlp.py).
"""
import numpy as np


def n_params(n_in, H, n_out):
    return n_in * H + H + H * H + H + H * n_out + n_out


def unpack(theta, n_in, H, n_out):
    o = 0
    out = []
    for shape in ((n_in, H), (H,), (H, H), (H,), (H, n_out), (n_out,)):
        k = int(np.prod(shape))
        out.append(theta[o:o + k].reshape(shape))
        o += k
    return out


def pack(parts):
    return np.concatenate([p.ravel() for p in parts])


def forward(theta, X, n_in, H, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, T, n_in, H, n_out):
    """MSE loss and its gradient with respect to theta (manual backward)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    y, (X, z1, h1, z2, h2) = forward(theta, X, n_in, H, n_out)
    B = X.shape[0]
    diff = y - T
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / (B * n_out)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0.0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0.0)
    dW1 = X.T @ dz1
    db1 = dz1.sum(axis=0)
    return loss, pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(n_in, H, n_out, rng):
    """He-uniform weights, zero biases (the caller passes the generator)."""
    parts = []
    for fi, fo in ((n_in, H), (H, H), (H, n_out)):
        lim = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, size=(fi, fo)))
        parts.append(np.zeros(fo))
    return pack(parts)


# ------------------------------------------------------------------ features
def neighbours(nelem, e):
    """Face neighbours of element e in the order -x, +x, -y, +y, -z, +z."""
    d = len(nelem)
    c = []
    r = e
    for m in range(d):
        c.append(r % nelem[m])
        r //= nelem[m]
    out = []
    for m in range(d):
        for s in (-1, 1):
            cc = list(c)
            cc[m] = (cc[m] + s) % nelem[m]
            g = 0
            mul = 1
            for k in range(d):
                g += cc[k] * mul
                mul *= nelem[k]
            out.append(g)
    return out


def features(nelem, rt, w, a1dt, bcoef, elems):
    """Feature rows and scales for the listed elements.

    rt, w: arrays (nE, ne).  Returns X (len(elems), (2d+1) 2 ne + 2), s."""
    rt = np.asarray(rt).reshape(int(np.prod(nelem)), -1)
    w = np.asarray(w).reshape(rt.shape)
    rows, scales = [], []
    for e in elems:
        patch = [e] + neighbours(nelem, e)
        r = np.concatenate([rt[p] for p in patch])
        s = np.sqrt(np.mean(r * r)) + 1e-30
        x = np.concatenate([r / s] + [w[p] for p in patch] + [np.array([a1dt, bcoef])])
        rows.append(x)
        scales.append(s)
    return np.array(rows), np.array(scales)


def apply_learned(dg, theta, H, w, v_w, v_s, a1dt, bcoef):
    """Learned preconditioner P^-1 (v_w, v_s) in FP64 (module docstring)."""
    nE = dg.mesh.n_elem
    ne = dg.nvar * dg.nnode
    n_in = (2 * dg.d + 1) * 2 * ne + 2
    rt = v_w - bcoef * dg.r2(w, v_s)
    X, s = features(dg.mesh.nelem, rt, w, a1dt, bcoef, range(nE))
    y, _ = forward(theta, X, n_in, H, ne)
    dw = (y * s[:, None]).reshape(w.shape)
    ds = v_s + dg.r2(w, dw)
    return dw, ds
