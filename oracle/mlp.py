"""Reference for the learned per-element preconditioner (an addition to the
paper's method: the paper's preconditioners are BJ_ext / BJ^H_ext, Sec. 3.2.3).

The preconditioner keeps the structure of BJ_ext, the exact inverse of the
extended Jacobian with R1'(w) replaced by its element-local part K (every
quantity read from a neighbour held constant), and replaces the element
solve S_e^-1, S_e = I - a1dt K_e + bcoef K_e^2, by a network on patch
features: given a Krylov vector v = (v_w, v_sigma),

    r~  = v_w - bcoef K v_sigma                           (element Schur right-hand side)
    dw_e = s_e f(x_e)                                     (per element, below)
    dsigma = v_sigma + K dw                               (second block row)

Features of element e (2-D: self + 4 face neighbours; 3-D: self + 6):
    x_e = [x_r | x_w],  x_r = r~ tiles of the patch / s_e,
                        x_w = [w tiles of the patch, ln a1dt, ln bcoef]
with s_e = RMS of the r~ patch (+1e-30), tile order (self, -x, +x, -y, +y,
-z, +z), each tile in the w[e][v][node] layout.  Output: dw_e / s_e.

Network f (two hidden layers of width H): the state path is a ReLU MLP whose
activations gate the residual path, which is linear,
    g1 = relu(x_w W1w + b1),      g2 = relu(g1 W2w + b2),
    h1 = (x_r W1r) * g1,          h2 = (h1 W2r) * g2,       f = h2 W3,
so that for a fixed state the preconditioner is a linear map of v (FGMRES
builds its search space from it; a map that is not odd and additive in v
stalls there).  Loss = mean over batch and outputs of (f - t)^2.  Adam
(Kingma & Ba) with bias correction.  All FP64.

Parameter vector layout (shared with the library's ABI), row-major, W[i][j]
from input i to output j: W1r (n_r x H), W1w (n_w x H), b1 (H), W2r (H x H),
W2w (H x H), b2 (H), W3 (H x n_out), with n_r = (n_in - 2) / 2 residual
inputs and n_w = n_r + 2 state inputs.

Parity unpinned: the trained weights and the iteration savings have no
external reference; the forward/backward arithmetic is pinned by central
finite differences, linearity in the residual by superposition, the block
structure (r~ and the back-substitution) by reproducing BJ_ext's four-block
apply when the element solve is the exact S_e^-1, the BF16 rounding by its
tie cases and by torch's own float32 -> bfloat16 conversion
(tests/test_oracle_mlp.py).
"""
import numpy as np


def split(n_in):
    """(n_r, n_w): residual and state inputs of a feature row of length n_in."""
    n_r = (n_in - 2) // 2
    return n_r, n_in - n_r


def n_params(n_in, H, n_out):
    n_r, n_w = split(n_in)
    return n_r * H + n_w * H + H + 2 * H * H + H + H * n_out


def shapes(n_in, H, n_out):
    n_r, n_w = split(n_in)
    return ((n_r, H), (n_w, H), (H,), (H, H), (H, H), (H,), (H, n_out))


NAMES = ("W1r", "W1w", "b1", "W2r", "W2w", "b2", "W3")


def unpack(theta, n_in, H, n_out):
    o = 0
    out = []
    for shape in shapes(n_in, H, n_out):
        k = int(np.prod(shape))
        out.append(theta[o:o + k].reshape(shape))
        o += k
    return out


def pack(parts):
    return np.concatenate([p.ravel() for p in parts])


def round_bf16(x):
    """Nearest bfloat16 value, ties to even, reached through float32: the
    rounding of an operand fed to a BF16 matrix multiply.  bfloat16 keeps the
    sign, the 8 exponent bits and the top 7 fraction bits of a float32, so
    rounding adds half of the dropped 16-bit range (0x7FFF, plus one when the
    lowest kept bit is set, which breaks ties towards even) and truncates.
    Finite inputs only."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return x


def forward(theta, X, n_in, H, n_out, q=None):
    """Network output for feature rows X.  q (optional) rounds every operand
    of the matrix products, e.g. round_bf16 to model BF16 operands with exact
    accumulation; biases, ReLU and the gating act on unrounded values."""
    q = q or _ident
    n_r, _ = split(n_in)
    W1r, W1w, b1, W2r, W2w, b2, W3 = unpack(theta, n_in, H, n_out)
    Xr, Xw = X[:, :n_r], X[:, n_r:]
    z1 = q(Xw) @ q(W1w) + b1
    g1 = np.maximum(z1, 0.0)
    z2 = q(g1) @ q(W2w) + b2
    g2 = np.maximum(z2, 0.0)
    a1 = q(Xr) @ q(W1r)
    h1 = a1 * g1
    a2 = q(h1) @ q(W2r)
    h2 = a2 * g2
    y = q(h2) @ q(W3)
    return y, (Xr, Xw, g1, g2, a1, h1, a2, h2)


def loss_and_grad(theta, X, T, n_in, H, n_out, q=None):
    """MSE loss and its gradient with respect to theta (manual backward).
    q as in forward, applied to both operands of every matrix product of the
    forward and the backward pass (bias gradients are plain column sums)."""
    q = q or _ident
    W1r, W1w, b1, W2r, W2w, b2, W3 = unpack(theta, n_in, H, n_out)
    y, (Xr, Xw, g1, g2, a1, h1, a2, h2) = forward(theta, X, n_in, H, n_out, q)
    B = X.shape[0]
    diff = y - T
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / (B * n_out)
    dW3 = q(h2).T @ q(dy)
    dh2 = q(dy) @ q(W3).T
    da2 = dh2 * g2
    dz2 = dh2 * a2 * (g2 > 0.0)
    dW2r = q(h1).T @ q(da2)
    dh1 = q(da2) @ q(W2r).T
    da1 = dh1 * g1
    dW1r = q(Xr).T @ q(da1)
    dW2w = q(g1).T @ q(dz2)
    db2 = dz2.sum(axis=0)
    dg1 = dh1 * a1 + q(dz2) @ q(W2w).T
    dz1 = dg1 * (g1 > 0.0)
    dW1w = q(Xw).T @ q(dz1)
    db1 = dz1.sum(axis=0)
    return loss, pack([dW1r, dW1w, db1, dW2r, dW2w, db2, dW3])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(n_in, H, n_out, rng):
    """Uniform weights with variance 2/fan_in on the ReLU state path and
    1/fan_in on the linear residual path, zero biases (the caller passes the
    generator)."""
    n_r, n_w = split(n_in)
    parts = []
    for shape in shapes(n_in, H, n_out):
        if len(shape) == 1:
            parts.append(np.zeros(shape))
            continue
        gain = 6.0 if len(parts) in (1, 4) else 3.0   # W1w, W2w feed a ReLU
        lim = np.sqrt(gain / shape[0])
        parts.append(rng.uniform(-lim, lim, size=shape))
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
        x = np.concatenate([r / s] + [w[p] for p in patch] + [np.log([a1dt, bcoef])])
        rows.append(x)
        scales.append(s)
    return np.array(rows), np.array(scales)


def schur_apply(dg, w, v_w, v_s, bcoef, element_solve):
    """The preconditioner's block structure (module docstring) with a given
    element solve: r~ = v_w - bcoef K v_s, dw = element_solve(r~),
    ds = v_s + K dw, K v the element-local linearisation
    dg.r2(w, v, local=True).  With element_solve = S_e^-1 for every element
    this is BJ_ext (Sec. 3.2.3) exactly, because S_e is a polynomial in K_e
    and commutes with it."""
    rt = v_w - bcoef * dg.r2(w, v_s, local=True)
    dw = np.asarray(element_solve(rt)).reshape(w.shape)
    ds = v_s + dg.r2(w, dw, local=True)
    return dw, ds


def network_solve(dg, theta, H, w, a1dt, bcoef):
    """Element solve of the learned preconditioner: dw_e = s_e f(x_e) for every
    element, x_e the patch features of r~ and w."""
    nE = dg.mesh.n_elem
    ne = dg.nvar * dg.nnode
    n_in = (2 * dg.d + 1) * 2 * ne + 2

    def solve(rt):
        X, s = features(dg.mesh.nelem, rt, w, a1dt, bcoef, range(nE))
        y, _ = forward(theta, X, n_in, H, ne)
        return y * s[:, None]
    return solve


def apply_learned(dg, theta, H, w, v_w, v_s, a1dt, bcoef):
    """Learned preconditioner P^-1 (v_w, v_s) in FP64 (module docstring)."""
    return schur_apply(dg, w, v_w, v_s, bcoef, network_solve(dg, theta, H, w, a1dt, bcoef))
