"""Learned coarse correction, FP64 reference (oracle; test infrastructure).

The correction added to the RAS preconditioner (Sec. II-B) is

    z = M_RAS^{-1} r + P0( ||R0 r|| * MLP(R0 r / ||R0 r||) )

R0 averages r over the unknowns each subdomain owns, per component, giving a
coarse vector laid out [3][nsub] (subdomains in C order z, y, x); P0 injects a
coarse vector as a constant per subdomain and component on the owned unknowns.
The MLP is in -> hidden (ReLU) -> hidden (ReLU) -> in.  Its training target
for a residual r with error e = A^{-1} r is R0(e - M_RAS^{-1} r), in the same
normalisation.  This part is not in the paper; the shapes follow the workload
description (3 x 8^3 inputs, two hidden layers of 256).

Parameters are one flat vector in the order W1[h][in], b1[h], W2[h][h],
b2[h], W3[in][h], b3[in].  The loss is the mean of squared errors over all
batch x in entries.
"""
import numpy as np

from . import ras, yee


def _owned_slices(nx, ny, nz, sub):
    out = []
    for s in ras.subdomains(nx, ny, nz, sub, 1):
        (x0, x1), (y0, y1), (z0, z1) = s["own"]
        out.append((slice(z0, z1), slice(y0, y1), slice(x0, x1)))
    return out


def restrict(r_pad, sub):
    """R0: mean of r over the owned unknowns of each subdomain, per component."""
    _, nz, ny, nx = r_pad.shape
    mask = yee.wall_mask(nx, ny, nz)
    sl = _owned_slices(nx, ny, nz, sub)
    out = np.zeros((3, len(sl)))
    for s, (a, b, c) in enumerate(sl):
        for q in range(3):
            m = mask[q, a, b, c]
            out[q, s] = r_pad[q, a, b, c][m].mean() if m.any() else 0.0
    return out.ravel()


def prolong(yc, shape, sub):
    """P0: constant per subdomain and component on the owned unknowns."""
    _, nz, ny, nx = shape
    mask = yee.wall_mask(nx, ny, nz)
    sl = _owned_slices(nx, ny, nz, sub)
    y = np.asarray(yc).reshape(3, len(sl))
    z = np.zeros(shape)
    for s, (a, b, c) in enumerate(sl):
        for q in range(3):
            z[q, a, b, c] = y[q, s]
    return np.where(mask, z, 0.0)


def unpack(params, n_in, hidden):
    p = np.asarray(params, dtype=np.float64)
    sizes = [hidden * n_in, hidden, hidden * hidden, hidden, n_in * hidden, n_in]
    parts, o = [], 0
    for sz in sizes:
        parts.append(p[o:o + sz])
        o += sz
    W1, b1, W2, b2, W3, b3 = parts
    return (W1.reshape(hidden, n_in), b1, W2.reshape(hidden, hidden), b2,
            W3.reshape(n_in, hidden), b3)


def n_params(n_in, hidden):
    return 2 * n_in * hidden + hidden * hidden + 2 * hidden + n_in


def forward(params, X, n_in, hidden):
    """Rows of X are inputs; returns (output, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, hidden)
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    O = H2 @ W3.T + b3
    return O, (X, Z1, H1, Z2, H2)


def loss_grad(params, X, Y, n_in, hidden):
    """Mean squared error and its gradient, by the chain rule written out."""
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, hidden)
    O, (X, Z1, H1, Z2, H2) = forward(params, X, n_in, hidden)
    D = O - Y
    loss = float(np.mean(D * D))
    dO = 2.0 * D / D.size
    gW3 = dO.T @ H2
    gb3 = dO.sum(0)
    dZ2 = (dO @ W3) * (Z2 > 0)
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round FP32 values to bf16 (nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def correction(r_pad, sub, params, n_in, hidden):
    """P0(||R0 r|| MLP(R0 r / ||R0 r||)) in FP64 with the given weights."""
    rc = restrict(r_pad, sub)
    nrm = np.linalg.norm(rc)
    if nrm == 0.0:
        return np.zeros_like(r_pad)
    O, _ = forward(params, (rc / nrm)[None, :], n_in, hidden)
    return prolong(nrm * O[0], r_pad.shape, sub)
