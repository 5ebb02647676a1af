"""Training and evaluation of the learned coarse correction.

Pairs come from the solver itself: for each right-hand side b, FGMRES with the
plain FlashMP preconditioner gives a tight solution x* and its first iterates
x_k (captured by fmp_solve).  With r_k = b - A x_k and e_k = x* - x_k, a pair
is (R0 r_k, R0(e_k - M_RAS r_k)), both divided by ||R0 r_k||.  Because R0 and
M_RAS are linear, every large-vector operation is one library call
(fmp_curlcurl_apply, fmp_apply_precond, fmp_coarse_restrict) and only coarse
vectors (3 x subdomains entries) are combined on the host.

Training runs the library's MLP kernels (bf16 MFMA forward and backward with
FP32 accumulation, FP32 master weights, Adam).
"""
import time

import numpy as np
import torch

from . import api, inputs


def init_params(n_in, hidden, seed=0, out_scale=1e-2):
    """He-uniform hidden layers, a small output layer (the correction starts near 0)."""
    rng = np.random.default_rng(seed)
    lim1, lim2, lim3 = np.sqrt(6.0 / n_in), np.sqrt(6.0 / hidden), out_scale * np.sqrt(6.0 / hidden)
    parts = [rng.uniform(-lim1, lim1, hidden * n_in), np.zeros(hidden),
             rng.uniform(-lim2, lim2, hidden * hidden), np.zeros(hidden),
             rng.uniform(-lim3, lim3, n_in * hidden), np.zeros(n_in)]
    return np.concatenate(parts).astype(np.float32)


def _restrict(h, v, n_in):
    rc = torch.zeros(n_in, dtype=torch.float64, device=h.device)
    api.fmp_coarse_restrict(h, v, rc)
    return rc


def generate_pairs(h, dims, n_rhs, per_rhs, seed0, rtol_star=1e-11, log=None):
    """Return (X, Y) float32 numpy arrays of n_rhs * per_rhs normalised pairs."""
    nx, ny, nz = dims
    n_in = api.fmp_coarse_size(h)
    api.fmp_set_coarse_model(h, 0, None)          # pairs use the plain preconditioner
    dev = h.device
    cap = torch.zeros(per_rhs, h.length, dtype=torch.float64, device=dev)
    xs = h.new_vector()
    y = h.new_vector()
    my = h.new_vector()
    mb = h.new_vector()
    X = np.zeros((n_rhs * per_rhs, n_in), np.float32)
    Y = np.zeros_like(X)
    row = 0
    t0 = time.perf_counter()
    for s in range(n_rhs):
        b = inputs.extra_rhs_device(nx, ny, nz, seed0 + s, dev)
        xs.zero_()
        h.solve(b, xs, solver="fgmres", rtol=rtol_star, max_iter=400)
        x = h.new_vector()
        h.solve(b, x, solver="fgmres", rtol=1e-300, max_iter=per_rhs, capture=cap)
        h.apply_precond(b, mb)
        Rb, Rxs, Rmb = (_restrict(h, v, n_in).cpu().numpy() for v in (b, xs, mb))
        for k in range(per_rhs):
            h.curlcurl_apply(cap[k], y)
            h.apply_precond(y, my)
            Rx, Ry, Rmy = (_restrict(h, v, n_in).cpu().numpy() for v in (cap[k], y, my))
            rc = Rb - Ry                               # R0 r_k
            tc = (Rxs - Rx) - (Rmb - Rmy)              # R0 (e_k - M r_k)
            nrm = np.linalg.norm(rc)
            X[row] = rc / nrm
            Y[row] = tc / nrm
            row += 1
        if log and (s + 1) % max(1, n_rhs // 10) == 0:
            log(f"pairs: {s + 1}/{n_rhs} right-hand sides, {time.perf_counter() - t0:.1f} s")
    return X, Y


def train(X, Y, hidden=256, epochs=200, batch=100, lr=1e-3, seed=0, device="cuda", log=None):
    """Adam on the MSE with the library's kernels; returns (params float32, loss history)."""
    n, n_in = X.shape
    rng = np.random.default_rng(seed)
    params = torch.from_numpy(init_params(n_in, hidden, seed)).to(device)
    grads = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    scratch = torch.empty(api.fmp_mlp_scratch_bytes(n_in, hidden, batch), dtype=torch.uint8,
                          device=device)
    hist = []
    t = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        Xd = torch.from_numpy(X[perm]).to(device)
        Yd = torch.from_numpy(Y[perm]).to(device)
        tot = 0.0
        nb = 0
        for i in range(0, n - batch + 1, batch):
            api.fmp_mlp_loss_grad(n_in, hidden, batch, params, Xd[i:i + batch], Yd[i:i + batch],
                                  grads, loss, scratch)
            t += 1
            api.fmp_mlp_adam(params, grads, m, v, t, lr)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        if log and (ep + 1) % max(1, epochs // 10) == 0:
            log(f"epoch {ep + 1}: mse {hist[-1]:.4e}")
    return params.cpu().numpy(), hist
