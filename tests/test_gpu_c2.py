"""The 128^3 workload at full size on the GPU (Sec. IV-A setup): 4 x 4 x 4
subdomains of 32^3 cells with overlap 1, eps_r U[1,10] on 8^3-cell cubes
(seed 2), c = 2, right-hand side N(0,1), BiCGSTAB in FP64 to 1e-8.

* One FP64 preconditioner apply: six sampled subdomains (corner, edge, face
  and interior boxes) against the oracle's per-subdomain solve, 1e-12 in the
  max norm of each owned block (the bound of the smaller parity cases).
* The stencil at sampled slots against the oracle's windowed operator.
* The solve against the oracle's own BiCGSTAB solve of the same problem,
  stored in tests/golden/c2_oracle.json by tests/golden/make_c2_golden.py:
  iterations within 2; both true residuals <= 1e-8 ||b||, so the solutions
  differ by at most ||A^-1|| (1e-8 + 1e-8) ||b||_2 with ||A^-1||_2 <=
  sqrt(eps_max / eps_min) = sqrt(10) (A is similar to an SPD matrix with
  eigenvalues >= 1 through diag(eps_e)^(1/2)); checked at the 512 stored slots.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import ras, yee
from paper_2508_07193_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.json")


@pytest.fixture(scope="module")
def c2():
    P = inputs.make_problem("c2")
    n = P["nx"]
    h = api.Handle([dict(nx=n, ny=n, nz=n, c=P["c"], eps=P["eps"], eps_block=P["eps_block"],
                         sub=P["sub"])], overlap=1, precision="fp64", device=DEV)
    b = torch.from_numpy(P["rhs"].ravel()).to(DEV)
    eps_cell = yee.expand_eps(P["eps"], P["eps_block"], n, n, n)
    yield P, h, b, eps_cell
    h.close()


def test_c2_sampled_precond_and_stencil(c2):
    P, h, b, eps_cell = c2
    n = P["nx"]
    z, y = h.new_vector(), h.new_vector()
    h.apply_precond(b, z)
    h.curlcurl_apply(b, y)
    torch.cuda.synchronize()
    zo = z.cpu().numpy().reshape(P["rhs"].shape)
    yo = y.cpu().numpy().reshape(P["rhs"].shape)
    which = [0, 3, 5, 21, 42, 63]            # corner, edge, face, interior, interior, corner
    blocks = ras.ras_apply_subset(P["rhs"], P["c"], P["sub"], 1, eps_cell, which)
    for idx, (own, blk) in blocks.items():
        (x0, x1), (y0, y1), (z0, z1) = own
        got = zo[:, z0:z1, y0:y1, x0:x1]
        err = np.abs(got - blk).max() / np.abs(blk).max()
        assert err < 1e-12, (idx, err)
    rng = np.random.default_rng(12)
    mask = inputs.unknown_slots(n, n, n)
    pts = np.argwhere(mask)
    pts = pts[rng.choice(len(pts), 150, replace=False)]
    edge = [(q, k, j, i) for q in range(3) for (k, j, i) in
            ((1, 1, 1), (n - 1, n - 1, n - 1), (1, 64, 0), (64, 1, 127), (127, 64, 64))
            if mask[q, k, j, i]]
    pts = [tuple(int(v) for v in p) for p in pts] + edge
    want = yee.apply_A_at(P["rhs"], P["c"], eps_cell, pts)
    got = np.array([yo[p] for p in pts])
    assert np.abs(got - want).max() <= 1e-13 * np.abs(P["rhs"]).max()


def test_c2_bicgstab_matches_oracle_solve(c2):
    P, h, b, _ = c2
    with open(GOLDEN) as f:
        G = json.load(f)
    x = h.new_vector()
    info = h.solve(b, x, solver="bicgstab", rtol=P["tol"], max_iter=500)
    assert info["status"] == "FMP_OK" and info["rel_residual_true"] <= P["tol"], info
    assert abs(info["iterations"] - G["iterations"]) <= 2, (info["iterations"], G["iterations"])
    idx = torch.tensor(G["sample_index"], device=DEV)
    got = x[idx].cpu().numpy()
    want = np.array(G["sample_value"])
    bnorm = float(np.linalg.norm(P["rhs"]))
    bound = np.sqrt(10.0) * 2.0 * P["tol"] * bnorm
    assert np.abs(got - want).max() <= bound, (np.abs(got - want).max(), bound)
    xn = float(torch.linalg.vector_norm(x))
    assert abs(xn - G["x_norm2"]) <= bound
    # Table III: two preconditioner and two operator applies per iteration, plus
    # the initial residual and the true residual recomputed at convergence
    assert info["n_precond"] == 2 * info["iterations"]
    assert info["n_spmv"] == 2 * info["iterations"] + 2
