"""The 64-domain batch at full size on the GPU: 64 cubic domains with sides
drawn from {24, 32, 48, 64, 96} (seed 4), c ~ U[0.5, 8], eps = 1, each split
into ceil(L / 32) equal owned blocks per axis, all in one handle (61.1 M
unknowns, concatenated vectors).

* One preconditioner apply on the whole batch in FP64: in sampled domains
  (every side that occurs, first and last domain) two subdomains each, a
  corner box and the last box, against the oracle's per-subdomain solve of
  that domain, 1e-12 in the max norm of each owned block (the bound of the
  smaller parity cases).  Sampling keeps the oracle to seconds.
* The same apply in FP32 (the batch's transform precision) against the same
  blocks, per box, within 12 u of the box's restricted input (the bound of
  the reduced-precision parity tests: six contraction stages of at most 2u
  each; the transforms are orthogonal and the 3x3 solve is a contraction).
* Independent FGMRES(30) per domain in FP64 to 1e-8: every domain meets the
  tolerance on its own right-hand side, checked with the library's stencil.
"""
import numpy as np
import pytest
import torch

from oracle import ras, yee
from paper_2508_07193_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def batch():
    doms = inputs.make_batch_c4()
    b = torch.cat([torch.from_numpy(d["rhs"].ravel()) for d in doms]).to(DEV)
    return doms, b


def _sample(doms):
    """Domain indices: first and last, and the first domain of every side."""
    pick = {0, len(doms) - 1}
    seen = set()
    for i, d in enumerate(doms):
        if d["nx"] not in seen:
            seen.add(d["nx"])
            pick.add(i)
    return sorted(pick)


def _apply(doms, b, precision):
    h = api.Handle([dict(nx=d["nx"], ny=d["ny"], nz=d["nz"], c=d["c"], sub=d["sub"]) for d in doms],
                   overlap=1, precision=precision, device=DEV)
    z = h.new_vector()
    h.apply_precond(b, z)
    torch.cuda.synchronize()
    out = z.cpu().numpy()
    offs = list(h.offsets)
    h.close()
    return out, offs


def _blocks(d):
    n = d["nx"]
    nsub = (n // d["sub"][0]) ** 3
    return ras.ras_apply_subset(d["rhs"], d["c"], d["sub"], 1, None, [0, nsub - 1])


def test_c4_batch_fp64_sampled_blocks(batch):
    doms, b = batch
    out, offs = _apply(doms, b, "fp64")
    for i in _sample(doms):
        d = doms[i]
        zd = out[offs[i]:offs[i + 1]].reshape(d["rhs"].shape)
        for idx, (own, blk) in _blocks(d).items():
            (x0, x1), (y0, y1), (z0, z1) = own
            err = np.abs(zd[:, z0:z1, y0:y1, x0:x1] - blk).max() / np.abs(blk).max()
            assert err < 1e-12, (i, d["nx"], idx, err)
        assert not np.any(zd[~inputs.unknown_slots(d["nx"], d["ny"], d["nz"])])


def test_c4_batch_fp32_sampled_blocks_within_bound(batch):
    doms, b = batch
    out, offs = _apply(doms, b, "fp32")
    u = 2.0**-24
    worst = 0.0
    for i in _sample(doms):
        d = doms[i]
        zd = out[offs[i]:offs[i + 1]].reshape(d["rhs"].shape)
        subs = ras.subdomains(d["nx"], d["ny"], d["nz"], d["sub"], 1)
        for idx, (own, blk) in _blocks(d).items():
            (x0, x1), (y0, y1), (z0, z1) = own
            (bx0, bx1), (by0, by1), (bz0, bz1) = subs[idx]["box"]
            rin = np.linalg.norm(yee.from_padded(d["rhs"][:, bz0:bz1, by0:by1, bx0:bx1]))
            e = np.linalg.norm((zd[:, z0:z1, y0:y1, x0:x1] - blk).ravel()) / rin
            worst = max(worst, e)
            assert e < 12 * u, (i, d["nx"], idx, e)
    print(f"fp32 batch: worst sampled box error {worst / u:.1f} u (bound 12 u)")


def test_c4_per_domain_fgmres_meets_tolerance(batch):
    doms, b = batch
    h = api.Handle([dict(nx=d["nx"], ny=d["ny"], nz=d["nz"], c=d["c"], sub=d["sub"]) for d in doms],
                   overlap=1, precision="fp32", device=DEV)
    x, y = h.new_vector(), h.new_vector()
    info = h.solve(b, x, solver="fgmres", rtol=1e-8, max_iter=200, per_domain=True)
    assert info["status"] == "FMP_OK"
    h.curlcurl_apply(x, y)
    for d in range(len(doms)):
        a, e = h.offsets[d], h.offsets[d + 1]
        rel = float(torch.linalg.vector_norm(b[a:e] - y[a:e]) / torch.linalg.vector_norm(b[a:e]))
        assert rel <= 1e-8 * (1 + 1e-6), (d, rel)
        assert info["domain_rel_residual"][d] <= 1e-8
    h.close()
