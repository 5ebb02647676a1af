"""Restricted additive Schwarz preconditioner from exact box solves (oracle).

What this follows
-----------------
Sec. II-B (Domain Decomposition): M_RAS^{-1} = sum_i S_i^{0T} A_i^{-1} S_i^gamma,
with S_i^gamma the restriction to subdomain i extended by an overlap of gamma
cells, A_i the subdomain operator and S_i^0 the restriction without overlap.
Sec. III-A supplies the exact solve of A_i.

Readings (the paper leaves these open)
--------------------------------------
* A subdomain owns a block of `sub` cells per axis; its box extends the block
  by `overlap` cells on each side, clipped at the global PEC walls.  The box
  unknowns are the unknowns strictly inside the box (tangential E on the box
  faces is held at zero), i.e. S_i^gamma A S_i^gammaT when eps is constant.
* A_i = I + alpha_i K_box with alpha_i = c / (mean eps over the owned cells).
* Ownership for S_i^0: a half-point index i belongs to the block whose cell
  range contains cell i; a node index j belongs to the block whose cell range
  contains cell j (so the node at a block's low face belongs to that block).
"""
import numpy as np

from . import transforms, yee


def axis_parts(n, sub, overlap):
    """[(own_lo, own_hi, box_lo, box_hi)] along one axis."""
    if sub <= 0:
        sub = n
    if n % sub:
        raise ValueError("domain side must be a multiple of the subdomain side")
    return [(a, a + sub, max(0, a - overlap), min(n, a + sub + overlap))
            for a in range(0, n, sub)]


def subdomains(nx, ny, nz, sub, overlap):
    """List of subdomains in (z, y, x) C order, each a dict of owned and box ranges."""
    out = []
    for pz in axis_parts(nz, sub[2], overlap):
        for py in axis_parts(ny, sub[1], overlap):
            for px in axis_parts(nx, sub[0], overlap):
                out.append(dict(own=(px[:2], py[:2], pz[:2]), box=(px[2:], py[2:], pz[2:])))
    return out


def subdomain_alpha(c, eps_cell, own):
    (x0, x1), (y0, y1), (z0, z1) = own
    if eps_cell is None:
        return float(c)
    return float(c) / float(np.mean(eps_cell[z0:z1, y0:y1, x0:x1]))


def ras_apply(r_pad, c, sub, overlap=1, eps_cell=None, solver="transform"):
    """z = M_RAS^{-1} r on padded (3, nz, ny, nx) arrays.

    `sub` = (sx, sy, sz) owned block sides (0 = the whole axis).  Each box is
    solved exactly with the transform solve (or dense LU for tiny boxes).
    """
    _, nz, ny, nx = r_pad.shape
    z = np.zeros_like(r_pad, dtype=np.float64)
    solve = transforms.box_solve_transform if solver == "transform" else transforms.box_solve_lu
    for s in subdomains(nx, ny, nz, sub, overlap):
        (ox0, ox1), (oy0, oy1), (oz0, oz1) = s["own"]
        (bx0, bx1), (by0, by1), (bz0, bz1) = s["box"]
        alpha = subdomain_alpha(c, eps_cell, s["own"])
        box = np.array(r_pad[:, bz0:bz1, by0:by1, bx0:bx1], dtype=np.float64)
        u = yee.from_padded(box)                      # S_i^gamma: drops the box-wall slots
        e = solve(u, bx1 - bx0, by1 - by0, bz1 - bz0, alpha)
        ebox = yee.to_padded(e, bx1 - bx0, by1 - by0, bz1 - bz0)
        z[:, oz0:oz1, oy0:oy1, ox0:ox1] = ebox[:, oz0 - bz0:oz1 - bz0,
                                               oy0 - by0:oy1 - by0, ox0 - bx0:ox1 - bx0]
    return z


def unknown_coords(nx, ny, nz):
    """(component, i, j, k) of every compact unknown, in compact order."""
    out = []
    for q, shp in enumerate(yee.component_shapes(nx, ny, nz)):
        z, y, x = np.meshgrid(*[np.arange(m) for m in shp], indexing="ij")
        # shift the node axes: node index = array index + 1
        i = x + (0 if q == 0 else 1)
        j = y + (0 if q == 1 else 1)
        k = z + (0 if q == 2 else 1)
        out.append(np.stack([np.full(x.size, q), i.ravel(), j.ravel(), k.ravel()], 1))
    return np.concatenate(out)


def ras_apply_matrix(r_pad, c, sub, overlap=1, eps_cell=None):
    """Brute-force RAS straight from the definition, with explicit index sets.

    A_i = I + alpha_i K[box_i, box_i] is solved densely; only tiny problems.
    """
    _, nz, ny, nx = r_pad.shape
    K = yee.double_curl(nx, ny, nz).toarray()
    coords = unknown_coords(nx, ny, nz)
    r = yee.from_padded(r_pad)
    z = np.zeros_like(r)
    q, i, j, k = coords.T
    for s in subdomains(nx, ny, nz, sub, overlap):
        (ox0, ox1), (oy0, oy1), (oz0, oz1) = s["own"]
        (bx0, bx1), (by0, by1), (bz0, bz1) = s["box"]

        def inside(v, lo, hi, half):
            # half-point index v sits in cell v; node v must lie strictly inside (lo, hi)
            return np.where(half, (v >= lo) & (v < hi), (v > lo) & (v < hi))

        box = (inside(i, bx0, bx1, q == 0) & inside(j, by0, by1, q == 1)
               & inside(k, bz0, bz1, q == 2))
        own = ((i >= ox0) & (i < ox1) & (j >= oy0) & (j < oy1) & (k >= oz0) & (k < oz1))
        idx = np.nonzero(box)[0]
        alpha = subdomain_alpha(c, eps_cell, s["own"])
        Ai = np.eye(idx.size) + alpha * K[np.ix_(idx, idx)]
        sol = np.linalg.solve(Ai, r[idx])
        keep = own[idx]
        z[idx[keep]] = sol[keep]
    return yee.to_padded(z, nx, ny, nz)


def ras_apply_subset(r_pad, c, sub, overlap, eps_cell, which):
    """Owned output blocks of M_RAS^{-1} r for the subdomains listed in `which`.

    Returns {index: (owned ranges, block (3, sz, sy, sx))}; used to check a
    sample of subdomains of a grid too large for the full oracle.
    """
    _, nz, ny, nx = r_pad.shape
    subs = subdomains(nx, ny, nz, sub, overlap)
    out = {}
    for idx in which:
        s = subs[idx]
        (ox0, ox1), (oy0, oy1), (oz0, oz1) = s["own"]
        (bx0, bx1), (by0, by1), (bz0, bz1) = s["box"]
        alpha = subdomain_alpha(c, eps_cell, s["own"])
        box = np.array(r_pad[:, bz0:bz1, by0:by1, bx0:bx1], dtype=np.float64)
        e = transforms.box_solve_transform(yee.from_padded(box), bx1 - bx0, by1 - by0,
                                           bz1 - bz0, alpha)
        ebox = yee.to_padded(e, bx1 - bx0, by1 - by0, bz1 - bz0)
        out[idx] = (s["own"], ebox[:, oz0 - bz0:oz1 - bz0, oy0 - by0:oy1 - by0,
                                   ox0 - bx0:ox1 - bx0])
    return out
