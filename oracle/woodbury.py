"""Index-block subdomain solve with the low-rank boundary correction (oracle).

Test infrastructure only (see the package docstring): a plain NumPy statement
of what the library's index-block preconditioner computes.

What this follows
-----------------
Sec. III-A as the paper states it for an index-block subdomain:

* The compact forward difference D^f (n x n: -1 on the diagonal, +1 above
  it; the node past the block's end is zero) and its SVD D^f = U S V^T
  (eq. (8)).  Backward differences are D^b = -(D^f)^T.
* The transform G: per field component, U^T along the component's own
  (half-point) axis and V^T along its two node axes (TrX/TrY/TrZ of eq. (9)).
* exact_solve (Algorithm 1): X_hat = G X, a 3x3 solve with B_ijk at every
  wavenumber (eq. (12)), Y = G^T Y_hat.  It inverts I + alpha M with M the
  double curl assembled from the compact differences.
* Step 4: the restriction of the global operator to the block differs from
  I + alpha M by the diagonal alpha Lambda, delta in {0, 1, 2} counting the
  node axes along which the slot sits on the block's low face (the half point
  below that face is dropped by the compact differences).  Lambda = Q W Q^T /
  alpha with Q the selection of the 6n^2 - 3n boundary slots; Woodbury gives
  (A0 + Q W Q^T)^{-1} = A0^{-1} - A0^{-1} Q C^{-1} Q^T A0^{-1},
  C = W^{-1} + Q^T A0^{-1} Q, and Algorithm 1's main body applies it:
  E = exact_solve(R); E -= exact_solve(Q C^{-1} Q^T E).

Readings (the paper leaves these open)
--------------------------------------
* Box of a subdomain: along each axis the index range [max(a - gamma, 0),
  min(a + n + gamma, N)) of the owned block [a, a + n) extended by the overlap
  gamma (0 allowed), for half points and nodes alike; every component of a
  box has all L_x * L_y * L_z slots.  Half point i sits between nodes i and
  i+1, so the block's own differences reach the node past its end (outside
  the box: zero, or the far PEC wall, also zero).
* A box that starts at a global PEC wall holds the wall node (index 0) of
  that axis: it is not an unknown.  Its slots are constrained to zero: the
  same Woodbury formula with those entries of W^{-1} set to 0 (the limit of
  an infinite weight), which solves the restricted system on the remaining
  unknowns exactly and returns zero on the wall slots whatever r holds there.
* alpha_s = c / (mean eps_r over the owned cells), as for the PEC boxes.
"""
import numpy as np

from . import ras, transforms, yee


def compact_diff(n):
    """D^f of the compact index block: (D y)_i = y_{i+1} - y_i, y_{n} = 0 (n x n)."""
    D = -np.eye(n)
    D[np.arange(n - 1), np.arange(1, n)] = 1.0
    return D


def compact_svd(n):
    """U, sigma, V with D^f = U diag(sigma) V^T (eq. (8)); numpy's SVD, any signs."""
    U, s, Vt = np.linalg.svd(compact_diff(n))
    return U, s, Vt.T


def _bases(L):
    """Per component, the (z, y, x) forward matrices of G: U^T on the own axis, V^T elsewhere."""
    Ut, Vt, sig = [], [], []
    for n in L:
        U, s, V = compact_svd(n)
        Ut.append(U.T)
        Vt.append(V.T)
        sig.append(s)
    Lx = [(Vt[2], Vt[1], Ut[0]), (Vt[2], Ut[1], Vt[0]), (Ut[2], Vt[1], Vt[0])]
    return Lx, sig


def exact_solve(X, L, alpha):
    """(I + alpha M)^{-1} X on box arrays X of shape (..., 3, Lz, Ly, Lx) (Algorithm 1).

    M is the double curl of the compact differences; L = (Lx, Ly, Lz).
      1. X_hat = G X                              (Step 1)
      2. per wavenumber, B_ijk Y' = X'            (Step 2, eq. (12), generic 3x3 solve)
      3. Y = G^T Y_hat                            (Step 3)
    Leading axes of X are a batch.
    """
    bases, sig = _bases(L)
    X = np.asarray(X, dtype=np.float64)
    lead = X.ndim - 4
    spec = np.empty_like(X)
    for q, (Tz, Ty, Tx) in enumerate(bases):
        a = transforms._along(Tx, X[..., q, :, :, :], lead + 2)
        a = transforms._along(Ty, a, lead + 1)
        spec[..., q, :, :, :] = transforms._along(Tz, a, lead)
    sx = sig[0][None, None, :]
    sy = sig[1][:, None][None, :, :]
    sz = sig[2][:, None, None]
    sx, sy, sz = np.broadcast_arrays(sx, sy, sz)
    B = np.zeros(sx.shape + (3, 3))
    B[..., 0, 0] = sy**2 + sz**2
    B[..., 1, 1] = sx**2 + sz**2
    B[..., 2, 2] = sx**2 + sy**2
    B[..., 0, 1] = B[..., 1, 0] = -sx * sy
    B[..., 0, 2] = B[..., 2, 0] = -sx * sz
    B[..., 1, 2] = B[..., 2, 1] = -sy * sz
    B = np.eye(3) + alpha * B
    Rp = np.moveaxis(spec, lead, -1)[..., None]                   # P: grid-major
    Ep = np.linalg.solve(np.broadcast_to(B, Rp.shape[:-2] + (3, 3)), Rp)[..., 0]
    spec = np.moveaxis(Ep, -1, lead)                              # P^T
    Y = np.empty_like(X)
    for q, (Tz, Ty, Tx) in enumerate(bases):
        a = transforms._along(Tz.T, spec[..., q, :, :, :], lead)
        a = transforms._along(Ty.T, a, lead + 1)
        Y[..., q, :, :, :] = transforms._along(Tx.T, a, lead + 2)
    return Y


def compact_operator(L):
    """Dense I-free double curl M = C^T C from the compact differences, on (3, Lz, Ly, Lx) slots."""
    Lx, Ly, Lz = L
    Dx, Dy, Dz = compact_diff(Lx), compact_diff(Ly), compact_diff(Lz)
    Ix, Iy, Iz = np.eye(Lx), np.eye(Ly), np.eye(Lz)
    k3 = lambda a, b, c: np.kron(np.kron(a, b), c)
    Z = np.zeros((Lx * Ly * Lz,) * 2)
    # H_x = d_y E_z - d_z E_y, H_y = d_z E_x - d_x E_z, H_z = d_x E_y - d_y E_x
    dX, dY, dZ = k3(Iz, Iy, Dx), k3(Iz, Dy, Ix), k3(Dz, Iy, Ix)
    C = np.block([[Z, -dZ, dY], [dZ, Z, -dX], [-dY, dX, Z]])
    return C.T @ C


def boundary_weights(L, low_wall, alpha):
    """Q as slot indices into the flattened (3, Lz, Ly, Lx) box, and W^{-1} per column.

    delta counts the node axes of a component along which the slot is on the
    box's low face (Step 4); Q takes every slot with delta > 0, in flattened
    order (6n^2 - 3n of them for a cubic box of side n).  W^{-1} = 1/(alpha
    delta), or 0 where the slot is a wall node (low_wall[a] and index 0 along
    a node axis a): a constraint.
    """
    Lx, Ly, Lz = L
    k, j, i = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    pos = (i, j, k)
    idx, winv = [], []
    for q in range(3):
        nodes = [a for a in range(3) if a != q]
        delta = sum((pos[a] == 0).astype(int) for a in nodes)
        wall = np.zeros_like(delta, dtype=bool)
        for a in nodes:
            if low_wall[a]:
                wall |= pos[a] == 0
        sel = np.nonzero(delta.ravel() > 0)[0]
        idx.append(q * Lx * Ly * Lz + sel)
        d = delta.ravel()[sel].astype(np.float64)
        w = 1.0 / (alpha * d)
        w[wall.ravel()[sel]] = 0.0
        winv.append(w)
    return np.concatenate(idx), np.concatenate(winv)


def correction_matrix(L, low_wall, alpha):
    """C = W^{-1} + Q^T A0^{-1} Q (dense), with A0^{-1} Q from exact_solve of Q's columns."""
    idx, winv = boundary_weights(L, low_wall, alpha)
    Lx, Ly, Lz = L
    m = idx.size
    cols = np.zeros((m, 3 * Lx * Ly * Lz))
    cols[np.arange(m), idx] = 1.0
    sol = exact_solve(cols.reshape(m, 3, Lz, Ly, Lx), L, alpha).reshape(m, -1)
    C = sol[:, idx].T + np.diag(winv)
    return idx, C


def woodbury_solve(R, L, low_wall, alpha, corr=None):
    """(A0 + Q W Q^T)^{-1} R on one box array (3, Lz, Ly, Lx): Algorithm 1's main body.

      E    = exact_solve(R)
      CorR = Q C^{-1} Q^T E          (the GEMV with the precomputed C^{-1})
      CorE = exact_solve(CorR)
      E    = E - CorE
    corr: optional precomputed (Q indices, C) of correction_matrix.
    """
    idx, C = correction_matrix(L, low_wall, alpha) if corr is None else corr
    E = exact_solve(R, L, alpha)
    corr = np.zeros(E.size)
    corr[idx] = np.linalg.solve(C, E.ravel()[idx])
    return E - exact_solve(corr.reshape(E.shape), L, alpha)


def index_boxes(nx, ny, nz, sub, overlap):
    """Subdomains in (z, y, x) C order with owned ranges and index-block box ranges.

    Along each axis the box is [max(a - overlap, 0), min(a + sub + overlap, n)).
    """
    out = []
    for s in ras.subdomains(nx, ny, nz, sub, 0):
        own = s["own"]
        box = tuple((max(lo - overlap, 0), min(hi + overlap, n))
                    for (lo, hi), n in zip(own, (nx, ny, nz)))
        out.append(dict(own=own, box=box))
    return out


def ras_apply_index(r_pad, c, sub, overlap=0, eps_cell=None, cache=None):
    """z = M_RAS^{-1} r with index-block subdomains solved by Algorithm 1 (Sec. II-B, III-A).

    r_pad, return value: padded (3, nz, ny, nx) arrays; wall slots of r are
    ignored and those of z are zero.  cache: optional dict that keeps the
    correction matrices C (one per box shape, wall pattern and alpha) between
    calls, as Algorithm 1 takes C^{-1} precomputed.
    """
    _, nz, ny, nx = r_pad.shape
    r_pad = r_pad * yee.wall_mask(nx, ny, nz)
    z = np.zeros_like(r_pad, dtype=np.float64)
    for s in index_boxes(nx, ny, nz, sub, overlap):
        (ox0, ox1), (oy0, oy1), (oz0, oz1) = s["own"]
        (bx0, bx1), (by0, by1), (bz0, bz1) = s["box"]
        L = (bx1 - bx0, by1 - by0, bz1 - bz0)
        alpha = ras.subdomain_alpha(c, eps_cell, s["own"])
        R = np.array(r_pad[:, bz0:bz1, by0:by1, bx0:bx1], dtype=np.float64)
        walls = (bx0 == 0, by0 == 0, bz0 == 0)
        corr = None
        if cache is not None:
            key = (L, walls, alpha)
            if key not in cache:
                cache[key] = correction_matrix(L, walls, alpha)
            corr = cache[key]
        E = woodbury_solve(R, L, walls, alpha, corr)
        z[:, oz0:oz1, oy0:oy1, ox0:ox1] = E[:, oz0 - bz0:oz1 - bz0, oy0 - by0:oy1 - by0,
                                            ox0 - bx0:ox1 - bx0]
    return z * yee.wall_mask(nx, ny, nz)
