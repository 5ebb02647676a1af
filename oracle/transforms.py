"""Discrete-transform exact solve of one PEC box (oracle; test infrastructure).

What this follows
-----------------
Sec. III-A, Steps 1-3 and the exact_solve function of Algorithm 1: transform
each field component with a tensor product of one-dimensional orthogonal
transforms (its own axis with one basis, the two transverse axes with the
other; the operator G), reorder to grid-major order (P), solve the 3x3 system
B_ijk e = r at every wavenumber (eq. (12)), reorder back and inverse
transform.

The paper builds the bases from the SVD of a compact forward-difference
matrix (eq. (8)) and needs a low-rank boundary correction (Step 4) because
its subdomain unknown set is not closed under the operator.  For a box whose
faces are PEC walls the singular vectors of the 1-D difference matrix
(n-1 interior nodes -> n half points) are known in closed form: the
orthonormal DCT-II of length n on the half points (U) and the orthonormal
DST-I of length n-1 on the nodes (V), with singular values
sigma_m = 2 sin(m pi / (2 n)).  With those bases the diagonalisation is exact
and Step 4 does not arise.

Index convention: spectral arrays share the padded shape (nz, ny, nx) of
their component; slot m of a node axis holds DST-I mode m (m >= 1), slot p of
the own (half-point) axis holds DCT-II mode p (p >= 0).
"""
import numpy as np

from . import yee


def dct2_matrix(n):
    """Orthonormal DCT-II, n x n: C[p, l] = sqrt(2/n) k_p cos(pi p (2l+1) / (2n)), k_0 = 1/sqrt(2)."""
    p = np.arange(n)[:, None]
    l = np.arange(n)[None, :]
    C = np.sqrt(2.0 / n) * np.cos(np.pi * p * (2 * l + 1) / (2 * n))
    C[0, :] /= np.sqrt(2.0)
    return C


def dst1_matrix(n):
    """Orthonormal DST-I on the n-1 interior nodes: S[m-1, l-1] = sqrt(2/n) sin(pi m l / n)."""
    m = np.arange(1, n)[:, None]
    l = np.arange(1, n)[None, :]
    return np.sqrt(2.0 / n) * np.sin(np.pi * m * l / n)


def sigma(n):
    """Singular values of the 1-D difference, indexed by mode m = 0..n-1 (sigma_0 = 0)."""
    return 2.0 * np.sin(np.pi * np.arange(n) / (2.0 * n))


def _along(Mat, arr, axis):
    """Contract matrix Mat (out x in) with `arr` along `axis` (the TrX/TrY/TrZ of eq. (9))."""
    out = np.tensordot(Mat, arr, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def component_bases(nx, ny, nz):
    """For each component, the (z, y, x) transform matrices: DCT-II on its own axis, DST-I elsewhere."""
    Cx, Cy, Cz = dct2_matrix(nx), dct2_matrix(ny), dct2_matrix(nz)
    Sx, Sy, Sz = dst1_matrix(nx), dst1_matrix(ny), dst1_matrix(nz)
    return [(Sz, Sy, Cx), (Sz, Cy, Sx), (Cz, Sy, Sx)]


def forward_G(u, nx, ny, nz):
    """G: compact unknown vector -> padded spectral array (3, nz, ny, nx)."""
    v = yee.to_padded(u, nx, ny, nz)
    comps = [v[0, 1:, 1:, :], v[1, 1:, :, 1:], v[2, :, 1:, 1:]]
    out = np.zeros((3, nz, ny, nx))
    for q, (Tz, Ty, Tx) in enumerate(component_bases(nx, ny, nz)):
        a = _along(Tx, comps[q], 2)
        a = _along(Ty, a, 1)
        a = _along(Tz, a, 0)
        if q == 0:
            out[0, 1:, 1:, :] = a
        elif q == 1:
            out[1, 1:, :, 1:] = a
        else:
            out[2, :, 1:, 1:] = a
    return out


def inverse_G(spec, nx, ny, nz):
    """G^{-1} = G^T: padded spectral array -> compact unknown vector."""
    comps = [spec[0, 1:, 1:, :], spec[1, 1:, :, 1:], spec[2, :, 1:, 1:]]
    parts = []
    for q, (Tz, Ty, Tx) in enumerate(component_bases(nx, ny, nz)):
        a = _along(Tz.T, comps[q], 0)
        a = _along(Ty.T, a, 1)
        a = _along(Tx.T, a, 2)
        parts.append(a.ravel())
    return np.concatenate(parts)


def block_matrices(nx, ny, nz, alpha):
    """B_ijk = I + alpha [[s_j^2+s_k^2, -s_i s_j, -s_i s_k], ...] at every wavenumber (eq. (12)).

    Returned with shape (nz, ny, nx, 3, 3); s_i, s_j, s_k are the x, y, z
    singular values of the wavenumber.  The off-diagonal signs are the minus
    signs of the B_ijk display (the scalar x-row printed just before it has
    them as plus, a typo).
    """
    sx = sigma(nx)[None, None, :]
    sy = sigma(ny)[None, :, None]
    sz = sigma(nz)[:, None, None]
    sx, sy, sz = np.broadcast_arrays(sx, sy, sz)
    B = np.zeros(sx.shape + (3, 3))
    B[..., 0, 0] = sy**2 + sz**2
    B[..., 1, 1] = sx**2 + sz**2
    B[..., 2, 2] = sx**2 + sy**2
    B[..., 0, 1] = B[..., 1, 0] = -sx * sy
    B[..., 0, 2] = B[..., 2, 0] = -sx * sz
    B[..., 1, 2] = B[..., 2, 1] = -sy * sz
    B *= alpha
    B[..., 0, 0] += 1.0
    B[..., 1, 1] += 1.0
    B[..., 2, 2] += 1.0
    return B


def box_solve_transform(u, nx, ny, nz, alpha):
    """exact_solve of (I + alpha K_box) e = u for a PEC box (Sec. III-A Step 3; Alg. 1).

    u, return value: compact unknown vectors of the box.
      1. R_hat = G u                               (Step 1, component-wise transform)
      2. reorder to grid-major: (r_x, r_y, r_z) per wavenumber   (Step 2, P)
      3. solve B_ijk e' = r' at each wavenumber    (eq. (12); a generic 3x3 solve)
      4. reorder back (P^T) and E = G^{-1} e'      (Step 3)
    Modes absent from a component (a DST slot 0) carry zero right-hand sides
    and come out zero, so the full 3x3 solve is used everywhere.
    """
    R = forward_G(u, nx, ny, nz)
    Rp = np.moveaxis(R, 0, -1)[..., None]                 # P: (nz, ny, nx, 3, 1)
    B = block_matrices(nx, ny, nz, alpha)
    Ep = np.linalg.solve(B, Rp)[..., 0]                   # per-point 3x3 solve
    E = np.moveaxis(Ep, -1, 0)                            # P^T
    return inverse_G(E, nx, ny, nz)


def box_solve_lu(u, nx, ny, nz, alpha):
    """Brute force: dense LU of the assembled box matrix I + alpha K_box."""
    import scipy.linalg as sla
    A = yee.assemble_A(nx, ny, nz, alpha).toarray()
    return sla.lu_solve(sla.lu_factor(A), u)
