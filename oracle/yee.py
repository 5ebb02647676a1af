"""Yee-grid operator of the CN-FDTD linear system (oracle; test infrastructure).

What this follows
-----------------
* Sec. II-A, eqs. (4)-(5): each Crank-Nicolson step solves A E = R with
  A = I + (dt^2/4) curl curl.
* Sec. III-A, eq. (6): the discrete curl built from first-order differences,
  C = [[0, -D_z, D_y], [D_z, 0, -D_x], [-D_y, D_x, 0]], and the double-curl
  M = C^T C that enters eq. (7), (I + alpha M) E = R.  The printed second row
  of the curl and the (1,3) block of M carry typos; the reading used here is
  the standard Yee curl, whose C^T C is symmetric with integer entries.

Grid conventions
----------------
A domain of nx * ny * nz unit cells with perfectly conducting (PEC) walls on
all six faces.  E_x lives at (i+1/2, j, k): half points along x, nodes along
y and z.  Tangential E vanishes on the walls, so the unknowns are

    E_x : i in [0, nx),   j in [1, ny-1], k in [1, nz-1]
    E_y : i in [1, nx-1], j in [0, ny),   k in [1, nz-1]
    E_z : i in [1, nx-1], j in [1, ny-1], k in [0, nz)

The *compact* vector stacks [E_x, E_y, E_z], each in C order over (z, y, x).
The *padded* layout is an array of shape (3, nz, ny, nx): component q at
slot [k][j][i]; node slot 0 of a node axis is the wall and holds zero, the
far wall node (index n) is not stored.

Permittivity enters as A = I + c diag(1/eps_e) K, eps_e being the mean of
the relative permittivity of the four cells that share the edge.
"""
import numpy as np
import scipy.sparse as sp


def diff_matrix(n):
    """1-D difference from interior nodes to half points, shape (n, n-1).

    Column m-1 holds node m (m = 1..n-1); row i is the half point i+1/2 and
    (D y)_i = y_{i+1} - y_i with the wall nodes y_0 = y_n = 0 (Sec. III-A,
    forward difference D^f restricted to the PEC unknowns).
    """
    rows, cols, vals = [], [], []
    for i in range(n):
        if i + 1 <= n - 1:          # node i+1 is interior
            rows.append(i); cols.append(i); vals.append(1.0)
        if i >= 1:                  # node i is interior
            rows.append(i); cols.append(i - 1); vals.append(-1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n - 1))


def component_shapes(nx, ny, nz):
    """Shapes (z, y, x) of the E_x, E_y, E_z unknown arrays."""
    return [(nz - 1, ny - 1, nx), (nz - 1, ny, nx - 1), (nz, ny - 1, nx - 1)]


def n_unknowns(nx, ny, nz):
    return sum(int(np.prod(s)) for s in component_shapes(nx, ny, nz))


def curl_matrix(nx, ny, nz):
    """Sparse discrete curl C: E unknowns -> H on the dual faces (eq. (6)).

    Rows are H_x at (i, j+1/2, k+1/2), H_y at (i+1/2, j, k+1/2) and
    H_z at (i+1/2, j+1/2, k), each block in C order (z, y, x):
        H_x = d_y E_z - d_z E_y
        H_y = d_z E_x - d_x E_z
        H_z = d_x E_y - d_y E_x
    H points on the walls, where both contributing tangential E vanish, are
    left out (their rows would be zero).
    """
    I = lambda m: sp.identity(m, format="csr")
    Dx, Dy, Dz = diff_matrix(nx), diff_matrix(ny), diff_matrix(nz)
    kron3 = lambda a, b, c: sp.kron(sp.kron(a, b), c, format="csr")
    sx, sy, sz = component_shapes(nx, ny, nz)
    nEx, nEy, nEz = (int(np.prod(s)) for s in (sx, sy, sz))

    # H_x: shape (nz, ny, nx-1)
    hx_dzEy = kron3(Dz, I(ny), I(nx - 1))
    hx_dyEz = kron3(I(nz), Dy, I(nx - 1))
    Hx = sp.hstack([sp.csr_matrix((hx_dzEy.shape[0], nEx)), -hx_dzEy, hx_dyEz])
    # H_y: shape (nz, ny-1, nx)
    hy_dzEx = kron3(Dz, I(ny - 1), I(nx))
    hy_dxEz = kron3(I(nz), I(ny - 1), Dx)
    Hy = sp.hstack([hy_dzEx, sp.csr_matrix((hy_dzEx.shape[0], nEy)), -hy_dxEz])
    # H_z: shape (nz-1, ny, nx)
    hz_dxEy = kron3(I(nz - 1), I(ny), Dx)
    hz_dyEx = kron3(I(nz - 1), Dy, I(nx))
    Hz = sp.hstack([-hz_dyEx, hz_dxEy, sp.csr_matrix((hz_dxEy.shape[0], nEz))])
    return sp.vstack([Hx, Hy, Hz], format="csr")


def double_curl(nx, ny, nz):
    """K = C^T C, the double-curl matrix M of Sec. III-A (unit spacing)."""
    C = curl_matrix(nx, ny, nz)
    return (C.T @ C).tocsr()


def expand_eps(eps_block, block, nx, ny, nz):
    """Cell permittivity (nz, ny, nx) from a table of constant cubes of side `block`."""
    eps_block = np.asarray(eps_block, dtype=np.float64)
    cell = np.repeat(np.repeat(np.repeat(eps_block, block, 0), block, 1), block, 2)
    return np.ascontiguousarray(cell[:nz, :ny, :nx])


def edge_eps(eps_cell):
    """Permittivity at each E unknown: mean of the four cells sharing the edge.

    Returns the compact vector (same ordering as the unknowns).
    """
    e = np.asarray(eps_cell, dtype=np.float64)
    ex = 0.25 * (e[:-1, :-1, :] + e[1:, :-1, :] + e[:-1, 1:, :] + e[1:, 1:, :])
    ey = 0.25 * (e[:-1, :, :-1] + e[1:, :, :-1] + e[:-1, :, 1:] + e[1:, :, 1:])
    ez = 0.25 * (e[:, :-1, :-1] + e[:, 1:, :-1] + e[:, :-1, 1:] + e[:, 1:, 1:])
    return np.concatenate([ex.ravel(), ey.ravel(), ez.ravel()])


def assemble_A(nx, ny, nz, c, eps_cell=None):
    """A = I + c diag(1/eps_e) K as a sparse matrix (eqs. (5), (7))."""
    K = double_curl(nx, ny, nz)
    n = K.shape[0]
    if eps_cell is None:
        scale = np.full(n, float(c))
    else:
        scale = float(c) / edge_eps(eps_cell)
    return (sp.identity(n, format="csr") + sp.diags(scale) @ K).tocsr()


def to_padded(u, nx, ny, nz):
    """Compact unknown vector -> padded (3, nz, ny, nx) array, walls zero."""
    sx, sy, sz = component_shapes(nx, ny, nz)
    u = np.asarray(u)
    a, b = int(np.prod(sx)), int(np.prod(sy))
    v = np.zeros((3, nz, ny, nx), dtype=u.dtype)
    v[0, 1:, 1:, :] = u[:a].reshape(sx)
    v[1, 1:, :, 1:] = u[a:a + b].reshape(sy)
    v[2, :, 1:, 1:] = u[a + b:].reshape(sz)
    return v


def from_padded(v):
    """Padded (3, nz, ny, nx) array -> compact unknown vector (wall slots dropped)."""
    v = np.asarray(v)
    return np.concatenate([v[0, 1:, 1:, :].ravel(), v[1, 1:, :, 1:].ravel(),
                           v[2, :, 1:, 1:].ravel()])


def wall_mask(nx, ny, nz):
    """Boolean padded mask, True on unknown slots."""
    m = np.zeros((3, nz, ny, nx), dtype=bool)
    m[0, 1:, 1:, :] = True
    m[1, 1:, :, 1:] = True
    m[2, :, 1:, 1:] = True
    return m


def apply_A_padded(v, c, eps_cell=None):
    """y = A v for a padded vector, through the sparse matrix (wall slots of y are 0)."""
    _, nz, ny, nx = v.shape
    A = assemble_A(nx, ny, nz, c, eps_cell)
    return to_padded(A @ from_padded(v), nx, ny, nz)


def apply_A_at(v, c, eps_cell, points):
    """(A v) at selected padded slots, for checks on grids too large to assemble.

    points: iterable of (q, k, j, i).  Each value comes from a window of up to
    5 cells per axis around the slot, assembled as its own PEC domain whose
    low faces start at least two cells before the slot; the stencil of the
    centre slot reaches one cell, so it only sees window-interior values and
    the result equals the global operator's.  A window face that coincides
    with a global wall is that wall.
    """
    _, nz, ny, nx = v.shape
    out = []
    for (q, k, j, i) in points:
        lo = [max(0, a - 2) for a in (i, j, k)]
        hi = [min(n, a + 3) for a, n in zip((i, j, k), (nx, ny, nz))]
        sub = v[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].copy()
        wnx, wny, wnz = hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]
        # a window slot 0 that is not a global wall is an ordinary value the
        # centre stencil never touches; zero it so the window is a valid input
        sub[0, 0, :, :] = 0; sub[0, :, 0, :] = 0
        sub[1, 0, :, :] = 0; sub[1, :, :, 0] = 0
        sub[2, :, 0, :] = 0; sub[2, :, :, 0] = 0
        ew = None if eps_cell is None else eps_cell[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        y = apply_A_padded(sub, c, ew)
        out.append(y[q, k - lo[2], j - lo[1], i - lo[0]])
    return np.array(out)
