"""Crank-Nicolson FDTD time stepping around the solve (oracle; test infrastructure).

What this follows
-----------------
Sec. II-A, eqs. (2)-(5): Maxwell's curl equations marched by Crank-Nicolson,
the new and old curls averaged,

    eps (E+ - E) / dt =  (1/2) curl (H+ + H)                     (2)
    mu  (H+ - H) / dt = -(1/2) curl (E+ + E)                     (3)

and H+ eliminated, so each step solves A E+ = R (eqs. (4)-(5)).  The paper
writes it for eps = mu = 1; with a relative permittivity eps (mu = 1, unit
cell size) the same elimination gives

    (I + c eps^-1 C^T C) E+ = E + dt eps^-1 C^T H - c eps^-1 C^T C E,
    c = dt^2 / 4,

where C is the discrete curl of Sec. III-A eq. (6) (E on Yee edges -> H on
the dual faces, yee.curl_matrix) and C^T the curl from H back to E.  The
operator is yee.assemble_A; the right-hand side is written here as
R = E + dt eps^-1 C^T (H - (dt/4) C E).  H+ then follows from eq. (3).

Reading: the time step of a domain is fixed by its c as dt = 2 sqrt(c)
(mu = 1, unit spacing), the relation the configurations state for c.

Vectors here are compact (unknowns only): E as in yee, H as the rows of
yee.curl_matrix (H_x, H_y, H_z blocks, each C order over (z, y, x)).  The
padded H layout matches the padded E layout: shape (3, nz, ny, nx), H_x at
(i, j+1/2, k+1/2) in slot [k][j][i] with i >= 1, H_y at (i+1/2, j, k+1/2)
with j >= 1, H_z at (i+1/2, j+1/2, k) with k >= 1; slot 0 of a component's
own (node) axis is a wall slot.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import yee


def h_shapes(nx, ny, nz):
    """Shapes (z, y, x) of the H_x, H_y, H_z unknown arrays."""
    return [(nz, ny, nx - 1), (nz, ny - 1, nx), (nz - 1, ny, nx)]


def h_to_padded(u, nx, ny, nz):
    sx, sy, sz = h_shapes(nx, ny, nz)
    a, b = int(np.prod(sx)), int(np.prod(sy))
    v = np.zeros((3, nz, ny, nx))
    v[0, :, :, 1:] = u[:a].reshape(sx)
    v[1, :, 1:, :] = u[a:a + b].reshape(sy)
    v[2, 1:, :, :] = u[a + b:].reshape(sz)
    return v


def h_from_padded(v):
    return np.concatenate([v[0, :, :, 1:].ravel(), v[1, :, 1:, :].ravel(), v[2, 1:, :, :].ravel()])


def h_mask(nx, ny, nz):
    m = np.zeros((3, nz, ny, nx), dtype=bool)
    m[0, :, :, 1:] = True
    m[1, :, 1:, :] = True
    m[2, 1:, :, :] = True
    return m


def time_step(c):
    """dt of a domain with operator coefficient c = dt^2 / 4 (mu = 1, unit spacing)."""
    return 2.0 * np.sqrt(c)


def edge_eps_or_one(nx, ny, nz, eps_cell):
    n = yee.n_unknowns(nx, ny, nz)
    return np.ones(n) if eps_cell is None else yee.edge_eps(eps_cell)


def cn_step(E, H, nx, ny, nz, c, eps_cell=None):
    """One CN step on compact vectors (eqs. (2)-(5)) with a direct sparse solve.

    Returns (E+, H+).
      R  = E + dt eps^-1 C^T (H - (dt/4) C E)       right-hand side of eq. (4)
      E+ = A^-1 R                                   eq. (5)
      H+ = H - (dt/2) C (E+ + E)                    eq. (3) with mu = 1
    """
    C = yee.curl_matrix(nx, ny, nz)
    A = yee.assemble_A(nx, ny, nz, c, eps_cell).tocsc()
    eps_e = edge_eps_or_one(nx, ny, nz, eps_cell)
    dt = time_step(c)
    R = E + (dt / eps_e) * (C.T @ (H - (dt / 4.0) * (C @ E)))
    E1 = spla.spsolve(A, R)
    H1 = H - (dt / 2.0) * (C @ (E1 + E))
    return E1, H1


def energy(E, H, eps_e):
    """Discrete electromagnetic energy (1/2)(sum eps_e E^2 + sum H^2) (mu = 1)."""
    return 0.5 * (float(np.dot(eps_e * E, E)) + float(np.dot(H, H)))


def _window(a, n):
    return max(0, a - 2), min(n, a + 3)


def curl_e_at(e_pad, points):
    """(C E) at selected padded H slots, for checks on grids too large to assemble.

    Each value comes from a window of up to 5 cells per axis around the slot,
    assembled as its own PEC domain (yee.curl_matrix): the face curl of the
    centre slot reads E at its own index and one above, both inside the
    window, so the window's own walls never enter it."""
    _, nz, ny, nx = e_pad.shape
    out = []
    for (q, k, j, i) in points:
        (x0, x1), (y0, y1), (z0, z1) = _window(i, nx), _window(j, ny), _window(k, nz)
        sub = e_pad[:, z0:z1, y0:y1, x0:x1] * yee.wall_mask(x1 - x0, y1 - y0, z1 - z0)
        C = yee.curl_matrix(x1 - x0, y1 - y0, z1 - z0)
        hw = h_to_padded(C @ yee.from_padded(sub), x1 - x0, y1 - y0, z1 - z0)
        out.append(hw[q, k - z0, j - y0, i - x0])
    return np.array(out)


def curl_h_at(h_pad, eps_cell, points):
    """(C^T H) and the edge permittivity at selected padded E slots (same
    window construction; the edge curl reads H at its own index and one
    below, and the four cells around the edge)."""
    _, nz, ny, nx = h_pad.shape
    ct, ee = [], []
    for (q, k, j, i) in points:
        (x0, x1), (y0, y1), (z0, z1) = _window(i, nx), _window(j, ny), _window(k, nz)
        wnx, wny, wnz = x1 - x0, y1 - y0, z1 - z0
        sub = h_pad[:, z0:z1, y0:y1, x0:x1] * h_mask(wnx, wny, wnz)
        C = yee.curl_matrix(wnx, wny, wnz)
        ew = yee.to_padded(C.T @ h_from_padded(sub), wnx, wny, wnz)
        ct.append(ew[q, k - z0, j - y0, i - x0])
        if eps_cell is None:
            ee.append(1.0)
        else:
            e_e = yee.to_padded(yee.edge_eps(eps_cell[z0:z1, y0:y1, x0:x1]), wnx, wny, wnz)
            ee.append(e_e[q, k - z0, j - y0, i - x0])
    return np.array(ct), np.array(ee)
