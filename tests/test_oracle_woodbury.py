"""Pins of the index-block subdomain oracle (Sec. III-A Step 4, Algorithm 1).

Each check compares oracle/woodbury.py against something it does not compute
itself: the closed-form singular values of the compact difference, the global
operator assembled over the whole grid and restricted to a block by explicit
index sets, dense LU of that restriction, and the counts the paper states
(6n^2 - 3n boundary slots, delta = 2 on the n edge slots of a component).
Mistakes planted in a copy of the oracle (delta on the high face, no 2 on the
edges, walls treated as ordinary low faces) each fail one of these.
"""
import numpy as np
import pytest

from oracle import ras, woodbury as wb, yee


def test_compact_svd_closed_form():
    for n in (1, 2, 5, 8, 13):
        U, s, V = wb.compact_svd(n)
        m = np.arange(1, n + 1)
        closed = 2.0 * np.sin((2 * m - 1) * np.pi / (2 * (2 * n + 1)))
        assert np.allclose(np.sort(s), np.sort(closed), atol=1e-14, rtol=0)
        D = wb.compact_diff(n)
        assert np.allclose(U @ np.diag(s) @ V.T, D, atol=1e-14)
        assert np.allclose(U.T @ U, np.eye(n), atol=1e-14)
        assert np.allclose(V.T @ V, np.eye(n), atol=1e-14)
        # the backward difference shares the factors: D^b = -(D^f)^T = -V S U^T
        assert np.allclose(-(V @ np.diag(s) @ U.T), -D.T, atol=1e-14)


def test_exact_solve_inverts_the_compact_operator():
    rng = np.random.default_rng(0)
    for L, a in (((4, 5, 3), 0.7), ((6, 6, 6), 2.0), ((2, 7, 4), 8.0)):
        M = wb.compact_operator(L)
        X = rng.standard_normal((3, L[2], L[1], L[0]))
        Y = wb.exact_solve(X, L, a)
        ref = np.linalg.solve(np.eye(M.shape[0]) + a * M, X.ravel())
        assert np.abs(Y.ravel() - ref).max() <= 1e-13 * np.abs(ref).max()
        # a batch axis gives the same columns
        Yb = wb.exact_solve(np.stack([X, 2 * X]), L, a)
        assert np.allclose(Yb[1], 2 * Y, atol=1e-13)


def _restriction(N, lo, hi):
    """Global double curl K (assembled over the N grid) restricted to the index
    block [lo, hi) by explicit index sets, and each kept unknown's slot in the
    flattened (3, Lz, Ly, Lx) box."""
    K = yee.double_curl(*N).toarray()
    q, i, j, k = ras.unknown_coords(*N).T
    pos = (i, j, k)
    keep = np.ones(q.size, bool)
    for a in range(3):
        keep &= (pos[a] >= lo[a]) & (pos[a] < hi[a])
    idx = np.nonzero(keep)[0]
    L = tuple(h - l for l, h in zip(lo, hi))
    slot = (q[idx] * L[0] * L[1] * L[2] + ((k[idx] - lo[2]) * L[1] + (j[idx] - lo[1])) * L[0]
            + (i[idx] - lo[0]))
    return K[np.ix_(idx, idx)], slot, L


def test_boundary_term_is_the_restriction_defect():
    """Restricted global operator = compact operator + Lambda (Step 4), off the walls."""
    N = (11, 10, 12)
    for lo, hi in (((3, 2, 4), (8, 7, 9)), ((0, 3, 2), (5, 8, 7)), ((6, 5, 7), (11, 10, 12)),
                   ((0, 0, 0), (4, 6, 5))):
        Kr, slot, L = _restriction(N, lo, hi)
        Mc = wb.compact_operator(L)[np.ix_(slot, slot)]
        defect = Kr - Mc
        assert np.abs(defect - np.diag(np.diag(defect))).max() == 0.0   # diagonal only
        idx, winv = wb.boundary_weights(L, tuple(l == 0 for l in lo), 1.0)
        delta = np.zeros(3 * np.prod(L))
        free = winv > 0
        delta[idx[free]] = 1.0 / winv[free]                                # alpha = 1
        assert np.array_equal(np.diag(defect), delta[slot])


def test_boundary_counts_of_the_paper():
    for n in (3, 5, 8):
        idx, winv = wb.boundary_weights((n, n, n), (False,) * 3, 1.0)
        assert idx.size == 6 * n * n - 3 * n
        d = 1.0 / winv
        assert np.count_nonzero(d == 2.0) == 3 * n           # edge slots, delta = 2
        assert np.count_nonzero(d == 1.0) == 6 * n * n - 6 * n
    # Table II: C^{-1} of a 32^3 block holds (6n^2 - 3n)^2 doubles
    n = 32
    assert (6 * n * n - 3 * n) ** 2 * 8 == 292_626_432


@pytest.mark.parametrize("lo,hi,alpha", [
    ((3, 2, 4), (8, 7, 9), 0.8),       # interior block
    ((0, 3, 2), (5, 8, 7), 2.0),       # low wall in x
    ((0, 0, 0), (5, 5, 5), 8.0),       # corner at three low walls
    ((6, 5, 7), (11, 10, 12), 2.0),    # touches the three far walls
    ((0, 2, 0), (11, 8, 12), 0.5),     # spans x and z wall to wall
])
def test_algorithm1_equals_dense_lu_of_the_restriction(lo, hi, alpha):
    N = (11, 10, 12)
    Kr, slot, L = _restriction(N, lo, hi)
    rng = np.random.default_rng(sum(lo) + 7)
    r = rng.standard_normal(slot.size)
    ref = np.linalg.solve(np.eye(slot.size) + alpha * Kr, r)
    R = rng.standard_normal(3 * np.prod(L))          # wall slots carry garbage
    R[slot] = r
    E = wb.woodbury_solve(R.reshape(3, L[2], L[1], L[0]), L, tuple(l == 0 for l in lo), alpha)
    E = E.ravel()
    assert np.abs(E[slot] - ref).max() <= 1e-13 * np.abs(ref).max()
    wall = np.setdiff1d(np.arange(E.size), slot)
    assert np.abs(E[wall]).max(initial=0.0) <= 1e-13 * np.abs(ref).max()


def test_algorithm1_at_n5_to_rounding():
    """The n = 5 interior block: Algorithm 1 reproduces A^{-1} R to about 1e-15."""
    Kr, slot, L = _restriction((9, 9, 9), (2, 2, 2), (7, 7, 7))
    A = np.eye(slot.size) + 0.9 * Kr
    R = np.random.default_rng(5).standard_normal(slot.size)
    E = wb.woodbury_solve(R.reshape(3, 5, 5, 5), L, (False,) * 3, 0.9).ravel()
    assert np.abs(E - np.linalg.solve(A, R)).max() < 1e-14


def _ras_index_bruteforce(r_pad, c, sub, overlap, eps_cell):
    """RAS with index blocks from explicit index sets and dense solves of I + alpha K[box, box]."""
    _, nz, ny, nx = r_pad.shape
    K = yee.double_curl(nx, ny, nz).toarray()
    q, i, j, k = ras.unknown_coords(nx, ny, nz).T
    pos = (i, j, k)
    r = yee.from_padded(r_pad)
    z = np.zeros_like(r)
    for s in ras.subdomains(nx, ny, nz, sub, 0):
        own = s["own"]
        inbox = np.ones(q.size, bool)
        inown = np.ones(q.size, bool)
        for a, ((o0, o1), n) in enumerate(zip(own, (nx, ny, nz))):
            inbox &= (pos[a] >= max(o0 - overlap, 0)) & (pos[a] < min(o1 + overlap, n))
            inown &= (pos[a] >= o0) & (pos[a] < o1)
        idx = np.nonzero(inbox)[0]
        alpha = c if eps_cell is None else c / np.mean(
            eps_cell[own[2][0]:own[2][1], own[1][0]:own[1][1], own[0][0]:own[0][1]])
        sol = np.linalg.solve(np.eye(idx.size) + alpha * K[np.ix_(idx, idx)], r[idx])
        z[idx[inown[idx]]] = sol[inown[idx]]
    return yee.to_padded(z, nx, ny, nz)


@pytest.mark.parametrize("overlap", [0, 1])
def test_ras_index_matches_definition(overlap):
    n, sub, c = 8, 4, 2.0
    rng = np.random.default_rng(3 + overlap)
    eps = rng.uniform(1.0, 10.0, (4, 4, 4))
    eps_cell = yee.expand_eps(eps, 2, n, n, n)
    r = yee.to_padded(rng.standard_normal(yee.n_unknowns(n, n, n)), n, n, n)
    r_garbage = r + (~yee.wall_mask(n, n, n)) * rng.standard_normal(r.shape)
    z = wb.ras_apply_index(r_garbage, c, (sub,) * 3, overlap, eps_cell)
    ref = _ras_index_bruteforce(r, c, (sub,) * 3, overlap, eps_cell)
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()
    assert not np.any(z[~yee.wall_mask(n, n, n)])


def test_overlap0_is_block_jacobi():
    """With overlap 0 the blocks partition the unknowns and M^{-1} r solves each
    diagonal block: (I + alpha K_ii) z_i = r_i."""
    n, sub, c = 8, 4, 1.5
    rng = np.random.default_rng(9)
    r = yee.to_padded(rng.standard_normal(yee.n_unknowns(n, n, n)), n, n, n)
    z = yee.from_padded(wb.ras_apply_index(r, c, (sub,) * 3, 0, None))
    K = yee.double_curl(n, n, n)
    q, i, j, k = ras.unknown_coords(n, n, n).T
    blk = (i // sub) + 2 * (j // sub) + 4 * (k // sub)
    Kd = K.multiply(blk[:, None] == blk[None, :]).tocsr()            # block diagonal part
    assert np.abs(z + c * (Kd @ z) - yee.from_padded(r)).max() < 1e-12
