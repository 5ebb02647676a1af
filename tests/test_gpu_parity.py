"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances (FP64): the stencil sums at most 13 products of an integer weight
and a value, scaled once by c/eps; its rounding error is below
16 u (1 + 12 c/eps_min) max|x| with u = 2^-53, so 1e-13 max|x| bounds it for
the c <= 8 used here.  The transform solve applies six orthogonal contractions
of length <= 34 and a pointwise 3x3 solve; each contraction adds at most
34 u relative error in the max norm, so 1e-12 relative (max norm) is a safe
bound with margin for the box solve's conditioning (eigenvalues of B in
[1, 1 + 12 alpha]).
"""
import numpy as np
import pytest
import torch

from oracle import krylov, ras, transforms, yee
from paper_2508_07193_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to(DEV)


def host(t, shape):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


def handle_for(P, **kw):
    return api.Handle([dict(nx=P["nx"], ny=P["ny"], nz=P["nz"], c=P["c"], eps=P["eps"],
                            eps_block=P.get("eps_block", 0), sub=P["sub"])], device=DEV, **kw)


def eps_cell_of(P):
    if P["eps"] is None:
        return None
    return yee.expand_eps(P["eps"], P["eps_block"], P["nx"], P["ny"], P["nz"])


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def problem(n, sub, c, eps_block, seed):
    return inputs.make_problem(dict(n=n, sub=sub, c=c, eps_block=eps_block, seed=seed))


# ------------------------------------------------------------------ stencil
def test_stencil_integer_inputs_bitwise():
    nx, ny, nz = 70, 10, 19           # ragged against the 64 x 4 x 16 tiles
    rng = np.random.default_rng(0)
    v = rng.integers(-8, 9, size=(3, nz, ny, nx)).astype(np.float64)
    # garbage on the wall slots must be ignored
    mask = inputs.unknown_slots(nx, ny, nz)
    ref = yee.apply_A_padded(np.where(mask, v, 0.0), 2.0)
    h = api.Handle([dict(nx=nx, ny=ny, nz=nz, c=2.0)], device=DEV)
    y = h.new_vector()
    h.curlcurl_apply(dev(v), y)
    out = host(y, ref.shape)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("shape,blk,c", [((40, 36, 34), 4, 2.0), ((17, 23, 9), 3, 8.0)])
def test_stencil_random_eps(shape, blk, c):
    nx, ny, nz = shape
    rng = np.random.default_rng(1)
    eps = inputs.eps_table(rng, nx, ny, nz, blk)       # ceil(n / blk) cubes per axis
    v = inputs.normal_rhs(rng, nx, ny, nz)
    ref = yee.apply_A_padded(v, c, yee.expand_eps(eps, blk, nx, ny, nz))
    h = api.Handle([dict(nx=nx, ny=ny, nz=nz, c=c, eps=eps, eps_block=blk)], device=DEV)
    y = h.new_vector()
    h.curlcurl_apply(dev(v), y)
    out = host(y, ref.shape)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(v).max()


def test_stencil_two_domains():
    rng = np.random.default_rng(2)
    d1 = dict(nx=12, ny=16, nz=8, c=0.5)
    d2 = dict(nx=24, ny=24, nz=24, c=3.0)
    v1 = inputs.normal_rhs(rng, 12, 16, 8)
    v2 = inputs.normal_rhs(rng, 24, 24, 24)
    h = api.Handle([d1, d2], device=DEV)
    assert h.offsets == [0, v1.size, v1.size + v2.size]
    y = h.new_vector()
    h.curlcurl_apply(torch.cat([dev(v1), dev(v2)]), y)
    out = y.cpu().numpy()
    r1 = yee.apply_A_padded(v1, 0.5)
    r2 = yee.apply_A_padded(v2, 3.0)
    assert relmax(out[:v1.size].reshape(r1.shape), r1) < 1e-14
    assert relmax(out[v1.size:].reshape(r2.shape), r2) < 1e-14


# ------------------------------------------------------------------ preconditioner
@pytest.mark.parametrize("n,sub,c,blk,overlap", [
    (32, 16, 2.0, 8, 1),               # 8 boxes of 17^3
    (48, 16, 8.0, 8, 1),               # 27 boxes of sides {17, 18}
    (24, 8, 2.0, 4, 2),                # overlap 2, boxes {10, 12}
    (16, 0, 0.5, 0, 1),                # one box = the whole domain (C1 shape)
    (96, 32, 2.0, 8, 3),               # size class 40: boxes {35, 38}
    (102, 34, 2.0, 6, 3),              # size class 40: boxes {37, 40}
    (84, 42, 8.0, 4, 3),               # size class 48: boxes of 45
    (12, 4, 2.0, 4, 1),                # size class 8: boxes {5, 6}
    (21, 7, 4.0, 3, 1),                # odd sides {8, 9}: classes 8 and 16 in one apply
])
def test_precond_fp64_matches_oracle(n, sub, c, blk, overlap):
    P = problem(n, sub, c, blk, seed=n + sub)
    h = handle_for(P, overlap=overlap)
    r = P["rhs"].copy()
    garbage = np.where(inputs.unknown_slots(n, n, n), r, 123.0)   # walls ignored on input
    z = h.new_vector()
    h.apply_precond(dev(garbage), z)
    ref = ras.ras_apply(r, c, P["sub"], overlap, eps_cell_of(P))
    out = host(z, ref.shape)
    assert relmax(out, ref) < 1e-12
    assert np.all(out[~inputs.unknown_slots(n, n, n)] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,sub", [(48, 16), (64, 0)])   # 27 boxes of 17/18; one box of 64
def test_precond_ignores_nonfinite_wall_slots(prec, n, sub):
    """Wall slots of r are outside the unknown set: NaN and +-Inf there must
    leave z bitwise as with zeros there.  The vector-ALU passes copy the wall
    slots into the transform staging unmasked (every DST-I skips its slot 0),
    so this checks that no such value reaches a consumed coefficient; the
    BF16 and large-box paths zero them on the gather."""
    P = problem(n, sub, 2.0, 8, seed=n + 7)
    h = handle_for(P, precision=prec)
    r = P["rhs"].copy()
    wall = ~inputs.unknown_slots(n, n, n)
    bad = r.copy()
    vals = np.array([np.nan, np.inf, -np.inf])
    bad[wall] = vals[np.arange(int(wall.sum())) % 3]
    z0, z1 = h.new_vector(), h.new_vector()
    h.apply_precond(dev(r), z0)
    h.apply_precond(dev(bad), z1)
    a, b = host(z0, r.shape), host(z1, r.shape)
    assert np.all(np.isfinite(b))
    assert np.array_equal(a, b)


def test_stencil_ignores_nonfinite_wall_slots():
    """The same for y = A x (default 64 x 8 tiles; the staging that masks
    the wall slots is common to every tile height)."""
    nx, ny, nz = 70, 21, 19
    rng = np.random.default_rng(8)
    x = inputs.normal_rhs(rng, nx, ny, nz)
    wall = ~inputs.unknown_slots(nx, ny, nz)
    bad = x.copy()
    bad[wall] = np.array([np.nan, np.inf, -np.inf])[np.arange(int(wall.sum())) % 3]
    eps = inputs.eps_table(rng, nx, ny, nz, 4)
    h = api.Handle([dict(nx=nx, ny=ny, nz=nz, c=2.0, eps=eps, eps_block=4)], device=DEV)
    y0, y1 = h.new_vector(), h.new_vector()
    h.curlcurl_apply(dev(x), y0)
    h.curlcurl_apply(dev(bad), y1)
    a, b = host(y0, x.shape), host(y1, x.shape)
    assert np.all(np.isfinite(b)) and np.array_equal(a, b)


def test_precond_anisotropic_domain():
    nx, ny, nz, sub, c = 48, 32, 24, (16, 16, 8), 1.5
    rng = np.random.default_rng(5)
    eps = inputs.eps_table(rng, nx, ny, nz, 8)
    r = inputs.normal_rhs(rng, nx, ny, nz)
    h = api.Handle([dict(nx=nx, ny=ny, nz=nz, c=c, eps=eps, eps_block=8, sub=sub)], device=DEV)
    z = h.new_vector()
    h.apply_precond(dev(r), z)
    ref = ras.ras_apply(r, c, sub, 1, yee.expand_eps(eps, 8, nx, ny, nz))
    assert relmax(host(z, ref.shape), ref) < 1e-12


def rel2(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


# Reduced precision: each of the six contractions rounds its inputs and the
# table entries (unit roundoff u: 2^-24 FP32, 2^-8 bf16), so each stage adds a
# 2-norm error of at most about 2u of its input's norm (the transforms are
# orthogonal and the 3x3 solve is a contraction, ||B^-1|| <= 1).  Bound, box by
# box: ||z_own - z_own_exact||_2 <= 12u ||S^gamma r||_2, the owned block's
# error against the norm of that box's restricted input.  A whole-vector norm
# would hide a box face that is wrong by O(1); a per-box one does not.
def per_box_errors(out, ref, rhs, sub, overlap):
    """[(subdomain, ||out - ref||_2 on its owned block / ||S^gamma rhs||_2)]."""
    _, nz, ny, nx = rhs.shape
    errs = []
    for idx, s in enumerate(ras.subdomains(nx, ny, nz, sub, overlap)):
        (x0, x1), (y0, y1), (z0, z1) = s["own"]
        (bx0, bx1), (by0, by1), (bz0, bz1) = s["box"]
        rin = np.linalg.norm(yee.from_padded(rhs[:, bz0:bz1, by0:by1, bx0:bx1]))
        d = out[:, z0:z1, y0:y1, x0:x1] - ref[:, z0:z1, y0:y1, x0:x1]
        errs.append((idx, np.linalg.norm(d.ravel()) / max(rin, 1e-300)))
    return errs


@pytest.mark.parametrize("n,sub,blk,overlap", [
    (12, 4, 4, 1),                     # size class 8: boxes {5, 6}
    (21, 7, 3, 1),                     # odd sides {8, 9}: classes 8 and 16
    (48, 16, 8, 1),                    # size class 24
    (96, 32, 8, 3),                    # size class 40
    (84, 42, 4, 3),                    # size class 48
])
@pytest.mark.parametrize("precision,u", [("fp32", 2.0**-24), ("bf16", 2.0**-8)])
def test_precond_reduced_precision_error_bound(precision, u, n, sub, blk, overlap):
    P = problem(n, sub, 2.0, blk, seed=7)
    h = handle_for(P, precision=precision, overlap=overlap)
    z = h.new_vector()
    h.apply_precond(dev(P["rhs"]), z)
    ref = ras.ras_apply(P["rhs"], 2.0, P["sub"], overlap, eps_cell_of(P))
    out = host(z, ref.shape)
    errs = per_box_errors(out, ref, P["rhs"], P["sub"], overlap)
    worst = max(errs, key=lambda e: e[1])
    print(f"{precision} n={n} sub={sub} overlap={overlap}: worst box {worst[0]} error "
          f"{worst[1]:.3e} (bound {12 * u:.3e}), whole vector {rel2(out, ref):.3e}")
    assert worst[1] < 12 * u, worst
    assert np.all(out[~inputs.unknown_slots(n, n, n)] == 0.0)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fgmres_with_reduced_precision_preconditioner(precision):
    """FP64 FGMRES stays exact to its tolerance with a reduced-precision preconditioner."""
    P = problem(32, 16, 2.0, 8, seed=2)
    A, Af, Mf = _oracle_ops(P)
    _, io = krylov.fgmres(Af, P["rhs"], M=Mf, tol=1e-8)
    h = handle_for(P, precision=precision)
    x = h.new_vector()
    info = h.solve(dev(P["rhs"]), x, solver="fgmres", rtol=1e-8, max_iter=300)
    assert info["status"] == "FMP_OK" and info["rel_residual_true"] <= 1e-8
    xs = host(x, P["rhs"].shape)
    res = np.linalg.norm(yee.from_padded(P["rhs"]) - A @ yee.from_padded(xs)) / np.linalg.norm(P["rhs"])
    assert res <= 1.5e-8
    assert info["iterations"] <= io["iterations"] + 3


@pytest.mark.parametrize("solver,restart,per_it", [("bicgstab", 30, 2), ("fgmres", 30, 1),
                                                    ("fgmres", 5, 1)])
def test_table3_operation_counts(solver, restart, per_it):
    """Table III: BiCGSTAB applies the preconditioner and the operator twice per
    iteration, GMRES once each.  Besides those, the device solver applies the
    operator for the initial residual and for the true residual recomputed at
    BiCGSTAB's convergence check or at the end of every GMRES cycle.  The
    oracle's drivers, with counting wrappers, do the same work (plus one last
    operator apply for the residual they report)."""
    import functools
    P = problem(32, 16, 2.0, 8, seed=2)
    _, Af, Mf = _oracle_ops(P)
    calls = dict(A=0, M=0)

    def Ac(v):
        calls["A"] += 1
        return Af(v)

    def Mc(v):
        calls["M"] += 1
        return Mf(v)
    run = krylov.bicgstab if solver == "bicgstab" else functools.partial(krylov.fgmres,
                                                                         restart=restart)
    _, io = run(Ac, P["rhs"], M=Mc, tol=1e-8, maxiter=300)
    h = handle_for(P)
    x = h.new_vector()
    info = h.solve(dev(P["rhs"]), x, solver=solver, restart=restart, rtol=1e-8, max_iter=300)
    it = info["iterations"]
    assert info["status"] == "FMP_OK" and it >= 5
    assert info["n_precond"] == per_it * it
    extra = 2 if solver == "bicgstab" else 1 + -(-it // restart)
    assert info["n_spmv"] == per_it * it + extra, info
    if io["iterations"] == it:
        assert calls["M"] == info["n_precond"] and calls["A"] - 1 == info["n_spmv"], (calls, info)


def test_precond_batching_and_determinism():
    P = problem(48, 16, 2.0, 8, seed=9)
    r = dev(P["rhs"])
    outs = []
    for bb in (0, 5, 1):
        h = handle_for(P, batch_boxes=bb)
        z = h.new_vector()
        h.apply_precond(r, z)
        outs.append(z.clone())
        z2 = h.new_vector()
        h.apply_precond(r, z2)
        assert torch.equal(z, z2)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_alias_is_rejected():
    P = problem(16, 8, 2.0, 0, seed=1)
    h = handle_for(P)
    r = dev(P["rhs"])
    with pytest.raises(api.FlashMPError, match="ALIAS"):
        h.apply_precond(r, r)
    with pytest.raises(api.FlashMPError, match="ALIAS"):
        h.curlcurl_apply(r, r)


# ------------------------------------------------------------------ solvers
def _oracle_ops(P):
    eps_cell = eps_cell_of(P)
    nx, ny, nz = P["nx"], P["ny"], P["nz"]
    A = yee.assemble_A(nx, ny, nz, P["c"], eps_cell)
    Af = lambda v: yee.to_padded(A @ yee.from_padded(v), nx, ny, nz)
    Mf = lambda v: ras.ras_apply(v, P["c"], P["sub"], 1, eps_cell)
    return A, Af, Mf


@pytest.mark.parametrize("solver", ["bicgstab", "fgmres"])
def test_solve_matches_oracle_iterations(solver):
    P = problem(32, 16, 2.0, 8, seed=2)
    A, Af, Mf = _oracle_ops(P)
    b = P["rhs"]
    if solver == "bicgstab":
        xo, io = krylov.bicgstab(Af, b, M=Mf, tol=1e-8)
    else:
        xo, io = krylov.fgmres(Af, b, M=Mf, tol=1e-8, restart=30)
    h = handle_for(P)
    x = h.new_vector()
    info = h.solve(dev(b), x, solver=solver, rtol=1e-8, max_iter=300, check_every=1)
    assert info["status"] == "FMP_OK"
    assert info["rel_residual_true"] <= 1e-8
    assert abs(info["iterations"] - io["iterations"]) <= 1, (info, io["iterations"])
    xs = host(x, b.shape)
    # the GPU's true residual, recomputed on the CPU
    res = np.linalg.norm(yee.from_padded(b) - A @ yee.from_padded(xs)) / np.linalg.norm(b)
    assert res <= 1.5e-8
    assert relmax(xs, xo) < 1e-6


def test_solve_unpreconditioned_and_restart():
    P = problem(16, 8, 2.0, 4, seed=3)
    A, Af, _ = _oracle_ops(P)
    b = P["rhs"]
    xo, io = krylov.fgmres(Af, b, tol=1e-8, restart=10)
    h = handle_for(P)
    x = h.new_vector()
    info = h.solve(dev(b), x, solver="fgmres", restart=10, precond=False, rtol=1e-8,
                   max_iter=1000)
    assert info["status"] == "FMP_OK"
    assert abs(info["iterations"] - io["iterations"]) <= 2, (info, io["iterations"])


def test_c1_one_exact_solve():
    """16^3 single box, c = 0.5: BiCGSTAB with the exact solve converges in one iteration."""
    P = inputs.make_problem("c1")
    h = handle_for(P)
    b = dev(P["rhs"])
    z = h.new_vector()
    h.apply_precond(b, z)
    ref = yee.to_padded(transforms.box_solve_transform(yee.from_padded(P["rhs"]), 16, 16, 16, 0.5),
                        16, 16, 16)
    assert relmax(host(z, ref.shape), ref) < 1e-12
    x = h.new_vector()
    info = h.solve(b, x, solver="bicgstab", rtol=1e-10, max_iter=10)
    assert info["status"] == "FMP_OK" and info["iterations"] == 1
    assert info["rel_residual_true"] < 1e-10


def test_failure_paths():
    P = problem(16, 8, 2.0, 0, seed=4)
    h = handle_for(P)
    b = dev(P["rhs"])
    x = h.new_vector()
    info = h.solve(b, x, solver="fgmres", rtol=1e-12, max_iter=1)
    assert info["status"] == "FMP_NOT_CONVERGED" and info["iterations"] == 1
    bn = b.clone()
    bn[100] = float("nan")        # E_x slot (i, j, k) = (4, 6, 0): a wall, ignored
    x = h.new_vector()
    info = h.solve(bn, x, solver="bicgstab", rtol=1e-8, max_iter=50)
    assert info["status"] == "FMP_OK"
    bn[(5 * 16 + 5) * 16 + 5] = float("nan")   # E_x unknown at (5, 5, 5)
    x = h.new_vector()
    with pytest.raises(api.FlashMPError, match="BREAKDOWN"):
        h.solve(bn, x, solver="bicgstab", rtol=1e-8, max_iter=5)
    x = h.new_vector()
    with pytest.raises(api.FlashMPError, match="BREAKDOWN"):
        h.solve(bn, x, solver="fgmres", rtol=1e-8, max_iter=5)


# ------------------------------------------------------------------ full-size samples
@pytest.mark.slow
def test_full_256_sampled_stencil_and_precond():
    """256^3, 8^3 subdomains of 32^3, eps U[1,10] on 8^3 cubes, c = 2 (the launch bench.py times)."""
    P = inputs.make_problem("c3")
    n = 256
    eps_cell = eps_cell_of(P)
    h = handle_for(P)
    r = dev(P["rhs"])
    y = h.new_vector()
    z = h.new_vector()
    h.curlcurl_apply(r, y)
    h.apply_precond(r, z)
    yo = host(y, P["rhs"].shape)
    zo = host(z, P["rhs"].shape)
    rng = np.random.default_rng(0)
    pts = [(int(q), int(k), int(j), int(i)) for q, k, j, i in
           zip(rng.integers(0, 3, 150), rng.integers(0, n, 150), rng.integers(0, n, 150),
               rng.integers(0, n, 150))]
    pts += [(0, 1, 1, 0), (1, 255, 0, 255), (2, 0, 255, 255), (0, 255, 255, 255)]
    ref = yee.apply_A_at(P["rhs"], P["c"], eps_cell, pts)
    got = np.array([yo[p] for p in pts])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(P["rhs"]).max()
    # corner, edge, face and interior subdomains (index = (sz*8 + sy)*8 + sx)
    which = [0, 7, 63, 511, 4 * 64 + 3 * 8 + 4, 3 * 64 + 4 * 8 + 5]
    blocks = ras.ras_apply_subset(P["rhs"], P["c"], P["sub"], 1, eps_cell, which)
    for idx, (own, blk) in blocks.items():
        (x0, x1), (y0, y1), (z0, z1) = own
        assert relmax(zo[:, z0:z1, y0:y1, x0:x1], blk) < 1e-12, idx


def test_precond_graph_replay_matches_eager():
    """Captured applies replay bitwise-equal to eager ones, with eager work in between."""
    P = problem(48, 16, 2.0, 8, seed=11)
    r = dev(P["rhs"])
    h0 = handle_for(P)
    ref = h0.new_vector()
    h0.apply_precond(r, ref)
    h = handle_for(P, use_graph=True)
    z = h.new_vector()
    y = h.new_vector()
    for rep in range(4):
        z.fill_(float("nan"))
        h.apply_precond(r, z)            # first call captures, later calls replay
        h.curlcurl_apply(z, y)           # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(z, ref), rep
    x = h.new_vector()
    info = h.solve(r, x, solver="fgmres", rtol=1e-8, max_iter=200)
    assert info["status"] == "FMP_OK"


def test_odd_length_vectors():
    """15^3 grid (odd vector length 10125): tails of the pair-wise vector kernels."""
    P = problem(15, 5, 2.0, 5, seed=13)
    A, Af, Mf = _oracle_ops(P)
    _, io = krylov.fgmres(Af, P["rhs"], M=Mf, tol=1e-8)
    h = handle_for(P)
    assert h.length % 2 == 1
    x = h.new_vector()
    cap = torch.zeros(3, h.length, dtype=torch.float64, device=DEV)   # odd-offset slots
    info = h.solve(dev(P["rhs"]), x, solver="fgmres", rtol=1e-8, max_iter=300, capture=cap)
    assert info["status"] == "FMP_OK" and abs(info["iterations"] - io["iterations"]) <= 1
    xs = host(x, P["rhs"].shape)
    res = np.linalg.norm(yee.from_padded(P["rhs"]) - A @ yee.from_padded(xs)) / np.linalg.norm(P["rhs"])
    assert res <= 1.5e-8
    assert torch.isfinite(cap).all()


def test_batch_of_uneven_domains_matches_oracle():
    """Several independent domains of different sizes and c in one handle (one apply)."""
    rng = np.random.default_rng(21)
    spec = [(24, 24, 1.5), (16, 16, 0.5), (12, 12, 8.0), (48, 24, 3.0)]   # (n, sub, c)
    doms, rhs = [], []
    for n, sub, c in spec:
        doms.append(dict(nx=n, ny=n, nz=n, c=c, sub=sub))
        rhs.append(inputs.normal_rhs(rng, n, n, n))
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5)):
        h = api.Handle(doms, precision=prec, device=DEV)
        r = torch.cat([dev(v) for v in rhs])
        z = h.new_vector()
        h.apply_precond(r, z)
        out = z.cpu().numpy()
        for d, ((n, sub, c), v) in enumerate(zip(spec, rhs)):
            ref = ras.ras_apply(v, c, (sub,) * 3, 1)
            got = out[h.offsets[d]:h.offsets[d + 1]].reshape(ref.shape)
            assert relmax(got, ref) < tol, (prec, d)
    x = h.new_vector()
    info = h.solve(r, x, solver="fgmres", rtol=1e-8, max_iter=300)
    assert info["status"] == "FMP_OK" and info["rel_residual_true"] <= 1e-8


def test_per_domain_fgmres_matches_independent_oracle_solves():
    """Independent FGMRES per domain, run in lockstep: each domain's step count,
    residual and solution match an oracle FGMRES of that domain alone.  The
    15^3 domain has odd length, so the later domains start at odd offsets."""
    spec = [(16, 8, 2.0, 4, 31), (15, 5, 0.5, 5, 32), (12, 12, 8.0, 0, 33), (20, 10, 3.0, 5, 34)]
    doms, probs = [], []
    for n, sub, c, blk, seed in spec:
        P = problem(n, sub, c, blk, seed)
        probs.append(P)
        doms.append(dict(nx=n, ny=n, nz=n, c=c, eps=P["eps"], eps_block=blk, sub=sub))
    h = api.Handle(doms, device=DEV)
    b = torch.cat([dev(P["rhs"]) for P in probs])
    x = h.new_vector()
    info = h.solve(b, x, solver="fgmres", restart=30, rtol=1e-8, max_iter=300, per_domain=True)
    assert info["status"] == "FMP_OK"
    xs = x.cpu().numpy()
    for d, P in enumerate(probs):
        A, Af, Mf = _oracle_ops(P)
        xo, io = krylov.fgmres(Af, P["rhs"], M=Mf, tol=1e-8, restart=30)
        assert abs(info["domain_iterations"][d] - io["iterations"]) <= 1, (d, info, io["iterations"])
        assert info["domain_rel_residual"][d] <= 1e-8
        xd = xs[h.offsets[d]:h.offsets[d + 1]].reshape(P["rhs"].shape)
        res = np.linalg.norm(yee.from_padded(P["rhs"]) - A @ yee.from_padded(xd)) / np.linalg.norm(P["rhs"])
        assert res <= 1.5e-8, d
        assert relmax(xd, xo) < 1e-6, d
    assert info["iterations"] == max(info["domain_iterations"])
    with pytest.raises(api.FlashMPError, match="UNSUPPORTED"):
        h.solve(b, x, solver="bicgstab", rtol=1e-8, per_domain=True)


def test_solve_ignores_wall_slots_of_b_and_x0():
    P = problem(16, 8, 2.0, 4, seed=41)
    h = handle_for(P)
    shape = P["rhs"].shape
    wall = ~yee.wall_mask(16, 16, 16)   # True on PEC-wall slots
    b = P["rhs"].copy()
    assert np.all(b[wall] == 0.0)
    x_clean = h.new_vector()
    i_clean = h.solve(dev(b), x_clean, solver="fgmres", rtol=1e-8)
    rng = np.random.default_rng(5)
    bg = b.copy()
    bg[wall] = rng.normal(size=int(wall.sum())) * 1e3
    x0 = np.zeros(shape)
    x0[wall] = 7.0
    x = dev(x0)
    i_g = h.solve(dev(bg), x, solver="fgmres", rtol=1e-8)
    assert i_g["iterations"] == i_clean["iterations"]
    xs = host(x, shape)
    assert np.all(xs[wall] == 0.0)
    assert np.array_equal(xs, host(x_clean, shape))


def test_autotune_keeps_results_bitwise():
    """fmp_autotune only changes the schedule: z is bit-identical before and after."""
    rng = np.random.default_rng(51)
    spec = [(24, 24, 1.5), (16, 16, 0.5), (12, 12, 8.0), (48, 24, 3.0), (32, 16, 2.0)]
    doms = [dict(nx=n, ny=n, nz=n, c=c, sub=sub) for n, sub, c in spec]
    r = torch.cat([dev(inputs.normal_rhs(rng, n, n, n)) for n, _, _ in spec])
    for prec, graph in (("fp32", True), ("fp64", False)):
        h = api.Handle(doms, precision=prec, device=DEV, batch_boxes=-1, use_graph=graph)
        z0, y0 = h.new_vector(), h.new_vector()
        h.apply_precond(r, z0)
        h.curlcurl_apply(r, y0)
        tune = h.autotune(r, h.new_vector())
        plans = [t for t in tune if t["stencil_ty"] == 0]
        tiles = [t for t in tune if t["stencil_ty"] > 0]
        assert sum(t["chosen"] for t in plans) == 1 and all(t["apply_ms"] > 0 for t in tune)
        assert {t["streams"] for t in plans} == {1, 2}
        assert {t["slab_order"] for t in plans} == {0, 1}
        assert sorted(t["stencil_ty"] for t in tiles) == [4, 8, 16]
        assert sum(t["chosen"] for t in tiles) == 1 and not any(t["cached"] for t in tune)
        z1, y1 = h.new_vector(), h.new_vector()
        h.apply_precond(r, z1)
        h.curlcurl_apply(r, y1)
        assert torch.equal(z0, z1), prec
        assert torch.equal(y0, y1), prec
    h = api.Handle(doms[:1], device=DEV)
    with pytest.raises(api.FlashMPError, match="UNSUPPORTED"):
        h.autotune(r[:h.length].contiguous())


@pytest.mark.parametrize("blk", [0, 4])
def test_stencil_tile_heights_agree_bitwise(blk):
    """The 64 x 4, 8 and 16 stencil tiles compute the same y bit for bit,
    with and without a permittivity table (each tile height is made current
    in turn through the plan cache)."""
    import os
    import tempfile
    nx, ny, nz = 70, 37, 21                          # ragged against every tile height
    P = inputs.make_problem(dict(n=(nx, ny, nz), sub=0, c=2.0, eps_block=blk, seed=9))
    x = dev(P["rhs"])
    dom = dict(nx=nx, ny=ny, nz=nz, c=2.0, sub=(0, 0, 0))
    eps_cell = None
    if blk:
        dom.update(eps=P["eps"], eps_block=blk)
        eps_cell = yee.expand_eps(P["eps"], blk, nx, ny, nz)
    ref = yee.apply_A_padded(P["rhs"], 2.0, eps_cell)
    outs = []
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "plans.txt")
        old = os.environ.get("FMP_TUNE_CACHE")
        os.environ["FMP_TUNE_CACHE"] = path
        try:
            h = api.Handle([dom], device=DEV, batch_boxes=-1)
            tune = h.autotune(x, h.new_vector())
            key, b, ns, so, ty = open(path).read().split()
            for t in (4, 8, 16):                     # rewrite the record, re-tune from it
                with open(path, "w") as f:
                    f.write(f"{key} {b} {ns} {so} {t}\n")
                hit = h.autotune(x, h.new_vector())
                assert all(e["cached"] for e in hit)
                assert [e["stencil_ty"] for e in hit if e["stencil_ty"]] == [t]
                y = h.new_vector()
                h.curlcurl_apply(x, y)
                outs.append(host(y, ref.shape))
            h.close()
        finally:
            if old is None:
                del os.environ["FMP_TUNE_CACHE"]
            else:
                os.environ["FMP_TUNE_CACHE"] = old
    assert any(e["chosen"] and e["stencil_ty"] for e in tune)
    for o in outs:
        assert np.array_equal(o, outs[0])
        assert np.abs(o - ref).max() <= 1e-13 * np.abs(ref).max()


def test_autotune_plan_cache_round_trip():
    """FMP_TUNE_CACHE: the first tuning appends a record, a second handle of the same
    problem takes the recorded plan without timing the candidates."""
    import os
    import tempfile
    spec = [(24, 12, 1.5), (16, 8, 0.5)]
    doms = [dict(nx=n, ny=n, nz=n, c=c, sub=sub) for n, sub, c in spec]
    rng = np.random.default_rng(5)
    r = torch.cat([dev(inputs.normal_rhs(rng, n, n, n)) for n, _, _ in spec])
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "plans.txt")
        old = os.environ.get("FMP_TUNE_CACHE")
        os.environ["FMP_TUNE_CACHE"] = path
        try:
            h1 = api.Handle(doms, device=DEV, batch_boxes=-1)
            t1 = h1.autotune(r, h1.new_vector())
            assert not any(e["cached"] for e in t1) and len(open(path).readlines()) == 1
            h2 = api.Handle(doms, device=DEV, batch_boxes=-1)
            t2 = h2.autotune(r, h2.new_vector())
            assert len(t2) == 2 and all(e["cached"] and e["chosen"] for e in t2)
            pick = lambda t: sorted((e["batch_boxes"], e["streams"], e["slab_order"], e["stencil_ty"])
                                    for e in t if e["chosen"])
            assert pick(t1) == pick(t2)
            z1, z2 = h1.new_vector(), h2.new_vector()
            h1.apply_precond(r, z1)
            h2.apply_precond(r, z2)
            assert torch.equal(z1, z2)
            # a different problem does not match the record
            h3 = api.Handle(doms[:1], device=DEV, batch_boxes=-1)
            t3 = h3.autotune(r[:h3.length].contiguous(), h3.new_vector())
            assert not any(e["cached"] for e in t3) and len(open(path).readlines()) == 2
        finally:
            if old is None:
                del os.environ["FMP_TUNE_CACHE"]
            else:
                os.environ["FMP_TUNE_CACHE"] = old


@pytest.mark.slow
@pytest.mark.parametrize("precision,u", [("fp32", 2.0**-24), ("bf16", 2.0**-8)])
def test_full_256_sampled_reduced_precision(precision, u):
    """256^3 C3 workload with FP32 / BF16 transforms: sampled subdomain blocks
    (corner, edge, face, interior) within the 12u bound of the smaller cases."""
    P = inputs.make_problem("c3")
    eps_cell = eps_cell_of(P)
    h = handle_for(P, precision=precision)
    z = h.new_vector()
    h.apply_precond(dev(P["rhs"]), z)
    zo = host(z, P["rhs"].shape)
    which = [0, 7, 63, 511, 4 * 64 + 3 * 8 + 4]
    blocks = ras.ras_apply_subset(P["rhs"], P["c"], P["sub"], 1, eps_cell, which)
    subs = ras.subdomains(256, 256, 256, P["sub"], 1)
    for idx, (own, blk) in blocks.items():
        (x0, x1), (y0, y1), (z0, z1) = own
        (bx0, bx1), (by0, by1), (bz0, bz1) = subs[idx]["box"]
        rin = np.linalg.norm(yee.from_padded(P["rhs"][:, bz0:bz1, by0:by1, bx0:bx1]))
        err = np.linalg.norm((zo[:, z0:z1, y0:y1, x0:x1] - blk).ravel()) / rin
        assert err < 12 * u, (idx, err)


@pytest.mark.parametrize("precision,tol,iters", [("fp64", 1e-13, 1), ("fp32", 1e-5, 2),
                                                  ("bf16", 5e-2, 5)])
def test_degenerate_c_zero_is_identity(precision, tol, iters):
    """c = 0: A = I and every box solve is a forward then an inverse orthonormal
    transform, so M^-1 r = r on the unknowns up to the transform's rounding and
    BiCGSTAB stops within a step or two; a Crank-Nicolson step with
    dt = 2 sqrt(c) = 0 starts from a zero residual and leaves E and the H
    unknowns unchanged, with zeros written on the H wall slots."""
    n, sub = 24, 8
    r = inputs.normal_rhs(np.random.default_rng(21), n, n, n)
    h = api.Handle([dict(nx=n, ny=n, nz=n, c=0.0, sub=(sub, sub, sub))], precision=precision,
                   device=DEV)
    z = h.new_vector()
    h.apply_precond(dev(r), z)
    assert np.abs(host(z, r.shape) - r).max() <= tol * np.abs(r).max()
    x = h.new_vector()
    info = h.solve(dev(r), x, solver="bicgstab", rtol=1e-8, max_iter=20)
    assert info["status"] == "FMP_OK" and info["iterations"] <= iters, info
    if precision == "fp64":
        E, H = dev(r), dev(r[::-1].copy() * 0.5)
        E0, H0 = E.clone(), H.clone()
        h.cn_step(E, H, solver="bicgstab", rtol=1e-12, max_iter=20)
        torch.cuda.synchronize()
        assert torch.equal(E, E0)
        from oracle import fdtd
        mask = torch.from_numpy(fdtd.h_mask(n, n, n).ravel()).to(DEV)
        assert torch.equal(H[mask], H0[mask]) and float(H[~mask].abs().max()) == 0.0
