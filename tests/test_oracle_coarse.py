"""Pins of the learned-correction oracle: gradients by finite differences,
restriction/prolongation identities, Adam's first step, bf16 rounding."""
import numpy as np
import pytest
import torch

from oracle import coarse
from paper_2508_07193_amd import inputs


def _params(n_in, hidden, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(coarse.n_params(n_in, hidden)) * 0.5


def test_backward_matches_central_differences():
    n_in, hidden, batch = 6, 5, 4
    rng = np.random.default_rng(1)
    p = _params(n_in, hidden)
    X = rng.standard_normal((batch, n_in))
    Y = rng.standard_normal((batch, n_in))
    _, g = coarse.loss_grad(p, X, Y, n_in, hidden)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (coarse.loss_grad(p + e, X, Y, n_in, hidden)[0] -
                 coarse.loss_grad(p - e, X, Y, n_in, hidden)[0]) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_forward_small_case_by_hand():
    """One input, hidden 1: O = W3 relu(W2 relu(W1 x + b1) + b2) + b3."""
    n_in, hidden = 1, 1
    p = np.array([2.0, -1.0, 3.0, 0.5, -2.0, 0.25])   # W1 b1 W2 b2 W3 b3
    O, _ = coarse.forward(p, np.array([[1.5]]), n_in, hidden)
    h1 = max(2.0 * 1.5 - 1.0, 0.0)
    h2 = max(3.0 * h1 + 0.5, 0.0)
    assert O[0, 0] == -2.0 * h2 + 0.25


def test_restrict_prolong_identities():
    n, sub = 16, (8, 8, 8)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(3 * 8)
    z = coarse.prolong(y, (3, n, n, n), sub)
    assert np.allclose(coarse.restrict(z, sub), y, rtol=0, atol=1e-15)
    assert np.all(z[~inputs.unknown_slots(n, n, n)] == 0)
    # a field equal to 1 on every unknown averages to 1 everywhere
    ones = inputs.unknown_slots(n, n, n).astype(float)
    assert np.allclose(coarse.restrict(ones, sub), 1.0)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = coarse.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 1e-2)
    np.testing.assert_allclose(p, -1e-2 * np.sign(g), rtol=1e-4)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(3).standard_normal(10000).astype(np.float32) * 7
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(coarse.bf16_round(x), ref)


@pytest.mark.slow
def test_ideal_coarse_correction_bounds_the_learned_gain():
    """Upper bound on what any coarse correction through P0 can gain.

    The learned part adds P0 MLP(R0 r) to the RAS step; the best any network
    can do is the exact restricted remaining error, z = M r + P0 R0 (A^-1 r -
    M r).  Beside that additive ideal, the coarse spaces of the same shape
    that domain decomposition would use are tried: the Galerkin coarse solve
    y = (P0^T A P0)^{-1} P0^T r added to the RAS step, the same coarse step
    composed multiplicatively (z = P0 y + M (r - A P0 y), the residual
    corrected before the RAS step), and the multiplicative form with the
    prolongation weighted by 1 / diag(A) (eps-aware).  On a 24^3 grid with
    8^3 subdomains and c = 8, with eps = 1 the multiplicative coarse step and
    the ideal correction save iterations; with eps_r U[1,10] on 4^3-cell
    cubes inside each subdomain none of them saves more than one: the RAS
    error there is the constant-coefficient box solve's mismatch inside the
    subdomains, which piecewise-constant coarse functions do not capture.
    """
    import scipy.sparse.linalg as spla
    from oracle import krylov, ras, yee
    n, sub, c = 24, (8, 8, 8), 8.0
    nsub = 27
    out = {}
    for name, blk in (("uniform", 0), ("contrast", 4)):
        P = inputs.make_problem(dict(n=n, sub=8, c=c, eps_block=blk, seed=3))
        shape = P["rhs"].shape
        eps_cell = yee.expand_eps(P["eps"], blk, n, n, n) if blk else None
        A = yee.assemble_A(n, n, n, c, eps_cell).tocsc()
        lu = spla.splu(A)
        Af = lambda v: yee.to_padded(A @ yee.from_padded(v), n, n, n)
        Mf = lambda v: ras.ras_apply(v, c, sub, 1, eps_cell)
        Ainv = lambda v: yee.to_padded(lu.solve(yee.from_padded(v)), n, n, n)
        ideal = lambda v: Mf(v) + coarse.prolong(coarse.restrict(Ainv(v) - Mf(v), sub), v.shape, sub)
        P0 = np.stack([coarse.prolong(np.eye(3 * nsub)[i], shape, sub).ravel()
                       for i in range(3 * nsub)], 1)
        wdiag = yee.to_padded(1.0 / A.diagonal(), n, n, n).ravel()

        def galerkin(Pm, mult):
            APm = np.stack([Af(Pm[:, i].reshape(shape)).ravel() for i in range(Pm.shape[1])], 1)
            Ac = Pm.T @ APm

            def M(v):
                Py = (Pm @ np.linalg.solve(Ac, Pm.T @ v.ravel())).reshape(shape)
                return Py + Mf(v - Af(Py)) if mult else Mf(v) + Py
            return M

        forms = dict(plain=Mf, ideal_additive=ideal, galerkin_additive=galerkin(P0, False),
                     galerkin_multiplicative=galerkin(P0, True),
                     eps_weighted_multiplicative=galerkin(P0 * wdiag[:, None], True))
        out[name] = {k: krylov.fgmres(Af, P["rhs"], M=M, tol=1e-8, restart=30)[1]["iterations"]
                     for k, M in forms.items()}
    print(out)
    u, k = out["uniform"], out["contrast"]
    assert u["ideal_additive"] <= u["plain"] - 2, out
    assert u["galerkin_multiplicative"] <= u["plain"] - 2, out
    for form in ("ideal_additive", "galerkin_additive", "galerkin_multiplicative",
                 "eps_weighted_multiplicative"):
        assert k[form] >= k["plain"] - 1, (form, out)
