"""Pins of the CN-FDTD oracle (Sec. II-A, eqs. (2)-(5)) against facts that do
not come from the oracle itself:

* the discrete curl annihilates discrete gradients (curl grad = 0 on the Yee
  grid, exact in integers), so a gradient field is a steady state;
* a cavity eigenmode of the PEC box (a transverse wavenumber of the closed-form
  DCT-II/DST-I diagonalisation, eigenvalue sigma_p^2 + sigma_q^2 + sigma_r^2)
  turns by the Crank-Nicolson angle theta = 2 atan(dt sqrt(lambda) / 2) per
  step, E_n = cos(n theta) E_0 and H_n = -sin(n theta) C E_0 / sqrt(lambda);
* Crank-Nicolson conserves the discrete energy (1/2)(E^T eps E + H^T H)
  exactly for any permittivity.
"""
import numpy as np

from oracle import fdtd, transforms, yee


def gradient_field(phi):
    """Padded E = grad phi for node values phi (nz+1, ny+1, nx+1) that vanish on the walls."""
    nz, ny, nx = (s - 1 for s in phi.shape)
    v = np.zeros((3, nz, ny, nx))
    v[0] = (phi[:-1, :-1, 1:] - phi[:-1, :-1, :-1])
    v[1] = (phi[:-1, 1:, :-1] - phi[:-1, :-1, :-1])
    v[2] = (phi[1:, :-1, :-1] - phi[:-1, :-1, :-1])
    return v * yee.wall_mask(nx, ny, nz)


def random_phi(rng, nx, ny, nz, integers=False):
    phi = np.zeros((nz + 1, ny + 1, nx + 1))
    inner = (nz - 1, ny - 1, nx - 1)
    phi[1:-1, 1:-1, 1:-1] = rng.integers(-9, 10, inner) if integers else rng.standard_normal(inner)
    return phi


def test_curl_of_gradient_vanishes():
    nx, ny, nz = 5, 4, 6
    phi = random_phi(np.random.default_rng(0), nx, ny, nz, integers=True)
    E = yee.from_padded(gradient_field(phi))
    assert np.any(E != 0)
    C = yee.curl_matrix(nx, ny, nz)
    assert np.array_equal(C @ E, np.zeros(C.shape[0]))


def test_padded_h_layout():
    nx, ny, nz = 4, 3, 5
    C = yee.curl_matrix(nx, ny, nz)
    assert fdtd.h_mask(nx, ny, nz).sum() == C.shape[0]
    u = np.arange(C.shape[0], dtype=float) + 1.0
    v = fdtd.h_to_padded(u, nx, ny, nz)
    assert np.array_equal(fdtd.h_from_padded(v), u)
    assert np.all(v[~fdtd.h_mask(nx, ny, nz)] == 0.0)


def test_gradient_field_is_stationary():
    nx, ny, nz, c = 6, 5, 4, 2.0
    rng = np.random.default_rng(1)
    eps = rng.uniform(1.0, 10.0, (nz, ny, nx))
    E0 = yee.from_padded(gradient_field(random_phi(rng, nx, ny, nz)))
    H0 = np.zeros(yee.curl_matrix(nx, ny, nz).shape[0])
    E1, H1 = fdtd.cn_step(E0, H0, nx, ny, nz, c, eps)
    assert np.abs(E1 - E0).max() <= 1e-12 * np.abs(E0).max()
    assert np.abs(H1).max() <= 1e-12 * np.abs(E0).max()


def test_cavity_mode_turns_by_the_cn_angle():
    nx, ny, nz, c = 7, 6, 5, 0.8
    p, q, r = 2, 3, 1                                   # wavenumber (all transverse modes >= 1)
    s = np.array([transforms.sigma(nx)[p], transforms.sigma(ny)[q], transforms.sigma(nz)[r]])
    lam = float(s @ s)
    e = np.cross(s, [0.3, -1.0, 0.7])                   # any direction orthogonal to s
    spec = np.zeros((3, nz, ny, nx))
    spec[:, r, q, p] = e
    E0 = transforms.inverse_G(spec, nx, ny, nz)
    E0 /= np.linalg.norm(E0)
    C = yee.curl_matrix(nx, ny, nz)
    K = (C.T @ C)
    assert np.abs(K @ E0 - lam * E0).max() < 1e-12    # it is an eigenmode
    dt = fdtd.time_step(c)
    theta = 2.0 * np.arctan(dt * np.sqrt(lam) / 2.0)
    E, H = E0.copy(), np.zeros(C.shape[0])
    for n in range(1, 6):
        E, H = fdtd.cn_step(E, H, nx, ny, nz, c)
        assert np.abs(E - np.cos(n * theta) * E0).max() < 1e-12
        assert np.abs(H + np.sin(n * theta) * (C @ E0) / np.sqrt(lam)).max() < 1e-12


def test_energy_is_conserved_with_permittivity():
    nx, ny, nz, c = 8, 6, 7, 3.0
    rng = np.random.default_rng(2)
    eps = yee.expand_eps(rng.uniform(1.0, 10.0, (4, 3, 4)), 2, nx, ny, nz)
    E = rng.standard_normal(yee.n_unknowns(nx, ny, nz))
    H = rng.standard_normal(yee.curl_matrix(nx, ny, nz).shape[0])
    eps_e = yee.edge_eps(eps)
    W0 = fdtd.energy(E, H, eps_e)
    for _ in range(4):
        E, H = fdtd.cn_step(E, H, nx, ny, nz, c, eps)
        assert abs(fdtd.energy(E, H, eps_e) - W0) <= 1e-11 * W0


def test_windowed_curls_match_the_assembled_operator():
    nx, ny, nz = 9, 7, 8
    rng = np.random.default_rng(3)
    eps = rng.uniform(1.0, 10.0, (nz, ny, nx))
    C = yee.curl_matrix(nx, ny, nz)
    e = rng.standard_normal(yee.n_unknowns(nx, ny, nz))
    hv = rng.standard_normal(C.shape[0])
    ep, hp = yee.to_padded(e, nx, ny, nz), fdtd.h_to_padded(hv, nx, ny, nz)
    Hf = fdtd.h_to_padded(C @ e, nx, ny, nz)
    Ef = yee.to_padded(C.T @ hv, nx, ny, nz)
    Ee = yee.to_padded(yee.edge_eps(eps), nx, ny, nz)
    def sample(mask):
        # every slot on a wall-adjacent layer, plus a seeded sample of the rest
        pts = np.argwhere(mask)
        edge = np.any((pts[:, 1:] <= 1) | (pts[:, 1:] >= np.array([nz, ny, nx]) - 2), axis=1)
        rest = pts[~edge][rng.choice(int((~edge).sum()), 60, replace=False)]
        return [tuple(int(v) for v in p) for p in np.concatenate([pts[edge][::3], rest])]
    hpts = sample(fdtd.h_mask(nx, ny, nz))
    epts = sample(yee.wall_mask(nx, ny, nz))
    got = fdtd.curl_e_at(ep, hpts)
    assert np.abs(got - np.array([Hf[p] for p in hpts])).max() < 1e-13
    ct, ee = fdtd.curl_h_at(hp, eps, epts)
    assert np.abs(ct - np.array([Ef[p] for p in epts])).max() < 1e-13
    assert np.abs(ee - np.array([Ee[p] for p in epts])).max() < 1e-14
