"""Seeded synthetic inputs for the FlashMP workloads.

This module only draws random numbers and places them in the padded field
layout; it holds none of the solver's arithmetic, so both the GPU library's
callers and the CPU checks can use it.

Padded layout: an array of shape (3, nz, ny, nx) (components E_x, E_y, E_z,
x fastest).  Slot 0 of each node axis of a component is a PEC wall and stays
zero: E_x has node axes y, z; E_y has x, z; E_z has x, y.

Draw order with ``numpy.random.default_rng(seed)``: the permittivity block
table (C order z, y, x) first, then the right-hand side over the unknown
slots, component by component in C order.
"""
import numpy as np

SIDES_C4 = (24, 32, 48, 64, 96)


def unknown_slots(nx, ny, nz):
    """Boolean padded mask: True where a slot holds an unknown."""
    m = np.zeros((3, nz, ny, nx), dtype=bool)
    m[0, 1:, 1:, :] = True
    m[1, 1:, :, 1:] = True
    m[2, :, 1:, 1:] = True
    return m


def n_unknowns(nx, ny, nz):
    return nx * (ny - 1) * (nz - 1) + (nx - 1) * ny * (nz - 1) + (nx - 1) * (ny - 1) * nz


def normal_rhs(rng, nx, ny, nz):
    """N(0,1) on every unknown slot (component-major, C order), zeros on walls."""
    v = np.zeros((3, nz, ny, nx))
    v[0, 1:, 1:, :] = rng.standard_normal((nz - 1, ny - 1, nx))
    v[1, 1:, :, 1:] = rng.standard_normal((nz - 1, ny, nx - 1))
    v[2, :, 1:, 1:] = rng.standard_normal((nz, ny - 1, nx - 1))
    return v


def eps_table(rng, nx, ny, nz, block, lo=1.0, hi=10.0):
    """Relative permittivity per cube of `block` cells, U[lo, hi], shape
    (ceil(nz/b), ceil(ny/b), ceil(nx/b)): cubes cut by the far walls count whole."""
    return rng.uniform(lo, hi, size=(-(-nz // block), -(-ny // block), -(-nx // block)))


# Single-domain problems: n = cells per side, sub = owned subdomain side (0 = one box),
# c = dt^2/(4 mu eps h^2), eps_block = side of the constant-permittivity cubes (0 = eps 1).
CONFIGS = {
    # 16^3 single PEC box, eps = 1, one exact solve then BiCGSTAB to 1e-10, seed 0
    "c1": dict(n=16, sub=0, c=0.5, eps_block=0, seed=0, solver="bicgstab", tol=1e-10,
               precision="fp64"),
    # 128^3 in 4x4x4 subdomains of 32^3, eps U[1,10] on 8^3 cubes, c = 2, BiCGSTAB to 1e-8
    "c2": dict(n=128, sub=32, c=2.0, eps_block=8, seed=2, solver="bicgstab", tol=1e-8,
               precision="fp64"),
    # 256^3 in 8x8x8 subdomains of 32^3, eps as above, FGMRES(30) to 1e-8
    "c3": dict(n=256, sub=32, c=2.0, eps_block=8, seed=3, solver="fgmres", tol=1e-8,
               precision="fp64"),
    # 256^3, c = 8, learned coarse correction on top of the subdomain preconditioner
    "c5": dict(n=256, sub=32, c=8.0, eps_block=8, seed=5, solver="fgmres", tol=1e-8,
               precision="fp64"),
    # scaled-down copies used by the parity tests
    "c2_small": dict(n=32, sub=16, c=2.0, eps_block=8, seed=2, solver="bicgstab", tol=1e-8,
                     precision="fp64"),
    "c3_small": dict(n=48, sub=16, c=2.0, eps_block=8, seed=3, solver="fgmres", tol=1e-8,
                     precision="fp64"),
}


def make_problem(name_or_cfg, n=None, seed=None):
    """Return dict(nx, ny, nz, sub, c, eps_block, eps (table or None), rhs (padded))."""
    cfg = dict(CONFIGS[name_or_cfg]) if isinstance(name_or_cfg, str) else dict(name_or_cfg)
    if n is not None:
        cfg["n"] = n
    if seed is not None:
        cfg["seed"] = seed
    nn = cfg["n"]
    nx, ny, nz = (nn, nn, nn) if np.isscalar(nn) else tuple(nn)
    rng = np.random.default_rng(cfg["seed"])
    eps = None
    if cfg.get("eps_block", 0):
        eps = eps_table(rng, nx, ny, nz, cfg["eps_block"])
    rhs = normal_rhs(rng, nx, ny, nz)
    sub = cfg.get("sub", 0)
    sub = (sub, sub, sub) if np.isscalar(sub) else tuple(sub)
    out = dict(cfg)
    out.update(nx=nx, ny=ny, nz=nz, sub=sub, eps=eps, rhs=rhs)
    return out


def extra_rhs(nx, ny, nz, seed):
    """A further right-hand side from its own seed (training / held-out draws)."""
    return normal_rhs(np.random.default_rng(seed), nx, ny, nz)


def extra_rhs_device(nx, ny, nz, seed, device):
    """N(0,1) on every unknown slot, zeros on walls, drawn on the device by
    torch's generator for `device` seeded with `seed` (fast draws of many
    training right-hand sides; a different stream from extra_rhs)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    v = torch.randn((3, nz, ny, nx), generator=g, dtype=torch.float64, device=device)
    v[0, 0, :, :] = 0.0
    v[0, :, 0, :] = 0.0
    v[1, 0, :, :] = 0.0
    v[1, :, :, 0] = 0.0
    v[2, :, 0, :] = 0.0
    v[2, :, :, 0] = 0.0
    return v.reshape(-1)


def make_batch_c4(seed=4, n_domains=64, sides=SIDES_C4, c_range=(0.5, 8.0)):
    """64 independent cubic domains: sides uniform over `sides`, c ~ U[0.5, 8], eps = 1.

    Each side L is split into ceil(L/32) equal owned blocks per axis.  Draw
    order: all sides, then all c, then the right-hand sides domain by domain.
    """
    rng = np.random.default_rng(seed)
    L = rng.choice(np.asarray(sides), size=n_domains)
    cs = rng.uniform(c_range[0], c_range[1], size=n_domains)
    doms = []
    for d in range(n_domains):
        n = int(L[d])
        parts = -(-n // 32)
        doms.append(dict(nx=n, ny=n, nz=n, sub=(n // parts,) * 3, c=float(cs[d]),
                         eps=None, rhs=normal_rhs(rng, n, n, n)))
    return doms
