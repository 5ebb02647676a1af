"""Thin Python binding of the FlashMP C ABI (argument marshalling only).

Every step of the solver runs inside libflashmp.so; PyTorch only provides
device memory (workspaces, vectors) and the current stream.  Vectors are
float64 CUDA tensors in the padded layout of include/flashmp.h.
"""
import ctypes as C

import numpy as np
import torch

from . import _lib


class FlashMPError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        name = _lib.STATUS.get(status, str(status))
        super().__init__(f"{where}: {name}{(' - ' + detail) if detail else ''}")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _check(st, where, h=None, ok=(0,)):
    if st in ok:
        return st
    detail = ""
    if h is not None and h.value:
        detail = _lib.load().fmp_last_error(h).decode()
    raise FlashMPError(st, where, detail)


def domain_desc(nx, ny, nz, c, eps=None, eps_block=0, sub=(0, 0, 0)):
    """Build an fmp_domain_desc; `eps` is the (ceil(nz/b), ceil(ny/b), ceil(nx/b))
    permittivity table or None."""
    d = _lib.DomainDesc()
    d.nx, d.ny, d.nz, d.c = int(nx), int(ny), int(nz), float(c)
    sub = (sub, sub, sub) if np.isscalar(sub) else tuple(sub)
    d.sub_x, d.sub_y, d.sub_z = (int(s) for s in sub)
    keep = None
    if eps is not None:
        keep = np.ascontiguousarray(eps, dtype=np.float64)
        b = int(eps_block)
        want = tuple(-(-int(n) // b) for n in (nz, ny, nx)) if b > 0 else None
        if want is None or keep.shape != want:
            raise ValueError(f"eps table of shape {keep.shape} for a {nx}x{ny}x{nz} domain "
                             f"with eps_block={eps_block}: expected {want}")
        d.eps_block = keep.ctypes.data_as(C.POINTER(C.c_double))
        d.eps_block_size = int(eps_block)
    else:
        d.eps_block = None
        d.eps_block_size = 0
    return d, keep


class Handle:
    """A set of domains with their RAS plans (fmp_setup_subdomains) and workspace."""

    def __init__(self, domains, overlap=1, precision="fp64", use_learned=False, batch_boxes=0,
                 use_graph=False, device="cuda", stream=None, subdomain="pec"):
        L = _lib.load()
        keep = []
        arr = (_lib.DomainDesc * len(domains))()
        for i, dom in enumerate(domains):
            d, k = domain_desc(**dom)
            arr[i] = d
            keep.append(k)
        pd = _lib.PrecondDesc(int(overlap), _lib.PRECISION[precision], int(bool(use_learned)),
                              int(batch_boxes), int(bool(use_graph)), _lib.SUBDOMAIN[subdomain])
        nbytes = C.c_size_t(0)
        h = C.c_void_p()
        s = _stream(stream)
        _check(L.fmp_setup_subdomains(arr, len(domains), C.byref(pd), None, C.byref(nbytes), s,
                                      C.byref(h)), "fmp_setup_subdomains(size)")
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        _check(L.fmp_setup_subdomains(arr, len(domains), C.byref(pd), _ptr(self.ws),
                                      C.byref(nbytes), s, C.byref(h)), "fmp_setup_subdomains")
        self.h = h
        self.n_domains = len(domains)
        self.precision = precision
        self.device = device
        offs = (C.c_int64 * (len(domains) + 1))()
        _check(L.fmp_vector_layout(h, offs), "fmp_vector_layout", h)
        self.offsets = [int(o) for o in offs]
        self.length = self.offsets[-1]
        self._solve_ws = None
        self._cn_ws = None

    def close(self):
        if self.h is not None and self.h.value:
            _lib.load().fmp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_vector(self):
        return torch.zeros(self.length, dtype=torch.float64, device=self.device)

    def autotune(self, r=None, z=None, stream=None):
        return fmp_autotune(self, r, z, stream)

    def curlcurl_apply(self, x, y, stream=None):
        return fmp_curlcurl_apply(self, x, y, stream)

    def apply_precond(self, r, z, stream=None):
        return fmp_apply_precond(self, r, z, stream)

    def solve(self, b, x, **kw):
        return fmp_solve(self, b, x, **kw)

    def curl_e(self, e1, h_out, e2=None, h_in=None, beta=0.0, m=1.0, stream=None):
        return fmp_curl_e(self, e1, h_out, e2, h_in, beta, m, stream)

    def curl_h(self, hf, e_out, e_in=None, m=1.0, stream=None):
        return fmp_curl_h(self, hf, e_out, e_in, m, stream)

    def cn_step(self, E, H, **kw):
        return fmp_cn_step(self, E, H, **kw)


def fmp_setup_subdomains(domains, **kw):
    return Handle(domains, **kw)


def fmp_curlcurl_apply(h, x, y, stream=None):
    _check(_lib.load().fmp_curlcurl_apply(h.h, _ptr(x), _ptr(y), _stream(stream)),
           "fmp_curlcurl_apply", h.h)


def fmp_apply_precond(h, r, z, stream=None):
    _check(_lib.load().fmp_apply_precond(h.h, _ptr(r), _ptr(z), _stream(stream)),
           "fmp_apply_precond", h.h)


def fmp_autotune(h, r=None, z=None, stream=None):
    """Time the candidate launch plans of the preconditioner and keep the fastest.

    r defaults to a seeded N(0,1) vector; returns the measured candidates."""
    if r is None:
        g = torch.Generator(device="cpu").manual_seed(0)
        r = torch.randn(h.length, generator=g, dtype=torch.float64).to(h.device)
    if z is None:
        z = h.new_vector()
    ent = (_lib.TuneEntry * 64)()
    n = C.c_int32(0)
    _check(_lib.load().fmp_autotune(h.h, _ptr(r), _ptr(z), ent, 64, C.byref(n), _stream(stream)),
           "fmp_autotune", h.h)
    return [dict(batch_boxes=e.batch_boxes, streams=e.streams, slab_order=e.slab_order,
                 apply_ms=e.apply_ms, chosen=bool(e.chosen), stencil_ty=e.stencil_ty,
                 cached=bool(e.cached)) for e in ent[:n.value]]


def solve_opts(solver="fgmres", restart=30, max_iter=500, rtol=1e-8, precond=True, check_every=1,
               capture=None, profile=False, per_domain=False):
    o = _lib.SolveOpts({"bicgstab": 0, "fgmres": 1}[solver], int(restart), int(max_iter),
                       float(rtol), int(bool(precond)), int(check_every), 0, None,
                       int(bool(profile)), int(bool(per_domain)), None, None)
    if capture is not None:   # (count, length) float64 CUDA tensor receiving x_1 .. x_count
        o.capture_count = int(capture.shape[0])
        o.capture = C.c_void_p(capture.data_ptr())
    return o


def fmp_solve(h, b, x, stream=None, raise_on_breakdown=True, **kw):
    """Solve A x = b in place of x; returns a dict with the solve statistics."""
    L = _lib.load()
    o = solve_opts(**kw)
    nbytes = C.c_size_t(0)
    _check(L.fmp_solve_workspace(h.h, C.byref(o), C.byref(nbytes)), "fmp_solve_workspace", h.h)
    if h._solve_ws is None or h._solve_ws.numel() < nbytes.value:
        h._solve_ws = None
        h._solve_ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=h.device)
    info = _lib.SolveInfo()
    nd = len(h.offsets) - 1
    dom_it = (C.c_int32 * nd)()
    dom_rel = (C.c_double * nd)()
    o.domain_iterations = C.cast(dom_it, C.POINTER(C.c_int32))
    o.domain_rel_residual = C.cast(dom_rel, C.POINTER(C.c_double))
    st = L.fmp_solve(h.h, _ptr(b), _ptr(x), C.byref(o), _ptr(h._solve_ws), nbytes.value,
                     C.byref(info), _stream(stream))
    ok = (0, 1) if raise_on_breakdown else (0, 1, -5)
    _check(st, "fmp_solve", h.h, ok=ok)
    out = dict(status=_lib.STATUS[st], iterations=info.iterations, n_precond=info.n_precond,
               n_spmv=info.n_spmv, used_fallback=info.used_fallback,
               rel_residual_true=info.rel_residual_true, t_total_ms=info.t_total_ms,
               domain_iterations=list(dom_it), domain_rel_residual=list(dom_rel))
    if o.profile:
        out.update(t_precond_ms=info.t_precond_ms, t_spmv_ms=info.t_spmv_ms,
                   t_orth_dot_ms=info.t_orth_dot_ms, t_orth_update_ms=info.t_orth_update_ms,
                   bytes_orth_dot=info.bytes_orth_dot, bytes_orth_update=info.bytes_orth_update,
                   n_orth_dot=info.n_orth_dot, n_orth_update=info.n_orth_update)
    return out


def fmp_curl_e(h, e1, h_out, e2=None, h_in=None, beta=0.0, m=1.0, stream=None):
    """h_out = beta h_in + m dt C (e1 + e2) per domain, dt = 2 sqrt(c)."""
    _check(_lib.load().fmp_curl_e(h.h, _ptr(e1), _ptr(e2) if e2 is not None else None,
                                  _ptr(h_in) if h_in is not None else None, float(beta), float(m),
                                  _ptr(h_out), _stream(stream)), "fmp_curl_e", h.h)


def fmp_curl_h(h, hf, e_out, e_in=None, m=1.0, stream=None):
    """e_out = e_in + m dt eps_e^-1 C^T hf per domain, dt = 2 sqrt(c)."""
    _check(_lib.load().fmp_curl_h(h.h, _ptr(hf), _ptr(e_in) if e_in is not None else None,
                                  float(m), _ptr(e_out), _stream(stream)), "fmp_curl_h", h.h)


def fmp_cn_step(h, E, H, stream=None, **kw):
    """One Crank-Nicolson step of (E, H) in place; returns the solve's statistics."""
    L = _lib.load()
    o = solve_opts(**kw)
    nbytes = C.c_size_t(0)
    _check(L.fmp_cn_workspace(h.h, C.byref(o), C.byref(nbytes)), "fmp_cn_workspace", h.h)
    if h._cn_ws is None or h._cn_ws.numel() < nbytes.value:
        h._cn_ws = None
        h._cn_ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=h.device)
    info = _lib.SolveInfo()
    st = L.fmp_cn_step(h.h, _ptr(E), _ptr(H), C.byref(o), _ptr(h._cn_ws), nbytes.value,
                       C.byref(info), _stream(stream))
    _check(st, "fmp_cn_step", h.h, ok=(0, 1))
    return dict(status=_lib.STATUS[st], iterations=info.iterations,
                rel_residual_true=info.rel_residual_true, t_total_ms=info.t_total_ms)


def release_solver_workspace(h):
    h._solve_ws = None


# ---------------------------------------------------------------- learned coarse correction
def fmp_coarse_size(h):
    n = C.c_int32(0)
    _check(_lib.load().fmp_coarse_size(h.h, C.byref(n)), "fmp_coarse_size", h.h)
    return int(n.value)


def fmp_set_coarse_model(h, hidden, params):
    """Upload FP32 parameters (flat, see include/flashmp.h); None disables the correction."""
    L = _lib.load()
    if params is None:
        _check(L.fmp_set_coarse_model(h.h, 0, None, 0), "fmp_set_coarse_model", h.h)
        return
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(L.fmp_set_coarse_model(h.h, int(hidden), p.ctypes.data_as(C.POINTER(C.c_float)),
                                  p.nbytes), "fmp_set_coarse_model", h.h)


def fmp_coarse_restrict(h, r, rc, stream=None):
    _check(_lib.load().fmp_coarse_restrict(h.h, _ptr(r), _ptr(rc), _stream(stream)),
           "fmp_coarse_restrict", h.h)


def fmp_mlp_scratch_bytes(in_dim, hidden, batch):
    return int(_lib.load().fmp_mlp_scratch_bytes(in_dim, hidden, batch))


def fmp_mlp_loss_grad(in_dim, hidden, batch, params, X, Y, grads, loss, scratch, stream=None):
    _check(_lib.load().fmp_mlp_loss_grad(in_dim, hidden, batch, _ptr(params), _ptr(X), _ptr(Y),
                                         _ptr(grads), _ptr(loss), _ptr(scratch), scratch.numel(),
                                         _stream(stream)), "fmp_mlp_loss_grad")


def fmp_mlp_adam(params, grads, m, v, t, lr, stream=None):
    _check(_lib.load().fmp_mlp_adam(params.numel(), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                                    int(t), float(lr), _stream(stream)), "fmp_mlp_adam")


def fmp_mlp_loss_grad_noalloc(in_dim, hidden, batch, params, X, Y, grads, loss, stream=None):
    """fmp_mlp_loss_grad with the library's static device scratch (allocates nothing)."""
    L = _lib.load()
    st = L.fmp_mlp_loss_grad_noalloc(in_dim, hidden, batch, _ptr(params), _ptr(X), _ptr(Y),
                                     _ptr(grads), _ptr(loss), _stream(stream))
    if st != 0:
        raise FlashMPError(st, "fmp_mlp_loss_grad_noalloc", L.fmp_last_error(None).decode())
