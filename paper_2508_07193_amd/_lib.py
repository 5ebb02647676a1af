"""ctypes declarations of the C ABI in include/flashmp.h (argument marshalling only)."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libflashmp.so")

FMP_OK, FMP_NOT_CONVERGED = 0, 1
STATUS = {0: "FMP_OK", 1: "FMP_NOT_CONVERGED", -1: "FMP_ERR_INVALID_ARG", -2: "FMP_ERR_ALIAS",
          -3: "FMP_ERR_WORKSPACE", -4: "FMP_ERR_HIP", -5: "FMP_ERR_BREAKDOWN",
          -6: "FMP_ERR_UNSUPPORTED"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
SUBDOMAIN = {"pec": 0, "index": 1}

# every symbol include/flashmp.h declares
EXPORTS = ["fmp_setup_subdomains", "fmp_vector_layout", "fmp_curlcurl_apply", "fmp_apply_precond",
           "fmp_autotune", "fmp_solve_workspace", "fmp_solve", "fmp_curl_e", "fmp_curl_h",
           "fmp_cn_workspace", "fmp_cn_step", "fmp_coarse_size", "fmp_set_coarse_model",
           "fmp_coarse_restrict", "fmp_mlp_loss_grad", "fmp_mlp_scratch_bytes", "fmp_mlp_adam",
           "fmp_destroy", "fmp_status_string", "fmp_last_error", "fmp_runtime_version",
           "fmp_mlp_loss_grad_noalloc"]


class DomainDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("c", C.c_double),
                ("eps_block", C.POINTER(C.c_double)), ("eps_block_size", C.c_int32),
                ("sub_x", C.c_int32), ("sub_y", C.c_int32), ("sub_z", C.c_int32)]


class PrecondDesc(C.Structure):
    _fields_ = [("overlap", C.c_int32), ("precision", C.c_int32), ("use_learned", C.c_int32),
                ("batch_boxes", C.c_int32), ("use_graph", C.c_int32), ("subdomain", C.c_int32)]


class TuneEntry(C.Structure):
    _fields_ = [("batch_boxes", C.c_int32), ("streams", C.c_int32), ("slab_order", C.c_int32),
                ("apply_ms", C.c_double), ("chosen", C.c_int32), ("stencil_ty", C.c_int32),
                ("cached", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("rtol", C.c_double), ("precond", C.c_int32), ("check_every", C.c_int32),
                ("capture_count", C.c_int32), ("capture", C.c_void_p), ("profile", C.c_int32),
                ("per_domain", C.c_int32), ("domain_iterations", C.POINTER(C.c_int32)),
                ("domain_rel_residual", C.POINTER(C.c_double))]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_precond", C.c_int32), ("n_spmv", C.c_int32),
                ("used_fallback", C.c_int32), ("rel_residual_true", C.c_double),
                ("t_total_ms", C.c_double), ("t_precond_ms", C.c_double),
                ("t_spmv_ms", C.c_double), ("t_orth_dot_ms", C.c_double),
                ("t_orth_update_ms", C.c_double), ("bytes_orth_dot", C.c_double),
                ("bytes_orth_update", C.c_double), ("n_orth_dot", C.c_int32),
                ("n_orth_update", C.c_int32)]


_lib = None


def load():
    """Load the built library; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2508_07193_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.fmp_setup_subdomains.argtypes = [C.POINTER(DomainDesc), i32, C.POINTER(PrecondDesc), vp,
                                       C.POINTER(sz), vp, C.POINTER(vp)]
    L.fmp_vector_layout.argtypes = [vp, C.POINTER(C.c_int64)]
    L.fmp_curlcurl_apply.argtypes = [vp, vp, vp, vp]
    L.fmp_apply_precond.argtypes = [vp, vp, vp, vp]
    L.fmp_autotune.argtypes = [vp, vp, vp, C.POINTER(TuneEntry), i32, C.POINTER(i32), vp]
    L.fmp_solve_workspace.argtypes = [vp, C.POINTER(SolveOpts), C.POINTER(sz)]
    L.fmp_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), vp, sz, C.POINTER(SolveInfo), vp]
    f8 = C.c_double
    L.fmp_curl_e.argtypes = [vp, vp, vp, vp, f8, f8, vp, vp]
    L.fmp_curl_h.argtypes = [vp, vp, vp, f8, vp, vp]
    L.fmp_cn_workspace.argtypes = [vp, C.POINTER(SolveOpts), C.POINTER(sz)]
    L.fmp_cn_step.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), vp, sz, C.POINTER(SolveInfo), vp]
    L.fmp_coarse_size.argtypes = [vp, C.POINTER(i32)]
    L.fmp_set_coarse_model.argtypes = [vp, i32, C.POINTER(C.c_float), sz]
    L.fmp_coarse_restrict.argtypes = [vp, vp, vp, vp]
    L.fmp_mlp_loss_grad.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fmp_mlp_scratch_bytes.argtypes = [i32, i32, i32]
    L.fmp_mlp_scratch_bytes.restype = sz
    L.fmp_mlp_adam.argtypes = [i32, vp, vp, vp, vp, i32, C.c_float, vp]
    L.fmp_mlp_loss_grad_noalloc.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp]
    L.fmp_destroy.argtypes = [vp]
    L.fmp_status_string.argtypes = [i32]
    L.fmp_status_string.restype = C.c_char_p
    L.fmp_last_error.argtypes = [vp]
    L.fmp_last_error.restype = C.c_char_p
    L.fmp_runtime_version.argtypes = [C.POINTER(i32), C.POINTER(i32)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("fmp_mlp_scratch_bytes", "fmp_status_string", "fmp_last_error"):
            f.restype = C.c_int32
    _lib = L
    return L
