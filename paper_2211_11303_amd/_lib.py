"""ctypes declarations of the C ABI in include/hlu.h (argument marshalling
only).  Loading fails loudly if libhlu.so has not been built."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HLU_LIB selects another build of the library (the host-sanitizer build in
# the CPU tests); the default is the in-tree libhlu.so.
LIB_PATH = os.environ.get("HLU_LIB") or os.path.join(HERE, "libhlu.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P_i32 = ctypes.POINTER(ctypes.c_int32)
P_f64 = ctypes.POINTER(ctypes.c_double)
P_u8 = ctypes.POINTER(ctypes.c_uint8)

HLU_OK = 0
STATUS = {
    0: "HLU_OK", -1: "HLU_ERR_INVALID_ARG", -2: "HLU_ERR_OUT_OF_MEMORY", -3: "HLU_ERR_DEVICE",
    -4: "HLU_ERR_ZERO_PIVOT", -5: "HLU_ERR_NOT_CONVERGED", -6: "HLU_ERR_STATE",
    -7: "HLU_ERR_RANK_OVERFLOW", -8: "HLU_ERR_UNSUPPORTED",
}
STATUS_CODES = {v: k for k, v in STATUS.items()}
HLU_FP64, HLU_FP32, HLU_FP32_ACC64 = 0, 1, 2


class HluCsr(ctypes.Structure):
    _fields_ = [("n", c_int32), ("nnz", c_int64), ("row_ptr", P_i32), ("col", P_i32), ("val", P_f64)]


class FactorOpts(ctypes.Structure):
    _fields_ = [("eps", c_double), ("max_rank", c_int32), ("prec", c_int32)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("restart", c_int32), ("max_iters", c_int32), ("tol", c_double)]


class RefineOpts(ctypes.Structure):
    _fields_ = [("refine_iters", c_int32), ("max_refines", c_int32), ("eps_factor", c_double)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("converged", c_int32), ("relres", c_double), ("abs_res", c_double)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", c_int64), ("num_clusters", c_int64), ("num_leaf_clusters", c_int64), ("depth", c_int64),
        ("num_admissible", c_int64), ("num_dense", c_int64), ("dense_entries", c_int64),
        ("lowrank_rows_plus_cols", c_int64), ("workspace_bytes", c_int64), ("factor_waves", c_int64),
        ("factor_tasks", c_int64), ("solve_waves", c_int64), ("max_rank", c_int32),
        ("capped_blocks", c_int32), ("mean_rank", c_double), ("lowrank_entries", c_double),
        ("min_abs_pivot", c_double), ("max_abs_pivot", c_double),
        ("solve_launches", c_int64), ("solve_columns", c_int64), ("solve_kernel_ms", c_double),
        ("factor_flops", c_double), ("factor_flops_getrf", c_double), ("factor_flops_tri", c_double),
        ("factor_flops_gemm", c_double), ("factor_flops_trunc", c_double),
        ("rank_capacity_entries", c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SchulzOpts(ctypes.Structure):
    _fields_ = [("max_iters", c_int32), ("tol", c_double)]


class SchulzInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("converged", c_int32), ("residual", c_double), ("residual0", c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("workers", c_int32), ("max_batch_rhs", c_int32), ("hbm_budget", c_size_t), ("eta", c_double),
                ("leaf", c_int32), ("factor", FactorOpts), ("gmres", GmresOpts), ("refine_iters", c_int32),
                ("max_refines", c_int32), ("refine_eps_factor", c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("failed", c_int64),
                ("factorizations", c_int64), ("cache_hits", c_int64), ("evictions", c_int64),
                ("gmres_calls", c_int64), ("coalesced_requests", c_int64), ("bytes_in_use", c_size_t),
                ("peak_bytes", c_size_t), ("cached_factors", c_int32), ("refinements", c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes)
SIGNATURES = {
    "hlu_last_error": (ctypes.c_char_p, []),
    "hlu_kuhn_sizes": (c_int32, [c_int32, P_i32, ctypes.POINTER(c_int64)]),
    "hlu_kuhn_load": (c_int32, [c_int32, P_f64, P_f64]),
    "hlu_kuhn_assemble": (c_int32, [c_int32, c_double, P_i32, P_i32, P_f64, P_i32]),
    "hlu_kuhn_domain_sizes": (c_int32, [c_int32, P_u8, P_i32, ctypes.POINTER(ctypes.c_int64)]),
    "hlu_kuhn_assemble_domain": (c_int32, [c_int32, c_double, P_u8, P_i32, c_double, P_i32, P_i32, P_f64, P_i32]),
    "hlu_kuhn_load_domain": (c_int32, [c_int32, P_u8, P_f64, P_f64]),
    "hlu_kuhn_domain_support_boxes": (c_int32, [c_int32, P_u8, P_i32, P_i32]),
    "hlu_kuhn_assemble_beta": (c_int32, [c_int32, c_double, P_i32, c_double, P_i32, P_i32, P_f64, P_i32]),
    "hlu_kuhn_support_boxes": (c_int32, [c_int32, P_i32, P_i32]),
    "hlu_fit_ranks": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), c_int32, ctypes.POINTER(c_size_t)]),
    "hlu_build_boxes": (c_int32, [ctypes.POINTER(HluCsr), P_i32, P_i32, P_i32, c_double, c_int32,
                                  ctypes.POINTER(c_void_p)]),
    "hlu_spmat_create": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "hlu_spmat_destroy": (None, [c_void_p]),
    "hlu_spmv": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_double, c_double, c_void_p]),
    "hlu_build": (c_int32, [ctypes.POINTER(HluCsr), P_i32, c_double, c_int32, ctypes.POINTER(c_void_p)]),
    "hlu_destroy": (None, [c_void_p]),
    "hlu_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), ctypes.POINTER(c_size_t)]),
    "hlu_bind_workspace": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "hlu_factor": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), c_void_p]),
    "hlu_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p]),
    "hlu_apply_lu": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p]),
    "gmres_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "gmres_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p,
                              ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo), c_void_p, c_size_t,
                              c_void_p]),
    "gmres_refined_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "gmres_solve_refined": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p,
                                      ctypes.POINTER(GmresOpts), ctypes.POINTER(RefineOpts),
                                      ctypes.POINTER(GmresInfo), P_i32, c_void_p, c_size_t, c_void_p]),
    "gmres_static_max_bytes": (c_size_t, []),
    "hlu_richardson_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "hlu_richardson": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_double, c_int32,
                                 ctypes.POINTER(GmresInfo), c_void_p, c_size_t, c_void_p]),
    "gmres_solve_static": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_void_p,
                                     ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo), c_void_p]),
    "hlu_inverse_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), ctypes.POINTER(c_size_t)]),
    "hlu_inverse": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), ctypes.POINTER(SchulzOpts), c_void_p, c_int32,
                              ctypes.POINTER(SchulzInfo), c_void_p]),
    "hlu_structure_sizes": (c_int32, [c_void_p, P_i32, P_i32, P_i32]),
    "hlu_export_structure": (c_int32, [c_void_p, P_i32, P_i32, P_i32, P_i32, P_i32, P_i32, P_i32, P_i32,
                                       P_i32]),
    "hlu_get_ranks": (c_int32, [c_void_p, P_i32]),
    "hlu_get_stats": (c_int32, [c_void_p, ctypes.POINTER(Stats)]),
    "hlu_set_timing": (c_int32, [c_void_p, c_int32]),
    "hlu_sync_status": (c_int32, [c_void_p, c_void_p]),
    "hlu_batch_sync_status": (c_int32, [c_void_p, c_void_p]),
    "hlu_check_trunc_rounds": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), c_int32,
                                         ctypes.POINTER(c_int64)]),
    "hlu_build_shared": (c_int32, [c_void_p, ctypes.POINTER(HluCsr), ctypes.POINTER(c_void_p)]),
    "hlu_batch_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(FactorOpts), c_int32,
                                   ctypes.POINTER(c_void_p)]),
    "hlu_batch_destroy": (None, [c_void_p]),
    "hlu_batch_sizes": (c_int32, [c_void_p, P_i32, P_i32, P_i32, ctypes.POINTER(c_int64),
                                  ctypes.POINTER(c_int64)]),
    "hlu_batch_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    "hlu_batch_bind_workspace": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "hlu_factor_batch": (c_int32, [c_void_p, c_void_p]),
    "hlu_solve_batch": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "gmres_batch_workspace_bytes": (c_size_t, [c_void_p, c_int32, c_int32]),
    "gmres_solve_batch": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.POINTER(GmresOpts),
                                    ctypes.POINTER(GmresInfo), c_void_p, c_size_t, c_void_p]),
    "hlu_device_bytes": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), ctypes.POINTER(c_size_t)]),
    "hlu_plan_device_bytes": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), ctypes.POINTER(c_size_t)]),
    "hlu_solve_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(FactorOpts), ctypes.POINTER(c_size_t)]),
    "hlu_bind_solve_workspace": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "hlu_server_create": (c_int32, [ctypes.POINTER(ServerOpts), ctypes.POINTER(c_void_p)]),
    "hlu_server_prepare": (c_int32, [c_void_p, c_int32]),
    "hlu_server_submit": (c_int32, [c_void_p, c_int32, c_double, c_int32, c_void_p, c_void_p,
                                    ctypes.POINTER(GmresInfo), ctypes.POINTER(c_int64)]),
    "hlu_server_wait": (c_int32, [c_void_p, c_int64, c_double, ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "hlu_server_get_stats": (c_int32, [c_void_p, ctypes.POINTER(ServerStats)]),
    "hlu_server_destroy": (None, [c_void_p]),
    "hlu_autotune_leaf": (c_int32, [c_int32, c_double, c_double, P_i32, c_int32, ctypes.POINTER(FactorOpts),
                                    ctypes.POINTER(GmresOpts), c_int32, ctypes.POINTER(c_double), P_i32, c_void_p]),
}

_lib = None


class HluError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if libhlu.so is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhlu.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != HLU_OK:
        raise HluError(status, lib().hlu_last_error().decode())
    return status
