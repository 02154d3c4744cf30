"""Python binding of libhlu with the names of the C ABI (include/hlu.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch provides device memory and the stream.  Blocks of
vectors are torch tensors of shape (nrhs, N) (contiguous), i.e. the
column-major N x nrhs layout of the C ABI with leading dimension N.
"""
import ctypes

import numpy as np

from . import _lib as L

PREC = {"fp64": L.HLU_FP64, "fp32": L.HLU_FP32, "fp32-acc64": L.HLU_FP32_ACC64}


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _as_block(t, N):
    """(N,) or (nrhs, N) float64 CUDA tensor -> (2-D view, nrhs)."""
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    t2 = t.reshape(1, -1) if t.dim() == 1 else t
    if t2.shape[-1] != N or not t2.is_contiguous():
        raise ValueError(f"expected a contiguous (nrhs, {N}) tensor")
    return t2, t2.shape[0]


# ------------------------------------------------------------------ problem
def hlu_kuhn_sizes(n):
    N = ctypes.c_int32()
    nnz = ctypes.c_int64()
    L.check(L.lib().hlu_kuhn_sizes(n, ctypes.byref(N), ctypes.byref(nnz)))
    return N.value, nnz.value


def hlu_kuhn_assemble(n, kappa):
    """A = K - kappa^2 M on the Kuhn cube with n^3 cubes: (row_ptr, col, val,
    mid2) as numpy arrays (host)."""
    N, nnz = hlu_kuhn_sizes(n)
    rp = np.empty(N + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    va = np.empty(nnz, np.float64)
    mid = np.empty((N, 3), np.int32)
    L.check(L.lib().hlu_kuhn_assemble(n, float(kappa), _ptr(rp, ctypes.c_int32), _ptr(ci, ctypes.c_int32),
                                      _ptr(va, ctypes.c_double), _ptr(mid, ctypes.c_int32)))
    return rp, ci, va, mid


def hlu_kuhn_domain_sizes(n, mask):
    """hlu_kuhn_domain_sizes: (N, nnz) on the union of the flagged cubes."""
    m = np.ascontiguousarray(mask, np.uint8)
    assert m.size == n ** 3
    N = ctypes.c_int32()
    nnz = ctypes.c_int64()
    L.check(L.lib().hlu_kuhn_domain_sizes(int(n), _ptr(m, ctypes.c_uint8), ctypes.byref(N), ctypes.byref(nnz)))
    return N.value, nnz.value


def hlu_kuhn_assemble_domain(n, kappa, mask, beta_box=None, beta_in=1.0):
    """hlu_kuhn_assemble_domain: A = K_beta - kappa^2 M on the union of the
    cubes flagged in mask (n^3 entries, cube (i, j, k) at i + n (j + n k))."""
    m = np.ascontiguousarray(mask, np.uint8)
    N, nnz = hlu_kuhn_domain_sizes(n, m)
    box = None if beta_box is None else np.ascontiguousarray(beta_box, np.int32)
    rp = np.empty(N + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    va = np.empty(nnz, np.float64)
    mid = np.empty((N, 3), np.int32)
    L.check(L.lib().hlu_kuhn_assemble_domain(int(n), float(kappa), _ptr(m, ctypes.c_uint8),
                                             None if box is None else _ptr(box, ctypes.c_int32), float(beta_in),
                                             _ptr(rp, ctypes.c_int32), _ptr(ci, ctypes.c_int32),
                                             _ptr(va, ctypes.c_double), _ptr(mid, ctypes.c_int32)))
    return rp, ci, va, mid


def hlu_kuhn_load_domain(n, mask, J=(1.0, 1.0, 1.0)):
    """hlu_kuhn_load_domain: b_j = <J, Phi_j> on the union of the flagged cubes."""
    m = np.ascontiguousarray(mask, np.uint8)
    N, _ = hlu_kuhn_domain_sizes(n, m)
    Jv = np.ascontiguousarray(J, np.float64)
    b = np.empty(N, np.float64)
    L.check(L.lib().hlu_kuhn_load_domain(int(n), _ptr(m, ctypes.c_uint8), _ptr(Jv, ctypes.c_double),
                                         _ptr(b, ctypes.c_double)))
    return b


def hlu_kuhn_domain_support_boxes(n, mask):
    """hlu_kuhn_domain_support_boxes: (lo2, hi2) on the union of the flagged cubes."""
    m = np.ascontiguousarray(mask, np.uint8)
    N, _ = hlu_kuhn_domain_sizes(n, m)
    lo = np.empty((N, 3), np.int32)
    hi = np.empty((N, 3), np.int32)
    L.check(L.lib().hlu_kuhn_domain_support_boxes(int(n), _ptr(m, ctypes.c_uint8), _ptr(lo, ctypes.c_int32),
                                                  _ptr(hi, ctypes.c_int32)))
    return lo, hi


def hlu_kuhn_assemble_beta(n, kappa, beta_box, beta_in):
    """hlu_kuhn_assemble_beta: A = K_beta - kappa^2 M with the curl-curl
    coefficient beta_in on the cubes (i, j, k) of the half-open index box
    beta_box = (i0, j0, k0, i1, j1, k1), 1 elsewhere."""
    N, nnz = hlu_kuhn_sizes(n)
    box = np.ascontiguousarray(beta_box, np.int32)
    assert box.shape == (6,)
    rp = np.empty(N + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    va = np.empty(nnz, np.float64)
    mid = np.empty((N, 3), np.int32)
    L.check(L.lib().hlu_kuhn_assemble_beta(n, float(kappa), _ptr(box, ctypes.c_int32), float(beta_in),
                                           _ptr(rp, ctypes.c_int32), _ptr(ci, ctypes.c_int32),
                                           _ptr(va, ctypes.c_double), _ptr(mid, ctypes.c_int32)))
    return rp, ci, va, mid


def hlu_kuhn_support_boxes(n):
    """hlu_kuhn_support_boxes: (lo2, hi2), N x 3 each, doubled lattice units."""
    N, _ = hlu_kuhn_sizes(n)
    lo = np.empty((N, 3), np.int32)
    hi = np.empty((N, 3), np.int32)
    L.check(L.lib().hlu_kuhn_support_boxes(int(n), _ptr(lo, ctypes.c_int32), _ptr(hi, ctypes.c_int32)))
    return lo, hi


def hlu_autotune_leaf(n, kappa, leaves=(32, 48, 64), eta=2.0, eps=1e-3, max_rank=0, prec="fp32", restart=50,
                      max_iters=1000, tol=1e-8, nrhs=1, stream=None):
    """hlu_autotune_leaf: (best leaf, [device seconds of factor + GMRES per
    candidate]) for the Kuhn-cube mesh n at wavenumber kappa."""
    cand = np.ascontiguousarray(leaves, np.int32)
    secs = np.empty(len(cand), np.float64)
    best = np.empty(1, np.int32)
    fo = L.FactorOpts(float(eps), int(max_rank), PREC[prec])
    go = L.GmresOpts(int(restart), int(max_iters), float(tol))
    L.check(L.lib().hlu_autotune_leaf(int(n), float(kappa), float(eta), _ptr(cand, ctypes.c_int32), len(cand),
                                      ctypes.byref(fo), ctypes.byref(go), int(nrhs),
                                      secs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _ptr(best, ctypes.c_int32), _stream(stream)))
    return int(best[0]), secs.tolist()


def hlu_kuhn_load(n, J=(0.0, 0.0, 1.0)):
    """b_j = <J, Phi_j> over the interior edges (host numpy array)."""
    N, _ = hlu_kuhn_sizes(n)
    Jv = np.ascontiguousarray(J, np.float64)
    b = np.empty(N, np.float64)
    L.check(L.lib().hlu_kuhn_load(int(n), _ptr(Jv, ctypes.c_double), _ptr(b, ctypes.c_double)))
    return b


# ------------------------------------------------------------ sparse matrix
class SpMat:
    """Device CSR of A (hlu_spmat)."""

    def __init__(self, row_ptr, col, val, device="cuda"):
        torch = _torch()
        self.n = len(row_ptr) - 1
        self.nnz = len(col)
        self.rp = torch.as_tensor(np.ascontiguousarray(row_ptr, np.int32)).to(device)
        self.ci = torch.as_tensor(np.ascontiguousarray(col, np.int32)).to(device)
        self.val = torch.as_tensor(np.ascontiguousarray(val, np.float64)).to(device)
        h = ctypes.c_void_p()
        L.check(L.lib().hlu_spmat_create(self.n, self.nnz, _dev_ptr(self.rp), _dev_ptr(self.ci),
                                         _dev_ptr(self.val), ctypes.byref(h)))
        self.handle = h
        # bound now: module globals may already be gone when the interpreter exits
        self._destroy = L.lib().hlu_spmat_destroy

    def __del__(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def hlu_spmv(self, x, y=None, alpha=1.0, beta=0.0, stream=None):
        torch = _torch()
        x2, nrhs = _as_block(x, self.n)
        if y is None:
            y = torch.zeros_like(x)
        y2, _ = _as_block(y, self.n)
        L.check(L.lib().hlu_spmv(self.handle, _dev_ptr(x2), _dev_ptr(y2), nrhs, self.n, float(alpha),
                                 float(beta), _stream(stream)))
        return y


# ------------------------------------------------------------- H-LU handle
class HLU:
    """hlu_build + workspace + hlu_factor / hlu_solve / hlu_apply_lu."""

    def __init__(self, row_ptr, col, val, mid2=None, eta=2.0, leaf=64, share=None, boxes=None):
        """hlu_build; with share=<HLU of the same sparsity pattern>,
        hlu_build_shared (mid2, eta and leaf are then the prototype's); with
        boxes=(lo2, hi2), hlu_build_boxes (admissibility on those boxes)."""
        self._rp = np.ascontiguousarray(row_ptr, np.int32)
        self._ci = np.ascontiguousarray(col, np.int32)
        self._va = np.ascontiguousarray(val, np.float64)
        csr = L.HluCsr(len(self._rp) - 1, len(self._ci), _ptr(self._rp, ctypes.c_int32),
                       _ptr(self._ci, ctypes.c_int32), _ptr(self._va, ctypes.c_double))
        h = ctypes.c_void_p()
        if share is not None:
            L.check(L.lib().hlu_build_shared(share.handle, ctypes.byref(csr), ctypes.byref(h)))
            eta, leaf = share.eta, share.leaf
        else:
            mid = np.ascontiguousarray(mid2, np.int32)
            if boxes is None:
                L.check(L.lib().hlu_build(ctypes.byref(csr), _ptr(mid, ctypes.c_int32), float(eta), int(leaf),
                                          ctypes.byref(h)))
            else:
                lo = np.ascontiguousarray(boxes[0], np.int32)
                hi = np.ascontiguousarray(boxes[1], np.int32)
                assert lo.shape == mid.shape and hi.shape == mid.shape
                L.check(L.lib().hlu_build_boxes(ctypes.byref(csr), _ptr(mid, ctypes.c_int32), _ptr(lo, ctypes.c_int32),
                                                _ptr(hi, ctypes.c_int32), float(eta), int(leaf), ctypes.byref(h)))
        self.handle = h
        self._destroy = L.lib().hlu_destroy
        self.n = len(self._rp) - 1
        self.leaf = leaf
        self.eta = eta
        self.work = None
        self.prec = None

    def __del__(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    @staticmethod
    def _opts(eps, max_rank, prec):
        return L.FactorOpts(float(eps), int(max_rank), PREC[prec])

    def hlu_workspace_bytes(self, eps, max_rank=0, prec="fp64"):
        o = self._opts(eps, max_rank, prec)
        b = ctypes.c_size_t()
        L.check(L.lib().hlu_workspace_bytes(self.handle, ctypes.byref(o), ctypes.byref(b)))
        return b.value

    def hlu_bind_workspace(self, nbytes):
        torch = _torch()
        if self.work is None or self.work.numel() < nbytes:
            self.work = None
            self.work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        L.check(L.lib().hlu_bind_workspace(self.handle, _dev_ptr(self.work), self.work.numel()))

    def hlu_factor(self, eps, max_rank=0, prec="fp64", stream=None, allow_overflow=False):
        nbytes = self.hlu_workspace_bytes(eps, max_rank, prec)
        self.hlu_bind_workspace(nbytes)
        o = self._opts(eps, max_rank, prec)
        st = L.lib().hlu_factor(self.handle, ctypes.byref(o), _stream(stream))
        if st == -7 and allow_overflow:
            st = L.HLU_OK
        L.check(st)
        self.prec = prec
        return self

    def hlu_device_bytes(self, eps, max_rank=0, prec="fp64"):
        """hlu_device_bytes: workspace, solve buffers, values and plans."""
        o = self._opts(eps, max_rank, prec)
        b = ctypes.c_size_t()
        L.check(L.lib().hlu_device_bytes(self.handle, ctypes.byref(o), ctypes.byref(b)))
        return b.value

    def hlu_fit_ranks(self, eps, margin=4, max_rank=0, prec="fp64"):
        """hlu_fit_ranks: capacities fitted to the ranks of the last
        hlu_factor (margin < 0: back to uniform).  Drops the old workspace;
        the next hlu_factor(eps, max_rank, prec) binds one of the returned
        size."""
        o = self._opts(eps, max_rank, prec)
        b = ctypes.c_size_t()
        L.check(L.lib().hlu_fit_ranks(self.handle, ctypes.byref(o), int(margin), ctypes.byref(b)))
        self.work = None
        return b.value

    def hlu_bind_solve_workspace(self, eps, max_rank=0, prec="fp64"):
        """Caller-owned (torch) memory for the persistent solve's buffers."""
        torch = _torch()
        o = self._opts(eps, max_rank, prec)
        b = ctypes.c_size_t()
        L.check(L.lib().hlu_solve_workspace_bytes(self.handle, ctypes.byref(o), ctypes.byref(b)))
        self.solve_work = torch.empty(b.value, dtype=torch.uint8, device="cuda")
        L.check(L.lib().hlu_bind_solve_workspace(self.handle, _dev_ptr(self.solve_work), self.solve_work.numel()))
        return b.value

    def hlu_inverse_workspace_bytes(self, eps, max_rank=0, prec="fp64"):
        o = self._opts(eps, max_rank, prec)
        b = ctypes.c_size_t()
        L.check(L.lib().hlu_inverse_workspace_bytes(self.handle, ctypes.byref(o), ctypes.byref(b)))
        return b.value

    def hlu_inverse(self, probe, eps, max_rank=0, prec="fp64", tol=1e-6, max_iters=60, stream=None):
        """Schulz inverse B_H (hlu_inverse) into the handle; probe: device
        block (nprobe, N) in the natural order.  Returns the info dict;
        afterwards hlu_solve / gmres_solve apply B_H."""
        nbytes = self.hlu_inverse_workspace_bytes(eps, max_rank, prec)
        self.hlu_bind_workspace(nbytes)
        p2, nprobe = _as_block(probe, self.n)
        o = self._opts(eps, max_rank, prec)
        so = L.SchulzOpts(int(max_iters), float(tol))
        info = L.SchulzInfo()
        L.check(L.lib().hlu_inverse(self.handle, ctypes.byref(o), ctypes.byref(so), _dev_ptr(p2), nprobe,
                                    ctypes.byref(info), _stream(stream)))
        self.prec = prec
        return {name: getattr(info, name) for name, _ in info._fields_}

    def hlu_solve(self, b, x=None, stream=None):
        torch = _torch()
        b2, nrhs = _as_block(b, self.n)
        if x is None:
            x = torch.empty_like(b)
        x2, _ = _as_block(x, self.n)
        L.check(L.lib().hlu_solve(self.handle, _dev_ptr(b2), _dev_ptr(x2), nrhs, self.n, _stream(stream)))
        return x

    def hlu_sync_status(self, stream=None):
        """Synchronise and raise HLU_ERR_DEVICE if a persistent solve of this
        handle gave up waiting since the last call."""
        L.check(L.lib().hlu_sync_status(self.handle, _stream(stream)))

    def hlu_apply_lu(self, v, stream=None):
        torch = _torch()
        v2, nrhs = _as_block(v, self.n)
        y = torch.empty_like(v)
        y2, _ = _as_block(y, self.n)
        L.check(L.lib().hlu_apply_lu(self.handle, _dev_ptr(v2), _dev_ptr(y2), nrhs, self.n, _stream(stream)))
        return y

    def hlu_get_stats(self):
        s = L.Stats()
        L.check(L.lib().hlu_get_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def hlu_set_timing(self, enable=True):
        """Bracket every persistent solve launch with HIP events (resets the
        totals that hlu_get_stats reports as solve_launches / solve_kernel_ms)."""
        L.check(L.lib().hlu_set_timing(self.handle, 1 if enable else 0))
        return self

    def hlu_check_trunc_rounds(self, eps, forced_rank, max_rank=0, prec="fp64"):
        """Host replay of the truncation rounds of the factor plan with every
        rank forced to forced_rank (no device work)."""
        o = self._opts(eps, max_rank, prec)
        out = (ctypes.c_int64 * 5)()
        L.check(L.lib().hlu_check_trunc_rounds(self.handle, ctypes.byref(o), int(forced_rank), out))
        return dict(zip(("ops", "rounds", "max_rounds", "stalled_rounds", "unfinished"), list(out)))

    def hlu_get_ranks(self):
        nb = self.structure_sizes()[2]
        r = np.empty(nb, np.int32)
        L.check(L.lib().hlu_get_ranks(self.handle, _ptr(r, ctypes.c_int32)))
        return r

    def structure_sizes(self):
        N, C, B = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().hlu_structure_sizes(self.handle, ctypes.byref(N), ctypes.byref(C), ctypes.byref(B)))
        return N.value, C.value, B.value

    def hlu_export_structure(self):
        N, C, B = self.structure_sizes()
        out = {k: np.empty(N if k == "perm" else (C if k in ("begin", "end", "level", "son0", "son1") else B),
                           np.int32)
               for k in ("perm", "begin", "end", "level", "son0", "son1", "brow", "bcol", "bkind")}
        L.check(L.lib().hlu_export_structure(self.handle, *[_ptr(out[k], ctypes.c_int32) for k in
                                                            ("perm", "begin", "end", "level", "son0", "son1",
                                                             "brow", "bcol", "bkind")]))
        return out


# -------------------------------------------------------------------- GMRES
def gmres_workspace_bytes(n, nrhs, restart):
    return L.lib().gmres_workspace_bytes(n, nrhs, restart)


def gmres_solve(A, b, precond=None, restart=50, tol=1e-8, max_iters=1000, stream=None, work=None,
                raise_on_fail=True):
    """Returns (x, infos) with infos a list of dicts (iters, converged,
    relres, abs_res) per right-hand side."""
    torch = _torch()
    b2, nrhs = _as_block(b, A.n)
    x = torch.zeros_like(b2)
    nbytes = gmres_workspace_bytes(A.n, nrhs, restart)
    if work is None or work.numel() < nbytes:
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    o = L.GmresOpts(int(restart), int(max_iters), float(tol))
    info = (L.GmresInfo * nrhs)()
    st = L.lib().gmres_solve(A.handle, _dev_ptr(b2), _dev_ptr(x), nrhs, A.n,
                             precond.handle if precond is not None else None, ctypes.byref(o), info,
                             _dev_ptr(work), work.numel(), _stream(stream))
    infos = [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres, abs_res=i.abs_res) for i in info]
    if st != L.HLU_OK and (raise_on_fail or st != -5):
        L.check(st)
    return x.reshape(b.shape), infos


def gmres_solve_refined(A, b, H, restart=50, tol=1e-8, max_iters=1000, refine_iters=100, max_refines=2,
                        eps_factor=0.1, stream=None, raise_on_fail=True):
    """gmres_solve_refined: GMRES that refactors H at a smaller eps for the
    columns that miss tol within refine_iters.  Returns (x, infos, refines)."""
    torch = _torch()
    b2, nrhs = _as_block(b, A.n)
    x = torch.zeros_like(b2)
    work = torch.empty(L.lib().gmres_refined_workspace_bytes(A.n, nrhs, int(restart)), dtype=torch.uint8,
                       device="cuda")
    o = L.GmresOpts(int(restart), int(max_iters), float(tol))
    r = L.RefineOpts(int(refine_iters), int(max_refines), float(eps_factor))
    info = (L.GmresInfo * nrhs)()
    refines = np.zeros(1, np.int32)
    st = L.lib().gmres_solve_refined(A.handle, _dev_ptr(b2), _dev_ptr(x), nrhs, A.n, H.handle, ctypes.byref(o),
                                     ctypes.byref(r), info, _ptr(refines, ctypes.c_int32), _dev_ptr(work),
                                     work.numel(), _stream(stream))
    infos = [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres, abs_res=i.abs_res) for i in info]
    if st != L.HLU_OK and (raise_on_fail or st != -5):
        L.check(st)
    return x.reshape(b.shape), infos, int(refines[0])


def hlu_richardson(A, b, precond, tol=1e-8, max_iters=100, stream=None):
    """Algorithm 1, steps III-IV (hlu_richardson): returns (x, infos) with
    infos a list of dicts (iters, converged, relres, abs_res) per column."""
    torch = _torch()
    b2, nrhs = _as_block(b, A.n)
    x = torch.zeros_like(b2)
    work = torch.empty(L.lib().hlu_richardson_workspace_bytes(A.n, nrhs), dtype=torch.uint8, device="cuda")
    info = (L.GmresInfo * nrhs)()
    L.check(L.lib().hlu_richardson(A.handle, _dev_ptr(b2), _dev_ptr(x), nrhs, A.n, precond.handle, float(tol),
                                   int(max_iters), info, _dev_ptr(work), work.numel(), _stream(stream)))
    infos = [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres, abs_res=i.abs_res) for i in info]
    return x.reshape(b.shape), infos


def gmres_solve_static(A, b, precond=None, restart=50, tol=1e-8, max_iters=1000, stream=None,
                       raise_on_fail=True):
    """gmres_solve on the library's static device workspace (no device
    allocation inside the call; x is the caller's output tensor)."""
    torch = _torch()
    b2, nrhs = _as_block(b, A.n)
    x = torch.zeros_like(b2)
    o = L.GmresOpts(int(restart), int(max_iters), float(tol))
    info = (L.GmresInfo * nrhs)()
    st = L.lib().gmres_solve_static(A.handle, _dev_ptr(b2), _dev_ptr(x), nrhs, A.n,
                                    precond.handle if precond is not None else None, ctypes.byref(o), info,
                                    _stream(stream))
    infos = [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres, abs_res=i.abs_res) for i in info]
    _check_gmres(st, raise_on_fail)
    return x.reshape(b.shape), infos


def gmres_static_max_bytes():
    return L.lib().gmres_static_max_bytes()


def _check_gmres(st, raise_on_fail):
    if st != L.HLU_OK and (raise_on_fail or st != -5):
        L.check(st)


# -------------------------------------------------------------------- batch
class HLUBatch:
    """hlu_batch_create / bind / hlu_factor_batch / hlu_solve_batch /
    gmres_solve_batch over member HLU handles.  Stacked vectors are torch
    tensors of shape (nrhs, n_total); problem p holds columns
    [row_base[p], row_base[p] + N_p)."""

    def __init__(self, members, eps, max_rank=0, prec="fp32", max_rhs=1):
        self.members = list(members)
        arr = (ctypes.c_void_p * len(self.members))(*[m.handle.value for m in self.members])
        o = HLU._opts(eps, max_rank, prec)
        b = ctypes.c_void_p()
        L.check(L.lib().hlu_batch_create(arr, len(self.members), ctypes.byref(o), int(max_rhs), ctypes.byref(b)))
        self.handle = b
        self._destroy = L.lib().hlu_batch_destroy
        self.prec = prec
        self.max_rhs = max_rhs
        count, ntot = ctypes.c_int32(), ctypes.c_int32()
        self.row_base = np.empty(len(self.members), np.int32)
        waves, tasks = ctypes.c_int64(), ctypes.c_int64()
        L.check(L.lib().hlu_batch_sizes(b, ctypes.byref(count), ctypes.byref(ntot),
                                        _ptr(self.row_base, ctypes.c_int32), ctypes.byref(waves),
                                        ctypes.byref(tasks)))
        self.n_total = ntot.value
        self.factor_waves = waves.value
        self.factor_tasks = tasks.value
        self.work = None

    def __del__(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def hlu_batch_workspace_bytes(self):
        n = ctypes.c_size_t()
        L.check(L.lib().hlu_batch_workspace_bytes(self.handle, ctypes.byref(n)))
        return n.value

    def hlu_batch_bind_workspace(self, work=None):
        torch = _torch()
        nbytes = self.hlu_batch_workspace_bytes()
        if work is None:
            work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.work = work
        L.check(L.lib().hlu_batch_bind_workspace(self.handle, _dev_ptr(work), work.numel()))
        return self

    def hlu_factor_batch(self, stream=None, allow_overflow=False):
        if self.work is None:
            self.hlu_batch_bind_workspace()
        st = L.lib().hlu_factor_batch(self.handle, _stream(stream))
        if st == -7 and allow_overflow:
            st = L.HLU_OK
        L.check(st)
        for m in self.members:
            m.prec = self.prec
        return self

    def stack(self, parts):
        """List of (nrhs, N_p) tensors -> one (nrhs, n_total) tensor."""
        torch = _torch()
        return torch.cat([p.reshape(-1, p.shape[-1]) for p in parts], dim=1).contiguous()

    def unstack(self, x):
        out = []
        for p, m in enumerate(self.members):
            r0 = int(self.row_base[p])
            out.append(x[:, r0:r0 + m.n])
        return out

    def hlu_batch_sync_status(self, stream=None):
        L.check(L.lib().hlu_batch_sync_status(self.handle, _stream(stream)))

    def hlu_solve_batch(self, b, stream=None):
        torch = _torch()
        b2, nrhs = _as_block(b, self.n_total)
        x = torch.empty_like(b2)
        L.check(L.lib().hlu_solve_batch(self.handle, _dev_ptr(b2), _dev_ptr(x), nrhs, _stream(stream)))
        return x.reshape(b.shape)

    def gmres_solve_batch(self, b, restart=50, tol=1e-8, max_iters=1000, stream=None, work=None,
                          raise_on_fail=True):
        """Returns (x, infos): infos[p][c] is the record of problem p,
        column c."""
        torch = _torch()
        b2, nrhs = _as_block(b, self.n_total)
        x = torch.zeros_like(b2)
        nbytes = L.lib().gmres_batch_workspace_bytes(self.handle, nrhs, restart)
        if work is None or work.numel() < nbytes:
            work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        o = L.GmresOpts(int(restart), int(max_iters), float(tol))
        P = len(self.members)
        info = (L.GmresInfo * (P * nrhs))()
        st = L.lib().gmres_solve_batch(self.handle, _dev_ptr(b2), _dev_ptr(x), nrhs, ctypes.byref(o), info,
                                       _dev_ptr(work), work.numel(), _stream(stream))
        infos = [[dict(iters=info[c * P + p].iters, converged=bool(info[c * P + p].converged),
                       relres=info[c * P + p].relres, abs_res=info[c * P + p].abs_res) for c in range(nrhs)]
                 for p in range(P)]
        _check_gmres(st, raise_on_fail)
        return x.reshape(b.shape), infos


# ------------------------------------------------------------------ serving
class Server:
    """hlu_server_*: request loop with a factor cache per (n, kappa),
    admission by device bytes and continuous batching of right-hand sides.
    Right-hand sides and results are host numpy arrays of shape (nrhs, N).
    refine_iters > 0: columns not converged after that many iterations make
    the cached factor be refactored with eps * refine_eps_factor (at most
    max_refines times) and are solved again."""

    def __init__(self, workers=4, max_batch_rhs=32, hbm_budget=200 << 30, eta=2.0, leaf=64, eps=1e-3,
                 max_rank=32, prec="fp32", restart=50, max_iters=1000, tol=1e-8, refine_iters=0, max_refines=2,
                 refine_eps_factor=0.1):
        o = L.ServerOpts(int(workers), int(max_batch_rhs), int(hbm_budget), float(eta), int(leaf),
                         L.FactorOpts(float(eps), int(max_rank), PREC[prec]),
                         L.GmresOpts(int(restart), int(max_iters), float(tol)), int(refine_iters), int(max_refines),
                         float(refine_eps_factor))
        h = ctypes.c_void_p()
        L.check(L.lib().hlu_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._destroy = L.lib().hlu_server_destroy
        self._live = {}

    def close(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def hlu_server_prepare(self, n):
        L.check(L.lib().hlu_server_prepare(self.handle, int(n)))

    def hlu_server_submit(self, n, kappa, b):
        """b: (nrhs, N) float64 host array.  Returns a ticket."""
        b = np.ascontiguousarray(b, np.float64)
        if b.ndim == 1:
            b = b.reshape(1, -1)
        x = np.empty_like(b)
        info = (L.GmresInfo * b.shape[0])()
        t = ctypes.c_int64()
        L.check(L.lib().hlu_server_submit(self.handle, int(n), float(kappa), b.shape[0],
                                          b.ctypes.data_as(ctypes.c_void_p), x.ctypes.data_as(ctypes.c_void_p),
                                          info, ctypes.byref(t)))
        self._live[t.value] = (b, x, info)
        return t.value

    def hlu_server_wait(self, ticket, timeout=-1.0, raise_on_fail=True):
        """Returns (x, infos, queued_s, latency_s)."""
        q, lat = ctypes.c_double(), ctypes.c_double()
        st = L.lib().hlu_server_wait(self.handle, ticket, float(timeout), ctypes.byref(q), ctypes.byref(lat))
        if st == -6 and timeout >= 0:
            L.check(st)
        b, x, info = self._live.pop(ticket)
        infos = [dict(iters=i.iters, converged=bool(i.converged), relres=i.relres, abs_res=i.abs_res) for i in info]
        _check_gmres(st, raise_on_fail)
        return x, infos, q.value, lat.value

    def hlu_server_get_stats(self):
        s = L.ServerStats()
        L.check(L.lib().hlu_server_get_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()
