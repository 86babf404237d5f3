"""Nested-dissection NEGF solver for MI355X: Python binding of libndnegf.so.

The binding marshals arguments for the C entry points (include/ndnegf.h);
every step of the computation runs in the library's HIP kernels.  PyTorch is
used only for device memory and streams.

    sym  = analyze(n, rowptr, col, val, contacts, coords)     # host, once per geometry
    plan = Plan(sym, max_batch=64)                             # device workspace
    gr, gl, gg = plan.solve(E, eta, sig_r, sig_less, V=None)   # torch tensors on the GPU
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import NDG_FP64, NDG_MIXED, NdgError, load  # noqa: F401

__all__ = ["analyze", "Symbolic", "Plan", "load", "NdgError", "NDG_FP64", "NDG_MIXED",
           "ndg_analyze", "ndg_symbolic_info", "ndg_symbolic_arrays", "ndg_plan_create",
           "ndg_plan_destroy", "ndg_plan_info", "ndg_solve", "ndg_plan_status",
           "ndg_plan_export_block", "ndg_plan_set_profiling", "ndg_plan_profile", "ndg_symbolic_costs",
           "ndg_density", "ndg_plan_enable_adjoint", "ndg_density_vjp", "ndg_density_vjp_noalloc",
           "NDDensity",
           "ndg_batch_create", "ndg_batch_destroy", "ndg_batch_solve", "ndg_batch_launches", "Batch",
           "ndg_plan_enable_scattering", "ndg_solve_scattering", "ndg_scba", "ndg_poisson_newton_step",
           "ndg_solve_transport",
           "ndg_status_string", "ndg_last_error"]


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ----------------------------------------------------------------------------
# thin wrappers with the C names
# ----------------------------------------------------------------------------

def ndg_analyze(n, rowptr, col, val, contacts, coords=None, leaf_max=0, max_cluster=0,
                tree_kind=0, slab=0, layer_of=None, layer_max=0):
    lib = load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    cs = [np.ascontiguousarray(c, dtype=np.int32) for c in contacts]
    cptrs = (_lib.I32P * max(1, len(cs)))(*[_ptr(c, C.c_int32) for c in cs])
    cn = np.array([len(c) for c in cs] or [0], dtype=np.int32)
    cc = None
    if coords is not None:
        coords = np.ascontiguousarray(coords, dtype=np.float64).reshape(n, 3)
        cc = _ptr(coords, C.c_double)
    lo = None
    if layer_of is not None:
        layer_of = np.ascontiguousarray(layer_of, dtype=np.int32).reshape(n)
        lo = _ptr(layer_of, C.c_int32)
    opts = _lib.TreeOpts(leaf_max, max_cluster, tree_kind, slab, layer_max, 0, lo)
    out = C.c_void_p()
    _lib.check(lib.ndg_analyze(n, _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32),
                               _ptr(val, C.c_double), len(cs), cptrs, _ptr(cn, C.c_int32), cc,
                               C.byref(opts), C.byref(out)))
    return out


def ndg_symbolic_info(sy) -> dict:
    info = _lib.Info()
    _lib.check(load().ndg_symbolic_info(sy, C.byref(info)))
    return info.as_dict()


def ndg_symbolic_arrays(sy) -> dict:
    info = ndg_symbolic_info(sy)
    n, nc, nb = info["n"], info["nclusters"], info["nnz_boundary"]
    out = {"perm": np.zeros(n, np.int32), "cl_off": np.zeros(nc + 1, np.int32),
           "parent": np.zeros(nc, np.int32), "height": np.zeros(nc, np.int32),
           "bptr": np.zeros(nc + 1, np.int64), "bidx": np.zeros(max(1, nb), np.int32)}
    _lib.check(load().ndg_symbolic_arrays(
        sy, _ptr(out["perm"], C.c_int32), _ptr(out["cl_off"], C.c_int32),
        _ptr(out["parent"], C.c_int32), _ptr(out["height"], C.c_int32),
        _ptr(out["bptr"], C.c_int64), _ptr(out["bidx"], C.c_int32)))
    out["bidx"] = out["bidx"][:nb]
    return out


def ndg_plan_create(sy, max_batch: int, device: int = 0):
    out = C.c_void_p()
    _lib.check(load().ndg_plan_create(sy, max_batch, device, C.byref(out)))
    return out


def ndg_plan_destroy(plan):
    _lib.check(load().ndg_plan_destroy(plan))


def ndg_plan_info(plan) -> dict:
    info = _lib.Info()
    _lib.check(load().ndg_plan_info(plan, C.byref(info)))
    return info.as_dict()


def ndg_solve(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, dgr_ptr, dgl_ptr, dgg_ptr,
              growth_ptr, prec, stream_ptr):
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    _lib.check(load().ndg_solve(plan, ne, e_ptr, eta, v_ptr, sr, sl, dgr_ptr, dgl_ptr, dgg_ptr,
                                growth_ptr, prec, stream_ptr))


def ndg_solve_transport(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, dgr_ptr, dgl_ptr,
                        dgg_ptr, t_ptr, growth_ptr, stream_ptr):
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    _lib.check(load().ndg_solve_transport(plan, ne, e_ptr, eta, v_ptr, sr, sl, dgr_ptr, dgl_ptr, dgg_ptr,
                                          t_ptr, growth_ptr, stream_ptr))


def ndg_plan_enable_scattering(plan):
    _lib.check(load().ndg_plan_enable_scattering(plan))


def ndg_solve_scattering(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, sr_ph_ptr,
                         sl_ph_ptr, dgr_ptr, dgl_ptr, dgg_ptr, growth_ptr, current_ptr, stream_ptr):
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    _lib.check(load().ndg_solve_scattering(plan, ne, e_ptr, eta, v_ptr, sr, sl, sr_ph_ptr, sl_ph_ptr,
                                           dgr_ptr, dgl_ptr, dgg_ptr, growth_ptr, current_ptr,
                                           stream_ptr))


def ndg_scba(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, d0, mix, tol, max_iter,
             sr_ph_ptr, sl_ph_ptr, dgr_ptr, dgl_ptr, dgg_ptr, current_ptr, stream_ptr):
    """Returns (iterations, residual)."""
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    it = C.c_int32()
    res = C.c_double()
    _lib.check(load().ndg_scba(plan, ne, e_ptr, eta, v_ptr, sr, sl, d0, mix, tol, max_iter, sr_ph_ptr,
                               sl_ph_ptr, dgr_ptr, dgl_ptr, dgg_ptr, current_ptr, C.byref(it),
                               C.byref(res), stream_ptr))
    return it.value, res.value


def ndg_poisson_newton_step(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, ce_ptr, k_rowptr_ptr,
                            k_col_ptr, k_val_ptr, k_nnz, beta, nd_ptr, cg_tol, cg_max_iter, delta_ptr,
                            stream_ptr):
    """Returns (||F||, cg iterations, final relative residual)."""
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    fn = C.c_double()
    it = C.c_int32()
    res = C.c_double()
    _lib.check(load().ndg_poisson_newton_step(plan, ne, e_ptr, eta, v_ptr, sr, sl, ce_ptr, k_rowptr_ptr,
                                              k_col_ptr, k_val_ptr, k_nnz, beta, nd_ptr, cg_tol, cg_max_iter,
                                              delta_ptr, C.byref(fn), C.byref(it), C.byref(res),
                                              stream_ptr))
    return fn.value, it.value, res.value


def ndg_density(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, ce_ptr, dens_ptr, prec,
                stream_ptr):
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    _lib.check(load().ndg_density(plan, ne, e_ptr, eta, v_ptr, sr, sl, ce_ptr, dens_ptr, prec,
                                  stream_ptr))


def ndg_plan_enable_adjoint(plan):
    _lib.check(load().ndg_plan_enable_adjoint(plan))


def ndg_density_vjp(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, ce_ptr, nbar_ptr,
                    vbar_ptr, prec, stream_ptr):
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    _lib.check(load().ndg_density_vjp(plan, ne, e_ptr, eta, v_ptr, sr, sl, ce_ptr, nbar_ptr,
                                      vbar_ptr, prec, stream_ptr))


def ndg_density_vjp_noalloc(plan, ne, e_ptr, eta, v_ptr, sig_r_ptrs, sig_less_ptrs, ce_ptr, nbar_ptr,
                            vbar_ptr, prec, stream_ptr):
    nc = len(sig_r_ptrs)
    sr = (C.c_void_p * max(1, nc))(*sig_r_ptrs)
    sl = (C.c_void_p * max(1, nc))(*sig_less_ptrs)
    _lib.check(load().ndg_density_vjp_noalloc(plan, ne, e_ptr, eta, v_ptr, sr, sl, ce_ptr, nbar_ptr,
                                              vbar_ptr, prec, stream_ptr))


def ndg_plan_status(plan):
    code, e, cl = C.c_int32(), C.c_int32(), C.c_int32()
    _lib.check(load().ndg_plan_status(plan, C.byref(code), C.byref(e), C.byref(cl)))
    return code.value, e.value, cl.value


def ndg_plan_export_block(plan, which, energy, cluster, count):
    out = np.zeros(max(1, count), np.complex128)
    _lib.check(load().ndg_plan_export_block(plan, which, energy, cluster, out.ctypes.data))
    return out[:count]


def ndg_plan_set_profiling(plan, enable):
    """enable: False/0 off, True/1 on, 2 on with every launch on the caller's
    stream (no overlap between the extractions)."""
    _lib.check(load().ndg_plan_set_profiling(plan, int(enable)))


def _stats(arr, cnt):
    return [{"name": arr[i].name.decode(), "height": arr[i].height,
             "size_class": arr[i].size_class, "launches": arr[i].launches, "ms": arr[i].ms,
             "flops": arr[i].flops, "bytes": arr[i].bytes} for i in range(cnt)]


def ndg_plan_profile(plan) -> list:
    cap = 1 << 16
    arr = (_lib.KernelStat * cap)()
    cnt = C.c_int32()
    _lib.check(load().ndg_plan_profile(plan, cap, arr, C.byref(cnt)))
    return _stats(arr, cnt.value)


def ndg_symbolic_costs(sy) -> list:
    cap = 1 << 16
    arr = (_lib.KernelStat * cap)()
    cnt = C.c_int32()
    _lib.check(load().ndg_symbolic_costs(sy, cap, arr, C.byref(cnt)))
    return _stats(arr, cnt.value)


def ndg_batch_create(plans):
    arr = (C.c_void_p * len(plans))(*[p.value if isinstance(p, C.c_void_p) else p for p in plans])
    out = C.c_void_p()
    _lib.check(load().ndg_batch_create(len(plans), arr, C.byref(out)))
    return out


def ndg_batch_destroy(batch):
    _lib.check(load().ndg_batch_destroy(batch))


def ndg_batch_launches(batch) -> int:
    return int(load().ndg_batch_launches(batch))


def ndg_batch_solve(batch, args, prec, stream_ptr):
    """args: one dict per plan with the ndg_solve arguments as integers
    (device addresses): nE, E, eta, V, sig_r (list), sig_less (list),
    diag_gr, diag_gless, diag_ggreater, growth (None for NULL)."""
    keep = []
    arr = (_lib.SolveArgs * len(args))()
    for k, a in enumerate(args):
        nc = len(a["sig_r"])
        sr = (C.c_void_p * max(1, nc))(*a["sig_r"])
        sl = (C.c_void_p * max(1, nc))(*a["sig_less"])
        keep += [sr, sl]
        arr[k] = _lib.SolveArgs(a["nE"], a["E"], a["eta"], a["V"],
                                C.cast(sr, C.POINTER(C.c_void_p)), C.cast(sl, C.POINTER(C.c_void_p)),
                                a["diag_gr"], a["diag_gless"], a["diag_ggreater"], a["growth"])
    _lib.check(load().ndg_batch_solve(batch, arr, prec, stream_ptr))


def ndg_status_string(code: int) -> str:
    return load().ndg_status_string(code).decode()


def ndg_last_error() -> str:
    return load().ndg_last_error().decode()


# ----------------------------------------------------------------------------
# convenience objects
# ----------------------------------------------------------------------------

class Symbolic:
    """Separator tree and symbolic analysis of one device geometry (host)."""

    def __init__(self, handle, ncontacts, contact_sizes):
        self.handle = handle
        self.ncontacts = ncontacts
        self.contact_sizes = contact_sizes

    def info(self) -> dict:
        return ndg_symbolic_info(self.handle)

    def arrays(self) -> dict:
        return ndg_symbolic_arrays(self.handle)

    def costs(self) -> list:
        """Algorithmic flops and bytes per energy of every launch group
        (kernel, height, size class) of a phonon-free solve."""
        return ndg_symbolic_costs(self.handle)

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "handle", None) and lib is not None:
            lib.ndg_symbolic_destroy(self.handle)
            self.handle = None


def analyze(n, rowptr, col, val, contacts, coords=None, leaf_max=0, max_cluster=0, tree_kind=0,
            slab=0, layers=None, layer_max=0):
    """Separator tree and symbolic analysis.  layers: optional list of site
    arrays in transport order (tree kinds 1 and 3), else layers are the sites
    of equal x coordinate."""
    layer_of = None
    if layers is not None:
        layer_of = np.full(n, -1, dtype=np.int32)
        for q, L in enumerate(layers):
            layer_of[np.asarray(L)] = q
        if (layer_of < 0).any():
            raise ValueError("layers must cover every site")
    h = ndg_analyze(n, rowptr, col, val, contacts, coords, leaf_max, max_cluster, tree_kind, slab,
                    layer_of, layer_max)
    return Symbolic(h, len(contacts), [len(c) for c in contacts])


class Plan:
    """Device workspace for up to max_batch energies in flight."""

    def __init__(self, sym: Symbolic, max_batch: int = 64, device: int = 0):
        self.sym = sym
        self.device = device
        self.handle = ndg_plan_create(sym.handle, max_batch, device)
        self.max_batch = max_batch
        self._info = ndg_plan_info(self.handle)

    def info(self) -> dict:
        return dict(self._info)

    def solve(self, E, eta, sig_r, sig_less, V=None, out=None, prec=NDG_FP64, stream=None,
              growth=None):
        """E: float64 [nE]; sig_r / sig_less: lists of complex128 [nE, nc, nc];
        V: float64 [n] or None; all torch tensors on this plan's GPU.  Returns
        (diag G^r, diag G^<, diag G^>) as complex128 [nE, n] tensors.
        growth: optional float64 [nE] tensor receiving, per energy, the
        largest ||A_ii^{-1}|| ||A_iB|| over the clusters (bound of ||Psi||)."""
        import torch
        n = self._info["n"]
        ne = int(E.shape[0])
        dev = E.device
        if dev.type != "cuda":
            raise ValueError("inputs must be GPU tensors")
        for t in list(sig_r) + list(sig_less) + ([V] if V is not None else []):
            if t.device != dev or not t.is_contiguous():
                raise ValueError("all inputs must be contiguous tensors on the plan's device")
        if E.dtype != torch.float64 or not E.is_contiguous():
            raise ValueError("E must be a contiguous float64 tensor")
        for k, (a, b) in enumerate(zip(sig_r, sig_less)):
            ncs = self.sym.contact_sizes[k]
            for t in (a, b):
                if t.dtype != torch.complex128 or tuple(t.shape) != (ne, ncs, ncs):
                    raise ValueError("contact %d self-energy must be complex128 [nE, %d, %d]"
                                     % (k, ncs, ncs))
        if V is not None and (V.dtype != torch.float64 or V.numel() != n):
            raise ValueError("V must be float64 [n]")
        if out is None:
            out = tuple(torch.empty((ne, n), dtype=torch.complex128, device=dev) for _ in range(3))
        gr, gl, gg = out
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        ndg_solve(self.handle, ne, E.data_ptr(), float(eta), V.data_ptr() if V is not None else None,
                  [t.data_ptr() for t in sig_r], [t.data_ptr() for t in sig_less],
                  gr.data_ptr(), gl.data_ptr(), gg.data_ptr() if gg is not None else None,
                  growth.data_ptr() if growth is not None else None,
                  prec, C.c_void_p(st.cuda_stream))
        return gr, gl, gg

    def solve_transport(self, E, eta, sig_r, sig_less, V=None, greater=True, transmission=True,
                        growth=None, stream=None):
        """FP64 solve plus G^> in its own step (G^r Sigma^> G^r+) and the
        transmission T(E) between the two contacts.  Returns (diag G^r,
        diag G^<, diag G^> or None, T or None)."""
        import torch
        n, ne, dev = self._check_inputs(E, sig_r, sig_less, V)
        gr, gl = (torch.empty((ne, n), dtype=torch.complex128, device=dev) for _ in range(2))
        gg = torch.empty((ne, n), dtype=torch.complex128, device=dev) if greater else None
        T = torch.empty(ne, dtype=torch.float64, device=dev) if transmission else None
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        ndg_solve_transport(self.handle, ne, E.data_ptr(), float(eta),
                            V.data_ptr() if V is not None else None,
                            [t.data_ptr() for t in sig_r], [t.data_ptr() for t in sig_less],
                            gr.data_ptr(), gl.data_ptr(), gg.data_ptr() if greater else None,
                            T.data_ptr() if transmission else None,
                            growth.data_ptr() if growth is not None else None, C.c_void_p(st.cuda_stream))
        return gr, gl, gg, T

    def _check_inputs(self, E, sig_r, sig_less, V):
        import torch
        n = self._info["n"]
        ne = int(E.shape[0])
        dev = E.device
        if dev.type != "cuda":
            raise ValueError("inputs must be GPU tensors")
        if E.dtype != torch.float64 or not E.is_contiguous():
            raise ValueError("E must be a contiguous float64 tensor")
        for t in list(sig_r) + list(sig_less) + ([V] if V is not None else []):
            if t.device != dev or not t.is_contiguous():
                raise ValueError("all inputs must be contiguous tensors on the plan's device")
        for k, (a, b) in enumerate(zip(sig_r, sig_less)):
            ncs = self.sym.contact_sizes[k]
            for t in (a, b):
                if t.dtype != torch.complex128 or tuple(t.shape) != (ne, ncs, ncs):
                    raise ValueError("contact %d self-energy must be complex128 [nE, %d, %d]"
                                     % (k, ncs, ncs))
        if V is not None and (V.dtype != torch.float64 or V.numel() != n):
            raise ValueError("V must be float64 [n]")
        return n, ne, dev

    def density(self, E, eta, sig_r, sig_less, cE, V=None, out=None, prec=NDG_FP64, stream=None):
        """n_i = sum_E cE (-i G^<_ii); float64 [n] on the GPU."""
        import torch
        n, ne, dev = self._check_inputs(E, sig_r, sig_less, V)
        if cE.dtype != torch.float64 or cE.numel() != ne or cE.device != dev:
            raise ValueError("cE must be float64 [nE] on the plan's device")
        out = torch.empty(n, dtype=torch.float64, device=dev) if out is None else out
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        ndg_density(self.handle, ne, E.data_ptr(), float(eta), V.data_ptr() if V is not None else None,
                    [t.data_ptr() for t in sig_r], [t.data_ptr() for t in sig_less],
                    cE.data_ptr(), out.data_ptr(), prec, C.c_void_p(st.cuda_stream))
        return out

    def enable_adjoint(self):
        ndg_plan_enable_adjoint(self.handle)

    def poisson_newton_step(self, E, eta, sig_r, sig_less, cE, V, k_rowptr, k_col, k_val, beta, nd,
                            cg_tol=1e-10, cg_max_iter=200, out=None, stream=None):
        """Newton step of the Schroedinger-Poisson problem (ndg_poisson_newton_step):
        K given as a CSR (int64 rowptr, int32 col, float64 val tensors on
        the GPU), nd float64 [n].  Returns (delta, ||F||, cg iterations,
        final relative residual); enable_adjoint() first."""
        import torch
        n, ne, dev = self._check_inputs(E, sig_r, sig_less, V)
        if V is None:
            raise ValueError("V is required")
        for t, dt in ((cE, torch.float64), (k_rowptr, torch.int64), (k_col, torch.int32),
                      (k_val, torch.float64), (nd, torch.float64)):
            if t.dtype != dt or t.device != dev or not t.is_contiguous():
                raise ValueError("cE, K and nd must be contiguous tensors on the plan's device "
                                 "(float64 / int64 / int32 / float64 / float64)")
        if k_rowptr.numel() != n + 1 or nd.numel() != n or cE.numel() != ne:
            raise ValueError("K must be n x n CSR, nd [n], cE [nE]")
        out = torch.empty(n, dtype=torch.float64, device=dev) if out is None else out
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        fn, it, res = ndg_poisson_newton_step(
            self.handle, ne, E.data_ptr(), float(eta), V.data_ptr(), [t.data_ptr() for t in sig_r],
            [t.data_ptr() for t in sig_less], cE.data_ptr(), k_rowptr.data_ptr(), k_col.data_ptr(),
            k_val.data_ptr(), int(k_col.numel()), float(beta), nd.data_ptr(), float(cg_tol), int(cg_max_iter),
            out.data_ptr(),
            C.c_void_p(st.cuda_stream))
        return out, fn, it, res

    def enable_scattering(self):
        ndg_plan_enable_scattering(self.handle)
        self._info = ndg_plan_info(self.handle)

    def scba(self, E, eta, sig_r, sig_less, d0, mix=0.7, tol=1e-10, max_iter=100, sig_r_ph=None,
             sig_less_ph=None, V=None, out=None, stream=None, current=None):
        """Self-consistent Born loop (local elastic scattering, ndg_scba).
        sig_r_ph / sig_less_ph: starting complex128 [nE, n] tensors, updated
        in place (zeros when None).  current: optional float64
        [nE, ncontacts] tensor receiving the terminal current spectral
        density of the last solve.  Returns (diag G^r, diag G^<, diag G^>,
        sig_r_ph, sig_less_ph, iterations, residual)."""
        import torch
        n, ne, dev = self._check_inputs(E, sig_r, sig_less, V)
        ph = []
        for t in (sig_r_ph, sig_less_ph):
            if t is None:
                t = torch.zeros((ne, n), dtype=torch.complex128, device=dev)
            elif (t.dtype != torch.complex128 or tuple(t.shape) != (ne, n) or t.device != dev
                  or not t.is_contiguous()):
                raise ValueError("phonon self-energies must be contiguous complex128 [nE, n] "
                                 "tensors on the plan's device")
            ph.append(t)
        if out is None:
            out = tuple(torch.empty((ne, n), dtype=torch.complex128, device=dev) for _ in range(3))
        gr, gl, gg = out
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        it, res = ndg_scba(self.handle, ne, E.data_ptr(), float(eta),
                           V.data_ptr() if V is not None else None,
                           [t.data_ptr() for t in sig_r], [t.data_ptr() for t in sig_less],
                           float(d0), float(mix), float(tol), int(max_iter), ph[0].data_ptr(),
                           ph[1].data_ptr(), gr.data_ptr(), gl.data_ptr(),
                           gg.data_ptr() if gg is not None else None,
                           self._current_ptr(current, ne, dev), C.c_void_p(st.cuda_stream))
        return gr, gl, gg, ph[0], ph[1], it, res

    def _current_ptr(self, current, ne, dev):
        import torch
        if current is None:
            return None
        nc = len(self.sym.contact_sizes)
        if (current.dtype != torch.float64 or tuple(current.shape) != (ne, nc) or current.device != dev
                or not current.is_contiguous()):
            raise ValueError("current must be a contiguous float64 [nE, ncontacts] tensor on the "
                             "plan's device")
        return current.data_ptr()

    def solve_scattering(self, E, eta, sig_r, sig_less, sig_r_ph=None, sig_less_ph=None, V=None,
                         out=None, stream=None, growth=None, current=None):
        """solve() in FP64 with diagonal phonon self-energies sig_r_ph,
        sig_less_ph: complex128 [nE, n] tensors on the plan's GPU (caller's
        site order) or None.  sig_less_ph needs enable_scattering() first.
        current: optional float64 [nE, ncontacts] tensor receiving the
        terminal current spectral density Tr[S^<_c G^>_cc - S^>_c G^<_cc]."""
        import torch
        n, ne, dev = self._check_inputs(E, sig_r, sig_less, V)
        for t in (sig_r_ph, sig_less_ph):
            if t is not None and (t.dtype != torch.complex128 or tuple(t.shape) != (ne, n)
                                  or t.device != dev or not t.is_contiguous()):
                raise ValueError("phonon self-energies must be contiguous complex128 [nE, n] "
                                 "tensors on the plan's device")
        if out is None:
            out = tuple(torch.empty((ne, n), dtype=torch.complex128, device=dev) for _ in range(3))
        gr, gl, gg = out
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        ndg_solve_scattering(self.handle, ne, E.data_ptr(), float(eta),
                             V.data_ptr() if V is not None else None,
                             [t.data_ptr() for t in sig_r], [t.data_ptr() for t in sig_less],
                             sig_r_ph.data_ptr() if sig_r_ph is not None else None,
                             sig_less_ph.data_ptr() if sig_less_ph is not None else None,
                             gr.data_ptr(), gl.data_ptr(), gg.data_ptr() if gg is not None else None,
                             growth.data_ptr() if growth is not None else None,
                             self._current_ptr(current, ne, dev), C.c_void_p(st.cuda_stream))
        return gr, gl, gg

    def density_vjp(self, E, eta, sig_r, sig_less, cE, nbar, V=None, out=None, prec=NDG_FP64,
                    stream=None, noalloc=False):
        """(d n / d V)^T nbar; float64 [n] on the GPU.  noalloc: through
        ndg_density_vjp_noalloc (the partials in the library's static device
        buffer; out must then be given, so nothing is allocated)."""
        import torch
        n, ne, dev = self._check_inputs(E, sig_r, sig_less, V)
        if nbar.dtype != torch.float64 or nbar.numel() != n or not nbar.is_contiguous():
            raise ValueError("nbar must be a contiguous float64 [n] tensor")
        out = torch.empty(n, dtype=torch.float64, device=dev) if out is None else out
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        fn = ndg_density_vjp_noalloc if noalloc else ndg_density_vjp
        fn(self.handle, ne, E.data_ptr(), float(eta),
                        V.data_ptr() if V is not None else None,
                        [t.data_ptr() for t in sig_r], [t.data_ptr() for t in sig_less],
                        cE.data_ptr(), nbar.data_ptr(), out.data_ptr(), prec,
                        C.c_void_p(st.cuda_stream))
        return out

    def status(self):
        return ndg_plan_status(self.handle)

    def set_profiling(self, enable):
        ndg_plan_set_profiling(self.handle, enable)

    def profile(self) -> list:
        return ndg_plan_profile(self.handle)

    def export_block(self, which: int, energy: int, cluster: int, shape):
        cnt = int(np.prod(shape))
        return ndg_plan_export_block(self.handle, which, energy, cluster, cnt).reshape(shape)

    def __del__(self):
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "handle", None) and lib is not None:
            lib.ndg_plan_destroy(self.handle)
            self.handle = None


class Batch:
    """Several devices (plans) of uneven sizes solved by one graph launch.

    solve() takes one tuple (E, eta, sig_r, sig_less, V) per plan and
    returns one (diag G^r, diag G^<, diag G^>) per plan.  Outputs are kept
    per batch and reused, so that repeated calls with the same input tensors
    replay the captured graph; copy results that must survive the next call."""

    def __init__(self, plans):
        self.plans = list(plans)
        self.handle = ndg_batch_create([p.handle for p in self.plans])
        self._outs = None
        self._stream = None

    def solve(self, inputs, prec=NDG_FP64, growth=None):
        """growth: optional list (one per plan) of float64 [nE] tensors that
        receive the per-energy growth indicator, as in Plan.solve."""
        import torch
        if len(inputs) != len(self.plans):
            raise ValueError("one input tuple per plan")
        shapes = []
        for p, (E, eta, sig_r, sig_less, V) in zip(self.plans, inputs):
            n, ne, dev = p._check_inputs(E, sig_r, sig_less, V)
            shapes.append((ne, n, dev))
        if self._outs is None or [tuple(o[0].shape) for o in self._outs] != [s[:2] for s in shapes]:
            self._outs = [tuple(torch.empty((ne, n), dtype=torch.complex128, device=dev)
                                for _ in range(3)) for ne, n, dev in shapes]
        if self._stream is None:
            # graph capture needs a created stream, not the legacy default one
            self._stream = torch.cuda.Stream(device=shapes[0][2])
        cur = torch.cuda.current_stream(shapes[0][2])
        self._stream.wait_stream(cur)
        args = []
        growth = growth if growth is not None else [None] * len(self.plans)
        for (E, eta, sig_r, sig_less, V), (gr, gl, gg), g in zip(inputs, self._outs, growth):
            args.append({"nE": int(E.shape[0]), "E": E.data_ptr(), "eta": float(eta),
                         "V": V.data_ptr() if V is not None else None,
                         "sig_r": [t.data_ptr() for t in sig_r],
                         "sig_less": [t.data_ptr() for t in sig_less],
                         "diag_gr": gr.data_ptr(), "diag_gless": gl.data_ptr(),
                         "diag_ggreater": gg.data_ptr(),
                         "growth": g.data_ptr() if g is not None else None})
        ndg_batch_solve(self.handle, args, prec, C.c_void_p(self._stream.cuda_stream))
        cur.wait_stream(self._stream)
        return list(self._outs)

    def launches(self) -> int:
        """Graph launches of the last solve (1: the whole energy range as one graph)."""
        return ndg_batch_launches(self.handle)

    def __del__(self):
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "handle", None) and lib is not None:
            lib.ndg_batch_destroy(self.handle)
            self.handle = None


def _autograd_function():
    import torch

    class NDDensity(torch.autograd.Function):
        """density = NDDensity.apply(V, plan, E, eta, sig_r, sig_less, cE).

        Forward: n_i(V) = sum_E cE (-i G^<_ii) by the library's fold and
        extraction.  Backward: the library's adjoint (ndg_density_vjp) gives
        Vbar = J^T nbar.  sig_r / sig_less are tuples of tensors treated as
        constants."""

        @staticmethod
        def forward(ctx, V, plan, E, eta, sig_r, sig_less, cE):
            ctx.plan, ctx.eta = plan, eta
            ctx.sig_r, ctx.sig_less = tuple(sig_r), tuple(sig_less)
            ctx.save_for_backward(V, E, cE)
            return plan.density(E, eta, sig_r, sig_less, cE, V=V.contiguous())

        @staticmethod
        def backward(ctx, nbar):
            V, E, cE = ctx.saved_tensors
            vbar = ctx.plan.density_vjp(E, ctx.eta, ctx.sig_r, ctx.sig_less, cE,
                                        nbar.contiguous().to(torch.float64), V=V.contiguous())
            return vbar, None, None, None, None, None, None

    return NDDensity


class _LazyFunction:
    _fn = None

    def apply(self, *args):
        if _LazyFunction._fn is None:
            _LazyFunction._fn = _autograd_function()
        return _LazyFunction._fn.apply(*args)


NDDensity = _LazyFunction()
