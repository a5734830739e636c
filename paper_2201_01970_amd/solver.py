"""Python face of the C ABI: a handle wrapper over torch device memory.

Only argument marshalling happens here; SETUP and every step of the solve run
inside libcpr_mi355x.so.  Device vectors are torch tensors on the current HIP
device; the handle works on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _capi as A


@dataclass
class Params:
    restart: int = 30
    max_restarts: int = 100
    theta_rs: float = 0.25
    theta_color: float = 0.05
    coarse_max: int = 50
    max_levels: int = 25
    pre_sweeps: int = 2
    post_sweeps: int = 2
    precond_fp32: bool = False
    reuse_mode: int = 2
    mu: int = 20
    reuse_factor: float = 1.3
    use_graphs: bool = True
    tail_nnz: int = 30000
    row_layout: int = 0
    second_stage: int = 0   # 0 block Gauss-Seidel, 1 block ILU(0)
    decoupling: int = 0     # 0 none, 1 quasi-IMPES, 2 ABF
    smoother: int = 0       # 0 PGS-SCM, 1 PGS-NO
    smoother_chunks: int = 256
    amg_kind: int = 0       # 0 RS AMG + V-cycle, 1 UA-AMG (pairwise matching) + nonlinear AMLI-cycle
    amli_inner: int = 2
    npair: int = 2
    pair_beta: float = 0.25
    coarse_solver: int = 0  # RS coarsest: 0 LU in the one-workgroup kernel, 1 explicit inverse (dense product)

    def to_c(self) -> A.cpr_params:
        p = A.cpr_params()
        for name, _ in A.cpr_params._fields_:
            setattr(p, name, getattr(self, name))
        p.precond_fp32 = int(bool(self.precond_fp32))
        p.use_graphs = int(bool(self.use_graphs))
        return p


def _torch():
    import torch

    return torch


def _host(arr):
    """A numpy view (or host copy) of a numpy array or torch tensor."""
    return arr if isinstance(arr, np.ndarray) else arr.detach().cpu().numpy()


def _check_device_vec(t, n, name, device):
    """Raise ValueError unless t is a contiguous float64 tensor of n entries on
    the handle's HIP device: the library reads and writes it as double[n]."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor on the GPU, got {type(t).__name__}")
    if not t.is_cuda or (device is not None and t.device != device):
        raise ValueError(f"{name} must live on {device}, got {t.device}")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must hold {n} entries, got {t.numel()}")


def _check_bsr_sizes(n, nnz, n_vals):
    if n < 1:
        raise ValueError("row_ptr must hold at least two entries")
    if nnz < 1:
        raise ValueError("col must not be empty")
    if n_vals != 9 * nnz:
        raise ValueError(f"vals must hold 9 * nnz_blocks = {9 * nnz} entries, got {n_vals}")


def _ptr(arr):
    """Address of a contiguous numpy array or torch tensor."""
    if isinstance(arr, np.ndarray):
        assert arr.flags.c_contiguous
        return arr.ctypes.data
    assert arr.is_contiguous()
    return arr.data_ptr()


class Solver:
    """CPR-FGMRES handle for one 3x3-block sparsity pattern (cpr_setup)."""

    def __init__(self, row_ptr, col, vals, params: Params | None = None, stream=None):
        torch = _torch()
        self._lib = A.lib()
        self.params = params or Params()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._keep = self._as_bsr(row_ptr, col, vals)
        self.n_b = int(self._bsr.n_block_rows)
        self.nnz_b = int(self._bsr.nnz_blocks)
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        h = C.c_void_p()
        pc = self.params.to_c()
        st = self._lib.cpr_setup(C.byref(self._bsr), C.byref(pc), C.c_void_p(s.cuda_stream), C.byref(h))
        A.check(st, None)
        self._h = h

    def _as_bsr(self, row_ptr, col, vals):
        torch = _torch()
        # one memory location covers the three arrays: the pattern follows the values
        if isinstance(vals, np.ndarray):
            rp = np.ascontiguousarray(_host(row_ptr), dtype=np.int32)
            cl = np.ascontiguousarray(_host(col), dtype=np.int32)
            vv = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1)
            loc = A.CPR_MEM_HOST
        else:
            rp = torch.as_tensor(row_ptr).to(dtype=torch.int32).contiguous()
            cl = torch.as_tensor(col).to(dtype=torch.int32).contiguous()
            vv = vals.to(dtype=torch.float64).contiguous().reshape(-1)
            loc = A.CPR_MEM_DEVICE if vv.is_cuda else A.CPR_MEM_HOST
            rp, cl = rp.to(vv.device), cl.to(vv.device)
        n = int(rp.shape[0]) - 1
        nnz = int(cl.shape[0])
        _check_bsr_sizes(n, nnz, int(vv.shape[0]))
        self._bsr = A.cpr_bsr(n, nnz, 3, _ptr(rp), _ptr(cl), _ptr(vv), loc)
        return (rp, cl, vv)

    # ------------------------------------------------------------------ API
    def update_values(self, vals, row_ptr=None, col=None):
        rp = self._keep[0] if row_ptr is None else row_ptr
        cl = self._keep[1] if col is None else col
        keep = self._as_bsr(rp, cl, vals)
        st = self._lib.cpr_update_values(self._h, C.byref(self._bsr))
        A.check(st, self._h)
        self._keep = keep

    def solve(self, b, x=None, tol=1e-6, allow_not_converged=False, noalloc=False):
        """noalloc=True calls cpr_solve_noalloc (no device allocation inside the
        call; x must then be given, and the caller owns both vectors)."""
        torch = _torch()
        _check_device_vec(b, 3 * self.n_b, "b", self.device)
        if x is None:
            if noalloc:
                raise ValueError("noalloc solve needs a caller-allocated x")
            x = torch.zeros_like(b)
        _check_device_vec(x, 3 * self.n_b, "x", self.device)
        info = A.cpr_solve_info()
        fn = self._lib.cpr_solve_noalloc if noalloc else self._lib.cpr_solve
        st = fn(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol), C.byref(info))
        allow = (A.CPR_OK, A.CPR_NOT_CONVERGED) if allow_not_converged else (A.CPR_OK,)
        A.check(st, self._h, allow)
        d = info.as_dict()
        d["status"] = A.status_name(st)
        return x, d

    def spmv(self, x, y=None):
        torch = _torch()
        _check_device_vec(x, 3 * self.n_b, "x", self.device)
        y = torch.empty_like(x) if y is None else y
        _check_device_vec(y, 3 * self.n_b, "y", self.device)
        A.check(self._lib.cpr_spmv(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())), self._h)
        return y

    def precond(self, v, z=None):
        torch = _torch()
        _check_device_vec(v, 3 * self.n_b, "v", self.device)
        z = torch.empty_like(v) if z is None else z
        _check_device_vec(z, 3 * self.n_b, "z", self.device)
        A.check(self._lib.cpr_precond_apply(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(z.data_ptr())), self._h)
        return z

    def second_stage(self, v, pe, z=None):
        """z = Pi_P pe + R (v - A Pi_P pe) with the handle's second stage."""
        torch = _torch()
        _check_device_vec(v, 3 * self.n_b, "v", self.device)
        _check_device_vec(pe, self.n_b, "pe", self.device)
        z = torch.empty_like(v) if z is None else z
        _check_device_vec(z, 3 * self.n_b, "z", self.device)
        A.check(self._lib.cpr_second_stage(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(pe.data_ptr()),
                                           C.c_void_p(z.data_ptr())), self._h)
        return z

    def bilu_factors(self):
        """Host copies of the block ILU(0) factors: dict with lu [nnz,3,3],
        uinv [n,3,3], flev, blev [n] and the two level counts."""
        lu = np.empty((self.nnz_b, 3, 3))
        uinv = np.empty((self.n_b, 3, 3))
        flev = np.empty(self.n_b, dtype=np.int32)
        blev = np.empty(self.n_b, dtype=np.int32)
        nl = np.zeros(2, dtype=np.int32)
        A.check(self._lib.cpr_bilu_factors(self._h, lu.ctypes.data, uinv.ctypes.data, flev.ctypes.data,
                                           blev.ctypes.data, nl.ctypes.data), self._h)
        return dict(lu=lu, uinv=uinv, flev=flev, blev=blev, n_flev=int(nl[0]), n_blev=int(nl[1]))

    def vcycle(self, r, e=None):
        torch = _torch()
        _check_device_vec(r, self.n_b, "r", self.device)
        e = torch.empty_like(r) if e is None else e
        _check_device_vec(e, self.n_b, "e", self.device)
        A.check(self._lib.cpr_vcycle(self._h, C.c_void_p(r.data_ptr()), C.c_void_p(e.data_ptr())), self._h)
        return e

    def smooth(self, level, x, b, sweeps=1, zero_start=False):
        n = self.level_info(level)["n"]
        _check_device_vec(x, n, "x", self.device)
        _check_device_vec(b, n, "b", self.device)
        A.check(self._lib.cpr_smooth(self._h, int(level), C.c_void_p(x.data_ptr()), C.c_void_p(b.data_ptr()),
                                     int(sweeps), int(bool(zero_start))), self._h)
        return x

    def level_info(self, level):
        out = np.zeros(8, dtype=np.int64)
        A.check(self._lib.cpr_level_info(self._h, int(level), out.ctypes.data), self._h)
        keys = ("n", "nnz", "n_colours", "n_coarse", "is_coarsest", "n_levels", "nnz_p", "n_block_colours")
        return dict(zip(keys, (int(v) for v in out)))

    def level_arrays(self, level):
        info = self.level_info(level)
        n, nnz = info["n"], info["nnz"]
        rp = np.zeros(n + 1, dtype=np.int32)
        cl = np.zeros(nnz, dtype=np.int32)
        va = np.zeros(nnz, dtype=np.float64)
        rs = np.zeros(nnz, dtype=np.uint8)
        cs = np.zeros(nnz, dtype=np.uint8)
        colour = np.full(n, -1, dtype=np.int32)
        cf = np.zeros(n, dtype=np.int8)
        coarsest = info["is_coarsest"] == 1
        A.check(self._lib.cpr_level_arrays(self._h, int(level), rp.ctypes.data, cl.ctypes.data, va.ctypes.data,
                                           None if coarsest else rs.ctypes.data,
                                           None if coarsest else cs.ctypes.data,
                                           None if coarsest else colour.ctypes.data,
                                           None if coarsest else cf.ctypes.data), self._h)
        out = dict(row_ptr=rp, col=cl, val=va)
        if not coarsest:
            out.update(rs_strong=rs.astype(bool), color_strong=cs.astype(bool), colour=colour, cf=cf)
        return out

    def level_aggregates(self, level):
        agg = np.empty(self.level_info(level)["n"], dtype=np.int32)
        A.check(self._lib.cpr_level_aggregates(self._h, int(level), agg.ctypes.data), self._h)
        return agg

    def level_interp(self, level):
        info = self.level_info(level)
        rp = np.zeros(info["n"] + 1, dtype=np.int32)
        cl = np.zeros(info["nnz_p"], dtype=np.int32)
        va = np.zeros(info["nnz_p"], dtype=np.float64)
        A.check(self._lib.cpr_level_interp(self._h, int(level), rp.ctypes.data, cl.ctypes.data, va.ctypes.data),
                self._h)
        return rp, cl, va

    def block_colours(self):
        c = np.zeros(self.n_b, dtype=np.int32)
        A.check(self._lib.cpr_block_colours(self._h, c.ctypes.data), self._h)
        return c

    def device_bytes(self):
        return int(self._lib.cpr_device_bytes(self._h))

    def profile(self, enable: bool):
        A.check(self._lib.cpr_profile_enable(self._h, int(bool(enable))), self._h)

    def profile_read(self, kind):
        n = C.c_int64()
        ms = C.c_double()
        by = C.c_double()
        A.check(self._lib.cpr_profile_read(self._h, int(kind), C.byref(n), C.byref(ms), C.byref(by)), self._h)
        return int(n.value), float(ms.value), float(by.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cpr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- host-only helpers
def host_grouping(s_ptr, s_col):
    s_ptr = np.ascontiguousarray(s_ptr, dtype=np.int32)
    s_col = np.ascontiguousarray(s_col, dtype=np.int32)
    n = s_ptr.shape[0] - 1
    colour = np.zeros(max(n, 1), dtype=np.int32)
    nc = C.c_int32()
    A.check(A.lib().cpr_host_grouping(n, s_ptr.ctypes.data, s_col.ctypes.data if s_col.size else None,
                                      colour.ctypes.data, C.byref(nc)))
    return colour[:n], int(nc.value)


def host_rs_split(s_ptr, s_col):
    s_ptr = np.ascontiguousarray(s_ptr, dtype=np.int32)
    s_col = np.ascontiguousarray(s_col, dtype=np.int32)
    n = s_ptr.shape[0] - 1
    cf = np.zeros(max(n, 1), dtype=np.int8)
    A.check(A.lib().cpr_host_rs_split(n, s_ptr.ctypes.data, s_col.ctypes.data if s_col.size else None,
                                      cf.ctypes.data))
    return cf[:n]


def host_interpolation(a_ptr, a_col, a_val, strong, cf):
    a_ptr = np.ascontiguousarray(a_ptr, dtype=np.int32)
    a_col = np.ascontiguousarray(a_col, dtype=np.int32)
    a_val = np.ascontiguousarray(a_val, dtype=np.float64)
    strong = np.ascontiguousarray(strong, dtype=np.uint8)
    cf = np.ascontiguousarray(cf, dtype=np.int8)
    n = a_ptr.shape[0] - 1
    p_ptr = np.zeros(n + 1, dtype=np.int32)
    p_col = np.zeros(max(1, a_col.size), dtype=np.int32)
    p_val = np.zeros(max(1, a_col.size), dtype=np.float64)
    nc = C.c_int32()
    A.check(A.lib().cpr_host_interpolation(n, a_ptr.ctypes.data, a_col.ctypes.data, a_val.ctypes.data,
                                           strong.ctypes.data, cf.ctypes.data, p_ptr.ctypes.data,
                                           p_col.ctypes.data, p_val.ctypes.data, C.byref(nc)))
    nnz = int(p_ptr[-1])
    return p_ptr, p_col[:nnz].copy(), p_val[:nnz].copy(), int(nc.value)


def host_galerkin(a_ptr, a_col, a_val, p_ptr, p_col, p_val, n_coarse):
    args = [np.ascontiguousarray(a, dtype=t) for a, t in
            ((a_ptr, np.int32), (a_col, np.int32), (a_val, np.float64), (p_ptr, np.int32), (p_col, np.int32),
             (p_val, np.float64))]
    a_ptr, a_col, a_val, p_ptr, p_col, p_val = args
    n = a_ptr.shape[0] - 1
    c_ptr = np.zeros(n_coarse + 1, dtype=np.int32)
    L = A.lib()
    ptrs = [a.ctypes.data for a in args]
    A.check(L.cpr_host_galerkin(n, n_coarse, *ptrs, c_ptr.ctypes.data, None, None))
    nnz = int(c_ptr[-1])
    c_col = np.zeros(max(nnz, 1), dtype=np.int32)
    c_val = np.zeros(max(nnz, 1), dtype=np.float64)
    A.check(L.cpr_host_galerkin(n, n_coarse, *ptrs, c_ptr.ctypes.data, c_col.ctypes.data, c_val.ctypes.data))
    return c_ptr, c_col[:nnz], c_val[:nnz]
