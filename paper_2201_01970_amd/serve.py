"""Python face of the serving runtime (include/cpr_serve.h): argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as A
from .solver import Params


class Server:
    """Continuous-batching solve server on the current HIP device."""

    def __init__(self, budget_bytes: int, max_slots: int = 4, params: Params | None = None):
        self._lib = A.lib()
        self.params = params or Params()
        h = C.c_void_p()
        pc = self.params.to_c()
        A.check(self._lib.cpr_server_create(int(budget_bytes), int(max_slots), C.byref(pc), C.byref(h)))
        self._h = h
        self._live = {}  # ticket -> arrays that must outlive the request

    def submit(self, case_id, row_ptr, col, vals, b, tol=1e-6):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vv = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1)
        bb = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        n, nnz = rp.shape[0] - 1, cl.shape[0]
        # the library reads vals as double[9 * nnz] and b, x as double[3 * n]
        if n < 1 or nnz < 1:
            raise ValueError("row_ptr must hold at least two entries and col at least one")
        if vv.shape[0] != 9 * nnz:
            raise ValueError(f"vals must hold 9 * nnz_blocks = {9 * nnz} entries, got {vv.shape[0]}")
        if bb.shape[0] != 3 * n:
            raise ValueError(f"b must hold 3 * n_block_rows = {3 * n} entries, got {bb.shape[0]}")
        x = np.zeros_like(bb)
        req = A.cpr_request(int(case_id), A.cpr_bsr(rp.shape[0] - 1, cl.shape[0], 3, rp.ctypes.data,
                                                   cl.ctypes.data, vv.ctypes.data, A.CPR_MEM_HOST),
                            bb.ctypes.data, x.ctypes.data, float(tol))
        t = C.c_int64()
        A.check(self._lib.cpr_server_submit(self._h, C.byref(req), C.byref(t)))
        self._live[t.value] = (rp, cl, vv, bb, x)
        return t.value

    def wait(self, ticket):
        info = A.cpr_solve_info()
        lat = C.c_double()
        st = self._lib.cpr_server_wait(self._h, int(ticket), C.byref(info), C.byref(lat))
        arrays = self._live.pop(ticket)
        d = info.as_dict()
        d["status"] = A.status_name(st)
        d["latency_ms"] = float(lat.value)
        if st not in (A.CPR_OK, A.CPR_NOT_CONVERGED):
            d["error"] = self._lib.cpr_server_last_error(self._h).decode()
        return arrays[4], d

    def stats(self):
        s = A.cpr_server_stats()
        A.check(self._lib.cpr_server_stats_get(self._h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cpr_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
