"""The Python binding rejects arguments the library would read or write out of
bounds, before any call into the library (CPU only: the checks run first)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"the library was called ({name}) despite an invalid argument")


def _solver_stub(n_b=10):
    from paper_2201_01970_amd.solver import Solver

    S = Solver.__new__(Solver)
    S._lib = _NoLib()
    S._h = None
    S.n_b = n_b
    S.nnz_b = 3 * n_b
    S.device = torch.device("cuda", 0)
    return S


def test_solve_rejects_host_wrong_dtype_and_wrong_length():
    S = _solver_stub()
    with pytest.raises(ValueError, match="must live on"):
        S.solve(torch.zeros(30, dtype=torch.float64))
    with pytest.raises(ValueError, match="torch tensor"):
        S.solve(np.zeros(30))
    for call in (S.spmv, S.precond):
        with pytest.raises(ValueError):
            call(torch.zeros(30, dtype=torch.float32))
    with pytest.raises(ValueError):
        S.vcycle(torch.zeros(10, dtype=torch.float64))


def test_vector_check_messages():
    from paper_2201_01970_amd.solver import _check_device_vec

    t = torch.zeros(12, dtype=torch.float64)
    with pytest.raises(ValueError, match="must live on"):
        _check_device_vec(t, 12, "b", torch.device("cuda", 0))


def test_matrix_value_count_checked():
    S = _solver_stub()
    rp = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([0, 1], dtype=np.int32)
    with pytest.raises(ValueError, match="9 \\* nnz_blocks"):
        S._as_bsr(rp, col, np.zeros(17))
    with pytest.raises(ValueError, match="9 \\* nnz_blocks"):
        S._as_bsr(rp, col, torch.zeros(19, dtype=torch.float64))
    with pytest.raises(ValueError, match="at least two"):
        S._as_bsr(np.array([0], dtype=np.int32), col, np.zeros(18))
    S._as_bsr(rp, col, np.zeros(18))  # consistent sizes pass


def test_server_submit_checks_sizes():
    from paper_2201_01970_amd.serve import Server

    srv = Server.__new__(Server)
    srv._lib = _NoLib()
    srv._h = None
    srv._live = {}
    rp = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([0, 1], dtype=np.int32)
    with pytest.raises(ValueError, match="vals"):
        srv.submit(1, rp, col, np.zeros(10), np.zeros(6))
    with pytest.raises(ValueError, match="b must hold"):
        srv.submit(1, rp, col, np.zeros(18), np.zeros(5))
