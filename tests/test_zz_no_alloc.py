"""The allocation-free solve (cpr_solve_noalloc) against cpr_solve, on the GPU.

cpr_solve_noalloc runs the same kernels as cpr_solve, launched one by one
instead of replayed from graphs, with the FGMRES scalars and partial sums in
the library's static device array; every sum keeps its order, so the result
must equal cpr_solve's bit for bit, with the same iteration count and
residuals.  Two calls in a row, the second on a smaller system (the static
array keeps the first call's contents), then a restarted solve, the FP32
preconditioner (also with the inverse coarsest level, the aggregation AMG
with the AMLI-cycle, and block ILU(0) as stage 2), and the two refusals: a restart above the array's limit, and
a solve for which the adaptive-setup rule asks a SETUP.
"""
import numpy as np
import pytest

from workloads import blackoil as bo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _solver(case, **kw):
    from paper_2201_01970_amd import Params, Solver

    return Solver(_dev(case.row_ptr), _dev(case.col), _dev(case.vals.reshape(-1)), Params(**kw))


def _reference(case, b, **kw):
    S = _solver(case, **kw)
    x, info = S.solve(_dev(b), tol=1e-6, allow_not_converged=True)
    S.close()
    return x.cpu().numpy(), info


def _noalloc(S, b):
    x = torch.zeros(b.shape[0], dtype=torch.float64, device="cuda")
    x, info = S.solve(_dev(b), x=x, tol=1e-6, noalloc=True, allow_not_converged=True)
    return x.cpu().numpy(), info


def _same(got, want):
    x, info = got
    xr, ir = want
    assert info["iterations"] == ir["iterations"]
    assert info["restarts"] == ir["restarts"]
    assert info["relres_true"] == ir["relres_true"]
    assert np.array_equal(x, xr)


def test_two_calls_in_a_row_second_smaller():
    big = bo.case_spe10_like(seed=1110, shape=(30, 40, 20))
    small = bo.case_small()
    b_big, b_small = bo.rhs(big.ndof, 1111), bo.rhs(small.ndof, 1001)
    print(f"[noalloc] big n_b={big.n_b} small n_b={small.n_b}", flush=True)
    want_big = _reference(big, b_big)
    want_small = _reference(small, b_small)
    S_big, S_small = _solver(big), _solver(small)
    got_big = _noalloc(S_big, b_big)
    got_small = _noalloc(S_small, b_small)
    _same(got_big, want_big)
    _same(got_small, want_small)
    # and once more on the larger system after the smaller one
    _same(_noalloc(S_big, b_big), want_big)
    S_big.close()
    S_small.close()


@pytest.mark.parametrize("kw", [dict(restart=4), dict(precond_fp32=1),
                                dict(precond_fp32=1, coarse_max=120, coarse_solver=1),
                                dict(precond_fp32=1, amg_kind=1, coarse_max=120),
                                dict(precond_fp32=1, second_stage=1)],
                         ids=["restart4", "fp32", "fp32-coarse-inverse", "fp32-aggregation-amli", "fp32-block-ilu0"])
def test_restarted_and_fp32(kw):
    case = bo.case_small(seed=21, shape=(14, 12, 6))
    b = bo.rhs(case.ndof, 22)
    print(f"[noalloc] {kw} n_b={case.n_b}", flush=True)
    want = _reference(case, b, **kw)
    S = _solver(case, **kw)
    _same(_noalloc(S, b), want)
    S.close()
    if "restart" in kw:
        assert want[1]["restarts"] >= 1


def test_refusals():
    from paper_2201_01970_amd import _capi as A

    case = bo.case_small(seed=31, shape=(8, 8, 4))
    b = bo.rhs(case.ndof, 32)
    S = _solver(case, restart=65)
    with pytest.raises(A.CprError, match="exceeds"):
        _noalloc(S, b)
    S.close()

    # reuse_mode 0 asks a SETUP for every new set of values: refused before any
    # state changes, after which cpr_solve runs the SETUP and a repeat solve on
    # the same values is allowed again
    S = _solver(case, reuse_mode=0)
    S.update_values(_dev(case.vals.reshape(-1) * 1.01))
    with pytest.raises(A.CprError, match="SETUP"):
        _noalloc(S, b)
    x, info = S.solve(_dev(b), tol=1e-6)
    assert info["rebuilt"] == 1
    got = _noalloc(S, b)
    assert got[1]["rebuilt"] == 0
    assert got[1]["iterations"] == info["iterations"]
    assert np.array_equal(got[0], x.cpu().numpy())
    S.close()
