"""Degenerate and ragged sizes through the C ABI: one cell, two cells, a
single-level hierarchy (the coarsest level is level 0, so the whole V-cycle
is the dense LU solve inside the one-workgroup kernel), two and three levels
with ragged last SELL slices.  Bars as for the larger cases: FP64 solve with
the oracle's iteration count and iterate within 1e-10 relative; V-cycle
within 1e-12 of the oracle and bit-identical between the per-colour and the
one-workgroup paths; FP32 preconditioner converged to 1e-6 (iterations at
most one more than FP64: these solves take 1-5 iterations, where a 10% band
is below one iteration).  The V-cycle bound widens with the conditioning of
the coarsest matrix: the oracle factors it with LAPACK, the library with its
own partial-pivoting LU, and two backward-stable solves agree to about
n_c * eps * cond(A_c) (≈ 1e-11 for the ill-conditioned 15-cell level).
"""
import numpy as np
import pytest

from oracle import amg, cpr, fgmres
from oracle.sparse import Csr
from workloads import blackoil as bo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(1, 1, 1), (2, 1, 1), (5, 3, 1), (7, 5, 3), (17, 13, 3)]
CHANNEL_SHAPES = [(20, 20, 10), (16, 24, 12)]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _solver(case, **kw):
    from paper_2201_01970_amd import Params, Solver

    return Solver(_dev(case.row_ptr), _dev(case.col), _dev(case.vals.reshape(-1)), Params(**kw))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_small_case_solves_match_oracle(shape):
    case = bo.case_small(seed=5, shape=shape)
    print(f"[shape {shape}] n_b={case.n_b}", flush=True)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A)
    b = bo.rhs(case.ndof, 6)
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)

    S = _solver(case)
    assert S.level_info(0)["n_levels"] == B.amg.n_levels
    x, info = S.solve(_dev(b), tol=1e-6)
    x = x.cpu().numpy()
    assert info["iterations"] == res.iterations
    assert np.linalg.norm(x - res.x) <= 1e-10 * np.linalg.norm(res.x)
    assert info["relres_true"] < 1e-6

    rng = np.random.default_rng(9)
    r = rng.standard_normal(case.n_b)
    want = amg.vcycle(B.amg, r)
    got = S.vcycle(_dev(r)).cpu().numpy()
    Ac = B.amg.levels[-1].A.to_dense()
    tol = max(1e-12, Ac.shape[0] * np.finfo(float).eps * np.linalg.cond(Ac))
    assert np.linalg.norm(got - want) <= tol * np.linalg.norm(want)
    S.close()

    S0 = _solver(case, tail_nnz=0)
    S1 = _solver(case, tail_nnz=10 ** 9)
    assert np.array_equal(S0.vcycle(_dev(r)).cpu().numpy(), S1.vcycle(_dev(r)).cpu().numpy())
    S0.close()
    S1.close()

    S32 = _solver(case, precond_fp32=True)
    x32, info32 = S32.solve(_dev(b), tol=1e-6)
    S32.close()
    assert info32["relres_true"] < 1e-6
    assert info32["iterations"] <= info["iterations"] + 1


@pytest.mark.parametrize("shape", CHANNEL_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_channelised_small_grids_match_oracle(shape):
    """Channelised permeability (1000 mD channels on 1 mD, kz/kx 0.01): 2-3
    colours on level 0 and 5 on the coarse levels, 6-7 levels.  FP64 solve
    with the oracle's iteration count and iterate within 1e-10 relative; the
    smoothers bit for bit on every level, in FP64 and in FP32 (against the
    oracle on float32 arrays); the FP32-preconditioned solve converged with
    iterations within 10%."""
    case = bo.case_channels(seed=21, shape=shape)
    print(f"[channels {shape}] n_b={case.n_b}", flush=True)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A)
    b = bo.rhs(case.ndof, 22)
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)
    S = _solver(case)
    x, info = S.solve(_dev(b), tol=1e-6)
    x = x.cpu().numpy()
    assert info["iterations"] == res.iterations
    assert np.linalg.norm(x - res.x) <= 1e-10 * np.linalg.norm(res.x)
    rng = np.random.default_rng(23)
    for l in range(B.amg.n_levels - 1):
        lev = B.amg.levels[l]
        bb = rng.standard_normal(lev.A.n_rows)
        x0 = rng.standard_normal(lev.A.n_rows)
        want = x0.copy()
        for _ in range(2):
            amg.colour_sweep(lev.A, lev.colours, want, bb)
        got = S.smooth(l, _dev(x0.copy()), _dev(bb), sweeps=2, zero_start=False).cpu().numpy()
        assert np.array_equal(got, want), l
    S.close()

    # the FP32 preconditioner: sweeps against the oracle's sweep on float32 arrays
    S32 = _solver(case, precond_fp32=True)
    for l in range(B.amg.n_levels - 1):
        lev = B.amg.levels[l]
        A32 = Csr(lev.A.n_rows, lev.A.n_cols, lev.A.indptr, lev.A.indices, lev.A.data.astype(np.float32))
        bb = rng.standard_normal(lev.A.n_rows)
        x0 = rng.standard_normal(lev.A.n_rows)
        want = x0.astype(np.float32)
        for _ in range(2):
            amg.colour_sweep(A32, lev.colours, want, bb.astype(np.float32), lev.diag.astype(np.float32))
        got = S32.smooth(l, _dev(x0.copy()), _dev(bb), sweeps=2, zero_start=False).cpu().numpy()
        assert np.array_equal(got, want.astype(np.float64)), ("fp32", l)
    x32, info32 = S32.solve(_dev(b), tol=1e-6)
    assert info32["relres_true"] < 1e-6
    assert abs(info32["iterations"] - info["iterations"]) <= max(1, 0.1 * info["iterations"])
    S32.close()
