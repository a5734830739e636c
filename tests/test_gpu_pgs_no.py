"""Smoother comparison of Section 6 on the GPU: PGS-SCM against PGS-NO.

PGS-NO (cpr_params.smoother = 1) is the natural-order parallel Gauss-Seidel
the paper compares PGS-SCM with: rows split into contiguous chunks,
Gauss-Seidel inside a chunk, other chunks' values from the sweep's start.
Its result depends on the chunk count (the paper's thread count NT), while
PGS-SCM's does not depend on how the GPU runs it.  Bars:
  * PGS-NO sweeps bit for bit against the oracle's natural_chunk_sweep on
    every smoothed level, for several chunk counts, from zero and from a
    random start; FP32 sweeps bit for bit against the oracle on float32;
  * PGS-NO V-cycle within 1e-12 of the oracle's; FP64 solve with the
    oracle's iteration count and iterate within 1e-10;
  * PGS-SCM: the FP64 solve's iterate is bit-identical for every storage
    form and launch shape of the level matrices (row_layout 1, 2, 4, 16 and
    with or without the one-workgroup tail), the GPU analogue of the
    paper's iterations being unchanged over thread counts at theta = 0.
"""
import numpy as np
import pytest

from oracle import amg, cpr, fgmres
from workloads import blackoil as bo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _solver(case, **kw):
    from paper_2201_01970_amd import Params, Solver

    return Solver(_dev(case.row_ptr), _dev(case.col), _dev(case.vals.reshape(-1)), Params(**kw))


@pytest.fixture(scope="module")
def mid():
    case = bo.case_spe10_like(seed=1110, shape=(30, 40, 20))
    print(f"[pgs-no] n_b={case.n_b}", flush=True)
    return case, cpr.Bsr.from_case(case), bo.rhs(case.ndof, 1111)


@pytest.mark.parametrize("chunks", [1, 7, 256, 100000])
def test_pgs_no_sweeps_bit_exact(mid, chunks):
    case, A, _ = mid
    B = cpr.setup(A, amg.AmgParams(smoother="pgs-no", gs_chunks=chunks))
    H = B.amg
    for fp32 in (False, True):
        S = _solver(case, smoother=1, smoother_chunks=chunks, precond_fp32=int(fp32))
        assert S.level_info(0)["n_levels"] == H.n_levels
        dt = np.float32 if fp32 else np.float64
        rng = np.random.default_rng(chunks)
        for l in range(H.n_levels - 1):
            lev = H.levels[l]
            Al = amg._cast(lev.A, dt)
            bb = rng.standard_normal(lev.A.n_rows).astype(dt)
            x0 = rng.standard_normal(lev.A.n_rows).astype(dt)
            want = x0.copy()
            for _ in range(2):
                amg.natural_chunk_sweep(Al, chunks, want, bb)
            got = S.smooth(l, _dev(x0.astype(np.float64)), _dev(bb.astype(np.float64)), sweeps=2).cpu().numpy()
            assert np.array_equal(got, want.astype(np.float64)), (l, fp32)
            want = np.zeros_like(bb)
            for _ in range(2):
                amg.natural_chunk_sweep(Al, chunks, want, bb)
            got = S.smooth(l, _dev(np.zeros(lev.A.n_rows)), _dev(bb.astype(np.float64)), sweeps=2,
                           zero_start=True).cpu().numpy()
            assert np.array_equal(got, want.astype(np.float64)), (l, fp32, "zero")
        S.close()


@pytest.mark.parametrize("chunks", [16, 4096])
def test_pgs_no_vcycle_and_solve(mid, chunks):
    case, A, b = mid
    B = cpr.setup(A, amg.AmgParams(smoother="pgs-no", gs_chunks=chunks))
    S = _solver(case, smoother=1, smoother_chunks=chunks)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(case.n_b)
    want = amg.vcycle(B.amg, r)
    got = S.vcycle(_dev(r)).cpu().numpy()
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)
    x, info = S.solve(_dev(b), tol=1e-6)
    x = x.cpu().numpy()
    print(f"[pgs-no {chunks}] its gpu {info['iterations']} oracle {res.iterations}", flush=True)
    assert info["iterations"] == res.iterations
    assert np.linalg.norm(x - res.x) <= 1e-10 * np.linalg.norm(res.x)
    S.close()


def test_pgs_scm_result_independent_of_launch_shape(mid):
    case, _, b = mid
    ref = None
    for kw in (dict(row_layout=0), dict(row_layout=1), dict(row_layout=2), dict(row_layout=4),
               dict(row_layout=16), dict(tail_nnz=0), dict(theta_color=0.0, row_layout=1),
               dict(theta_color=0.0, row_layout=2)):
        S = _solver(case, **kw)
        x, info = S.solve(_dev(b), tol=1e-6)
        S.close()
        x = x.cpu().numpy()
        key = kw.get("theta_color", 0.05)
        print(f"[pgs-scm {kw}] its {info['iterations']}", flush=True)
        if ref is None or key not in ref:
            ref = dict(ref or {})
            ref[key] = (x, info["iterations"])
            continue
        assert info["iterations"] == ref[key][1]
        assert np.array_equal(x, ref[key][0])
