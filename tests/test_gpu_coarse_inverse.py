"""Ruge-Stueben V-cycle with its coarsest level solved by the explicit inverse
(cpr_params.coarse_solver = 1) on the GPU, against the oracle.

The paper solves a coarsest space of thousands of unknowns directly (Section
6).  The oracle solves the coarsest level with LAPACK's LU factors; the GPU
forms A_L^{-1} by Gauss-Jordan elimination with partial pivoting at SETUP
and applies it as one dense FP64 product.  Both are the exact coarsest
solve up to rounding, so the bars are:
  * hierarchy (level sizes, colours) identical to the oracle's at the same
    coarse_max, and the levels above the coarsest swept bit for bit;
  * FP64 V-cycle and CPR apply within 1e-11 relative of the oracle's (the
    two coarsest solves differ by about cond(A_L) * eps relative, a few
    1e-13 here);
  * FP64 solve: the oracle's iteration count, iterate within 1e-10;
  * FP32 preconditioner: the float32 oracle's iteration count, iterate within
    1e-8 (as for the LU path);
  * graph replay bit-identical to eager launches.
"""
import numpy as np
import pytest

from oracle import amg, cpr, fgmres
from workloads import blackoil as bo

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (case, RHS seed, coarse_max): the 23400-cell SPE10-like grid leaves a
# coarsest level of 192 rows at coarse_max 400 (7 levels) and of 2265 rows at
# 2500 (4 levels; many 64-row tiles of the dense product and a ragged tail)
CASES = {
    "mid-400": lambda: (bo.case_spe10_like(seed=1110, shape=(30, 40, 20)), 1111, 400),
    "mid-2500": lambda: (bo.case_spe10_like(seed=1110, shape=(30, 40, 20)), 1111, 2500),
}


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _solver(case, **kw):
    from paper_2201_01970_amd import Params, Solver

    return Solver(_dev(case.row_ptr), _dev(case.col), _dev(case.vals.reshape(-1)), Params(**kw))


@pytest.fixture(scope="module", params=sorted(CASES))
def setup_inv(request):
    case, rseed, coarse = CASES[request.param]()
    print(f"[coarse inverse {request.param}] n_b={case.n_b} coarse_max={coarse}", flush=True)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, amg.AmgParams(coarse_max=coarse))
    b = bo.rhs(case.ndof, rseed)
    yield request.param, case, A, B, b, coarse


def test_hierarchy_and_sweeps_match_oracle(setup_inv):
    name, case, A, B, b, coarse = setup_inv
    H = B.amg
    S = _solver(case, coarse_max=coarse, coarse_solver=1)
    info = S.level_info(0)
    assert info["n_levels"] == H.n_levels
    nL = S.level_info(H.n_levels - 1)["n"]
    assert nL == H.levels[-1].A.n_rows
    print(f"[{name}] levels {H.n_levels}, coarsest {nL} rows")
    assert nL > 64
    rng = np.random.default_rng(21)
    for l in range(H.n_levels - 1):
        lev = H.levels[l]
        assert S.level_info(l)["n_colours"] == len(lev.colours)
        bb = rng.standard_normal(lev.A.n_rows)
        want = np.zeros(lev.A.n_rows)
        for _ in range(2):
            amg.colour_sweep(lev.A, lev.colours, want, bb)
        got = S.smooth(l, _dev(np.zeros(lev.A.n_rows)), _dev(bb), sweeps=2, zero_start=True).cpu().numpy()
        assert np.array_equal(got, want), l
    S.close()


@pytest.mark.parametrize("tail_nnz", [0, 30000])
def test_vcycle_and_apply_match_oracle(setup_inv, tail_nnz):
    """tail_nnz has no effect with the inverse (no single-workgroup kernel)."""
    name, case, A, B, b, coarse = setup_inv
    S = _solver(case, coarse_max=coarse, coarse_solver=1, tail_nnz=tail_nnz)
    S_lu = _solver(case, coarse_max=coarse, coarse_solver=0, tail_nnz=0)
    rng = np.random.default_rng(23)
    r = rng.standard_normal(A.n_b)
    want = amg.vcycle(B.amg, r)
    got = S.vcycle(_dev(r)).cpu().numpy()
    d_v = np.linalg.norm(got - want) / np.linalg.norm(want)
    d_lu = np.linalg.norm(got - S_lu.vcycle(_dev(r)).cpu().numpy()) / np.linalg.norm(want)
    v = rng.standard_normal(case.ndof)
    wa = B.apply(v)
    ga = S.precond(_dev(v)).cpu().numpy()
    d_a = np.linalg.norm(ga - wa) / np.linalg.norm(wa)
    print(f"[{name}] vcycle vs oracle {d_v:.2e}, vs GPU LU path {d_lu:.2e}; apply {d_a:.2e}")
    assert d_v <= 1e-11
    assert d_lu <= 1e-11
    assert d_a <= 1e-11
    S.close()
    S_lu.close()


def test_fp64_solve_matches_oracle(setup_inv):
    name, case, A, B, b, coarse = setup_inv
    S = _solver(case, coarse_max=coarse, coarse_solver=1)
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)
    x, info = S.solve(_dev(b), tol=1e-6)
    S.close()
    x = x.cpu().numpy()
    d = np.linalg.norm(x - res.x) / np.linalg.norm(res.x)
    print(f"[{name}] fp64 gpu its={info['iterations']} oracle its={res.iterations} iterate diff {d:.2e}")
    assert info["iterations"] == res.iterations
    assert d <= 1e-10
    assert info["relres_true"] < 1e-6


def test_fp32_solve_matches_fp32_oracle(setup_inv):
    name, case, A, B, b, coarse = setup_inv
    B32 = cpr.setup(A, amg.AmgParams(coarse_max=coarse), dtype=np.float32)
    res32 = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), lambda v: B32.apply(v).astype(np.float64), b, tol=1e-6)
    S = _solver(case, coarse_max=coarse, coarse_solver=1, precond_fp32=True)
    x, info = S.solve(_dev(b), tol=1e-6)
    S.close()
    x = x.cpu().numpy()
    d = np.linalg.norm(x - res32.x) / np.linalg.norm(res32.x)
    print(f"[{name}] fp32 gpu its={info['iterations']} oracle32 its={res32.iterations} iterate diff {d:.2e}")
    assert info["iterations"] == res32.iterations
    assert d <= 1e-8
    assert info["relres_true"] < 1e-6


def test_graph_replay_matches_eager(setup_inv):
    name, case, A, B, b, coarse = setup_inv
    for fp32 in (False, True):
        Se = _solver(case, coarse_max=coarse, coarse_solver=1, precond_fp32=fp32, use_graphs=False)
        Sg = _solver(case, coarse_max=coarse, coarse_solver=1, precond_fp32=fp32, use_graphs=True)
        xe, ie = Se.solve(_dev(b), tol=1e-6)
        xe = xe.cpu().numpy()
        for rep in range(3):
            xg, ig = Sg.solve(_dev(b), tol=1e-6)
            assert ig["iterations"] == ie["iterations"]
            assert np.array_equal(xg.cpu().numpy(), xe), (fp32, rep)
            Se.spmv(_dev(xe))  # eager work between replays
            torch.cuda.synchronize()
        Se.close()
        Sg.close()


def test_rejects_bad_coarse_solver():
    from paper_2201_01970_amd import CprError

    case = bo.case_small()
    with pytest.raises(CprError):
        _solver(case, coarse_solver=2)


def test_single_level_hierarchy_is_a_direct_solve():
    """coarse_max above the pressure size: the hierarchy is one level, the
    V-cycle is x = A_P^{-1} b (no smoothing), and CPR-FGMRES takes the
    oracle's iterations with the iterate within 1e-10.  The explicit inverse
    and LAPACK's solve differ by rounding amplified by the condition number
    of A_P (a nearly singular pressure matrix: accumulation terms of 3e-6
    against transmissibilities of 1e-3..1e-1), so the V-cycle bound is
    100 eps cond(A_P)."""
    case = bo.case_small()
    A = cpr.Bsr.from_case(case)
    b = bo.rhs(case.ndof, 1001)
    B = cpr.setup(A, amg.AmgParams(coarse_max=10 ** 6))
    assert B.amg.n_levels == 1
    S = _solver(case, coarse_max=10 ** 6, coarse_solver=1)
    assert S.level_info(0)["n_levels"] == 1
    rng = np.random.default_rng(29)
    r = rng.standard_normal(A.n_b)
    got = S.vcycle(_dev(r)).cpu().numpy()
    Ad = B.amg.levels[0].A.to_dense()
    want = np.linalg.solve(Ad, r)
    bound = 100 * np.finfo(np.float64).eps * np.linalg.cond(Ad)
    d = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"[direct] cond {np.linalg.cond(Ad):.2e}: vcycle diff {d:.2e}, bound {bound:.2e}", flush=True)
    assert d <= bound
    res = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=1e-6)
    x, info = S.solve(_dev(b), tol=1e-6)
    S.close()
    assert info["iterations"] == res.iterations
    assert np.linalg.norm(x.cpu().numpy() - res.x) <= 1e-10 * np.linalg.norm(res.x)


def test_newton_sequence_with_inverse_matches_oracle():
    """ASCPR over a drifting Newton sequence with the inverse path (rule
    It^(k-1) <= mu, mu = 7, so the sequence both reuses and rebuilds): each
    SETUP forms a new coarsest inverse in fresh SETUP memory, a reused B keeps
    the old one; rebuild flags and iterations equal the oracle's
    solve_sequence step by step, iterates within 1e-10."""
    from oracle import ascpr

    seq = list(bo.newton_sequence(n_steps=5, base_seed=1110, seed=1210, shape=(30, 40, 20), amp=0.2))
    steps = [(cpr.Bsr.from_case(c), b) for _, c, b in seq]
    reps = ascpr.solve_sequence(steps, amg.AmgParams(coarse_max=2500), mode="mu", mu=7)
    c0 = seq[0][1]
    S = _solver(c0, coarse_max=2500, coarse_solver=1, reuse_mode=1, mu=7)
    for k, ((_, case, b), rep) in enumerate(zip(seq, reps)):
        if k > 0:
            S.update_values(_dev(case.vals.reshape(-1)))
        x, info = S.solve(_dev(b), tol=1e-6)
        rebuilt = bool(info["rebuilt"]) or k == 0
        print(f"[inverse newton] step {k}: gpu its={info['iterations']} rebuilt={rebuilt} | "
              f"oracle its={rep.iterations} rebuilt={rep.rebuilt}", flush=True)
        assert rebuilt == rep.rebuilt, k
        assert info["iterations"] == rep.iterations, k
        assert np.linalg.norm(x.cpu().numpy() - rep.x) <= 1e-10 * np.linalg.norm(rep.x), k
    S.close()
    assert any(r.rebuilt for r in reps[1:]) and not all(r.rebuilt for r in reps[1:])


@pytest.mark.parametrize("solver", [0, 1])
def test_oversized_coarsest_is_refused(solver):
    """A coarsest level beyond the dense direct solve's limit (8192 rows by
    LU, 16384 by the inverse) is refused at SETUP with CPR_ERR_INVALID_ARG."""
    from paper_2201_01970_amd import CprError

    case = bo.case_spe10_like(seed=1110, shape=(30, 40, 20))  # 23400 pressure rows
    with pytest.raises(CprError, match="dense direct solve"):
        _solver(case, coarse_max=10 ** 6, coarse_solver=solver)


def _weak_pressure_diagonal_case(scale):
    """The 12x10x4 grid with the pressure entry of every diagonal block
    multiplied by `scale`: for scale 1e-3 the pressure matrix's largest entry
    of a column is off the diagonal, so partial pivoting interchanges rows at
    nearly every step (471 of 480 in LAPACK's factorisation)."""
    case = bo.case_small(seed=7, shape=(12, 10, 4))
    v = case.vals.copy()
    for i in range(case.n_b):
        lo, hi = case.row_ptr[i], case.row_ptr[i + 1]
        v[lo + int(np.nonzero(case.col[lo:hi] == i)[0][0]), 0, 0] *= scale
    case.vals = v
    return case


def test_inverse_with_row_interchanges():
    """A single-level hierarchy whose 480-row pressure matrix needs row
    interchanges at nearly every elimination step (7 full column panels and
    a ragged one): the V-cycle, A_P^{-1} r, within 100 eps cond(A_P) of
    LAPACK's solve, and the CPR apply within 1e-10 of the oracle's."""
    import scipy.linalg as sl

    case = _weak_pressure_diagonal_case(1e-3)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, amg.AmgParams(coarse_max=10 ** 6))
    assert B.amg.n_levels == 1
    Ad = B.amg.levels[0].A.to_dense()
    _, piv = sl.lu_factor(Ad)
    assert (piv != np.arange(Ad.shape[0])).sum() > 400
    S = _solver(case, coarse_max=10 ** 6, coarse_solver=1)
    rng = np.random.default_rng(31)
    r = rng.standard_normal(A.n_b)
    got = S.vcycle(_dev(r)).cpu().numpy()
    want = np.linalg.solve(Ad, r)
    bound = 100 * np.finfo(np.float64).eps * np.linalg.cond(Ad)
    d = np.linalg.norm(got - want) / np.linalg.norm(want)
    v = rng.standard_normal(case.ndof)
    wa = B.apply(v)
    da = np.linalg.norm(S.precond(_dev(v)).cpu().numpy() - wa) / np.linalg.norm(wa)
    print(f"[interchanges] cond {np.linalg.cond(Ad):.2e}: vcycle diff {d:.2e} (bound {bound:.2e}), apply {da:.2e}",
          flush=True)
    S.close()
    assert d <= bound
    assert da <= 1e-10


def test_singular_coarsest_is_refused():
    """A pressure matrix with a zero column (the pressure entries of one cell's
    column set to zero; its 3x3 diagonal block stays invertible) has no pivot
    in that column: SETUP fails with CPR_ERR_SINGULAR_COARSE."""
    from paper_2201_01970_amd import CprError

    case = bo.case_small(seed=7, shape=(12, 10, 4))
    v = case.vals.copy()
    j = 137
    v[case.col == j, 0, 0] = 0.0
    case.vals = v
    with pytest.raises(CprError, match="singular"):
        _solver(case, coarse_max=10 ** 6, coarse_solver=1)


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 3, 1), (8, 8, 1), (13, 5, 1), (16, 8, 1)],
                         ids=lambda s: "x".join(map(str, s)))
def test_inverse_at_panel_boundaries(shape):
    """Single-level hierarchies of 1, 15, 64, 65 and 128 rows: one partial
    column panel, exactly one and two full panels, and a full panel plus a
    one-column panel of the blocked elimination.  The V-cycle is
    A_P^{-1} r within 100 eps cond(A_P) of LAPACK's solve."""
    case = bo.case_small(seed=41, shape=shape)
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, amg.AmgParams(coarse_max=10 ** 6))
    Ad = B.amg.levels[0].A.to_dense()
    S = _solver(case, coarse_max=10 ** 6, coarse_solver=1)
    assert S.level_info(0)["n_levels"] == 1
    r = np.random.default_rng(43).standard_normal(A.n_b)
    got = S.vcycle(_dev(r)).cpu().numpy()
    S.close()
    want = np.linalg.solve(Ad, r)
    bound = 100 * np.finfo(np.float64).eps * np.linalg.cond(Ad)
    d = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"[panels {A.n_b}] vcycle diff {d:.2e}, bound {bound:.2e}", flush=True)
    assert d <= bound
