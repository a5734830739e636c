"""Adaptive SETUP (Algorithm "ASCPR") on a Newton sequence, against the oracle,
and the error paths of the C ABI.

The sequence is the drifting-Jacobian generator (fixed pattern, +-5% value
drift per step) on a 16x14x8 grid.  For each rule the GPU's rebuild
decisions and iteration counts must equal the oracle's step by step (the
decisions are a pure function of the iteration history, so they must agree
exactly), every step must reach the true relative residual, and in FP64 every
step's iterate must match the oracle's within 1e-10 relative (reused steps
included: they run on the frozen B of the last SETUP).  Also: new values
before the first solve rebuild in every mode; reuse_mode 0 rebuilds on every
new set of values; a reused B is bit-identical before and after new values
arrive; a failed rebuild leaves the previous B usable.
"""
import numpy as np
import pytest

from oracle import ascpr, cpr
from workloads import blackoil as bo

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(scope="module")
def sequence():
    steps = list(bo.newton_sequence(n_steps=6, shape=(16, 14, 8)))
    return [(c, b) for _, c, b in steps]


RULES = [
    dict(mode="factor", factor=1.3, reuse_mode=2, mu=0),
    dict(mode="mu", factor=1.3, reuse_mode=1, mu=0),
    dict(mode="mu", factor=1.3, reuse_mode=1, mu=10 ** 6),
    dict(mode="mu", factor=1.3, reuse_mode=1, mu=6),
]


@pytest.mark.parametrize("rule", RULES, ids=lambda r: f"{r['mode']}-{r['mu']}")
@pytest.mark.parametrize("fp32", [False, True])
def test_sequence_matches_oracle(sequence, rule, fp32):
    from paper_2201_01970_amd import Params, Solver

    dt = np.float32 if fp32 else np.float64
    reps = ascpr.solve_sequence([(cpr.Bsr.from_case(c), b) for c, b in sequence], mode=rule["mode"],
                                mu=rule["mu"], factor=rule["factor"], dtype=dt)
    c0 = sequence[0][0]
    S = Solver(_dev(c0.row_ptr), _dev(c0.col), _dev(c0.vals.reshape(-1)),
               Params(precond_fp32=fp32, reuse_mode=rule["reuse_mode"], mu=rule["mu"],
                      reuse_factor=rule["factor"]))
    for k, ((case, b), rep) in enumerate(zip(sequence, reps)):
        if k > 0:
            S.update_values(_dev(case.vals.reshape(-1)))
        x, info = S.solve(_dev(b), tol=1e-6)
        rel = np.linalg.norm(cpr.bsr_residual(cpr.Bsr.from_case(case), x.cpu().numpy(), b)) / np.linalg.norm(b)
        print(f"[{rule['mode']}-{rule['mu']} fp32={fp32}] step {k}: gpu its={info['iterations']} "
              f"rebuilt={info['rebuilt']} | oracle its={rep.iterations} rebuilt={rep.rebuilt} relres={rel:.2e}")
        assert rel < 1e-6
        if k > 0:
            assert bool(info["rebuilt"]) == rep.rebuilt
        if not fp32:
            assert info["iterations"] == rep.iterations
            xg = x.cpu().numpy()
            assert np.linalg.norm(xg - rep.x) <= 1e-10 * np.linalg.norm(rep.x), k
        else:
            assert abs(info["iterations"] - rep.iterations) <= max(1, 0.1 * rep.iterations)
    S.close()


def test_values_from_host_or_device_agree(sequence):
    """cpr_setup and cpr_update_values take the matrix from host or device
    memory; a handle fed from the host (numpy, or a CPU tensor), one fed from
    the device, and one set up on the device and updated from the host give
    the same rebuild decisions, iteration counts and iterates bit for bit."""
    from paper_2201_01970_amd import Params, Solver

    c0 = sequence[0][0]
    p = Params(reuse_mode=1, mu=6)
    S_dev = Solver(_dev(c0.row_ptr), _dev(c0.col), _dev(c0.vals.reshape(-1)), p)
    S_host = Solver(c0.row_ptr, c0.col, c0.vals.reshape(-1), p)
    S_mix = Solver(_dev(c0.row_ptr), _dev(c0.col), _dev(c0.vals.reshape(-1)), p)
    for k, (case, b) in enumerate(sequence):
        if k > 0:
            S_dev.update_values(_dev(case.vals.reshape(-1)))
            S_host.update_values(np.ascontiguousarray(case.vals.reshape(-1)))
            hv = torch.from_numpy(np.ascontiguousarray(case.vals.reshape(-1)))
            S_mix.update_values(hv if k % 2 else hv.numpy())
        out = [S.solve(_dev(b), tol=1e-6) for S in (S_dev, S_host, S_mix)]
        x0 = out[0][0].cpu().numpy()
        for x, info in out[1:]:
            assert info["iterations"] == out[0][1]["iterations"], k
            assert info["rebuilt"] == out[0][1]["rebuilt"], k
            assert np.array_equal(x.cpu().numpy(), x0), k
    for S in (S_dev, S_host, S_mix):
        S.close()


def test_error_paths(sequence):
    from paper_2201_01970_amd import CprError, Params, Solver
    from paper_2201_01970_amd import _capi as capi

    case, b = sequence[0]
    S = Solver(_dev(case.row_ptr), _dev(case.col), _dev(case.vals.reshape(-1)), Params())
    # different size
    small = bo.case_small(shape=(5, 4, 3))
    with pytest.raises(CprError) as e:
        S.update_values(_dev(small.vals.reshape(-1)), _dev(small.row_ptr), _dev(small.col))
    assert e.value.status == capi.CPR_ERR_SIZE_MISMATCH
    # same sizes, different pattern (two column indices of row 0 swapped out)
    col = case.col.copy()
    r0 = slice(case.row_ptr[1], case.row_ptr[2])
    col[r0] = np.sort((col[r0] + 1) % case.n_b)
    with pytest.raises(CprError) as e:
        S.update_values(_dev(case.vals.reshape(-1)), _dev(case.row_ptr), _dev(col))
    assert e.value.status in (capi.CPR_ERR_PATTERN_MISMATCH,)
    # NaN in the right-hand side
    bad = b.copy()
    bad[7] = np.nan
    with pytest.raises(CprError) as e:
        S.solve(_dev(bad), tol=1e-6)
    assert e.value.status == capi.CPR_ERR_NAN
    # the handle still works afterwards
    x, info = S.solve(_dev(b), tol=1e-6)
    assert info["relres_true"] < 1e-6
    # zero right-hand side: converged with zero iterations
    x, info = S.solve(_dev(np.zeros_like(b)), tol=1e-6)
    assert info["iterations"] == 0 and np.all(x.cpu().numpy() == 0)
    S.close()


def test_invalid_matrices_rejected():
    from paper_2201_01970_amd import CprError, Params, Solver
    from paper_2201_01970_amd import _capi as capi

    case = bo.case_small(shape=(4, 4, 2))
    # missing diagonal block in row 3
    rp, col, vals = case.row_ptr.copy(), case.col.copy(), case.vals.copy()
    keep = np.ones(case.nnz_b, dtype=bool)
    d = rp[3] + int(np.nonzero(col[rp[3]:rp[4]] == 3)[0][0])
    keep[d] = False
    rp2 = rp.copy()
    rp2[4:] -= 1
    with pytest.raises(CprError) as e:
        Solver(rp2, col[keep], vals[keep], Params())
    assert e.value.status == capi.CPR_ERR_INVALID_ARG
    # singular diagonal block
    vals2 = vals.copy()
    d0 = int(np.nonzero(col[rp[0]:rp[1]] == 0)[0][0])
    vals2[d0] = 0.0
    with pytest.raises(CprError) as e:
        Solver(rp, col, vals2, Params())
    assert e.value.status == capi.CPR_ERR_SINGULAR_BLOCK


@pytest.mark.parametrize("reuse_mode", [0, 1, 2])
def test_values_before_first_solve_rebuild(sequence, reuse_mode):
    """setup(A0), update_values(A1), solve: the first solve runs on a B built
    from A1 (the oracle's solve k = 1 sets up on the matrix it solves)."""
    from paper_2201_01970_amd import Params, Solver

    steps = [(cpr.Bsr.from_case(c), b) for c, b in sequence[1:4]]
    mode = {0: "never", 1: "mu", 2: "factor"}[reuse_mode]
    reps = ascpr.solve_sequence(steps, mode=mode, mu=6, factor=1.3)
    c0 = sequence[0][0]
    S = Solver(_dev(c0.row_ptr), _dev(c0.col), _dev(c0.vals.reshape(-1)),
               Params(reuse_mode=reuse_mode, mu=6, reuse_factor=1.3))
    for k, ((A, b), rep) in enumerate(zip(steps, reps)):
        S.update_values(_dev(A.vals.reshape(-1)))
        x, info = S.solve(_dev(b), tol=1e-6)
        print(f"[first-solve mode {reuse_mode}] step {k}: gpu its={info['iterations']} rebuilt={info['rebuilt']} "
              f"| oracle its={rep.iterations} rebuilt={rep.rebuilt}", flush=True)
        assert bool(info["rebuilt"]) == rep.rebuilt, k
        assert info["iterations"] == rep.iterations, k
        assert np.linalg.norm(x.cpu().numpy() - rep.x) <= 1e-10 * np.linalg.norm(rep.x), k
    if reuse_mode == 0:
        assert all(r.rebuilt for r in reps)
    S.close()


def test_reused_operator_is_frozen(sequence):
    """New values do not touch a reused B: cpr_precond_apply gives the same
    bits before update_values, after it, and after a solve that reused B."""
    from paper_2201_01970_amd import Params, Solver

    (c0, b0), (c1, b1) = sequence[0], sequence[1]
    S = Solver(_dev(c0.row_ptr), _dev(c0.col), _dev(c0.vals.reshape(-1)), Params(reuse_mode=1, mu=10 ** 6))
    S.solve(_dev(b0), tol=1e-6)
    v = _dev(bo.rhs(c0.ndof, 91))
    z_before = S.precond(v).cpu().numpy()
    S.update_values(_dev(c1.vals.reshape(-1)))
    assert np.array_equal(S.precond(v).cpu().numpy(), z_before)
    x, info = S.solve(_dev(b1), tol=1e-6)
    assert info["rebuilt"] == 0
    assert np.array_equal(S.precond(v).cpu().numpy(), z_before)
    # the oracle's frozen operator (SETUP on A0) gives the same z within 1e-12
    B0 = cpr.setup(cpr.Bsr.from_case(c0))
    z_or = B0.apply(v.cpu().numpy())
    assert np.linalg.norm(z_before - z_or) <= 1e-12 * np.linalg.norm(z_or)
    S.close()


def test_failed_rebuild_keeps_previous_operator(sequence):
    """A singular diagonal block makes the rebuilding solve fail; the handle
    keeps its previous B (inspection calls work and give the same bits), and
    the next valid values solve normally."""
    from paper_2201_01970_amd import CprError, Params, Solver
    from paper_2201_01970_amd import _capi as capi

    (c0, b0), (c1, b1) = sequence[0], sequence[1]
    S = Solver(_dev(c0.row_ptr), _dev(c0.col), _dev(c0.vals.reshape(-1)), Params(reuse_mode=0))
    v = _dev(bo.rhs(c0.ndof, 92))
    z0 = S.precond(v).cpu().numpy()
    bad = c1.vals.copy()
    d0 = int(np.nonzero(c1.col[c1.row_ptr[5]:c1.row_ptr[6]] == 5)[0][0]) + int(c1.row_ptr[5])
    bad[d0] = 0.0
    S.update_values(_dev(bad.reshape(-1)))
    with pytest.raises(CprError) as e:
        S.solve(_dev(b1), tol=1e-6)
    assert e.value.status == capi.CPR_ERR_SINGULAR_BLOCK
    assert np.array_equal(S.precond(v).cpu().numpy(), z0)
    S.update_values(_dev(c1.vals.reshape(-1)))
    x, info = S.solve(_dev(b1), tol=1e-6)
    assert info["rebuilt"] == 1 and info["relres_true"] < 1e-6
    S.close()
