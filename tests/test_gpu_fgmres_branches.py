"""The branches of flexible GMRES(m) (Algorithm "ASCPR-GMRES") that a
well-preconditioned solve never reaches, against the oracle.

* Restart cycles: m = 2, 4 and 6 on the 2000-cell grid to 1e-10, so the
  back substitution, x += Z y, the true residual and a new cycle run several
  times.
* Long cycles: without smoothing sweeps (0 pre, 0 post) the preconditioner is
  weak; to 1e-6 the first cycle runs 19 Arnoldi steps (the Gram-Schmidt dots
  and updates of steps j >= 16 are split over two kernel chunks), and to 1e-10
  the solve needs 31 steps, crossing a restart at m = 30.
* Non-convergence: m = 4, one cycle, tol 1e-12 ends with CPR_NOT_CONVERGED
  and the iterate of the oracle's single cycle.

Each case needs the oracle's iteration count exactly and its iterate within
1e-10 relative (the two sides differ only in the order of the FP64 dot
products).
"""
import numpy as np
import pytest

from oracle import amg, cpr, fgmres
from workloads import blackoil as bo

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def small():
    case = bo.case_small()
    return case, bo.rhs(case.ndof, 1001)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


CASES = [
    dict(id="restart4", restart=4, max_restarts=100, tol=1e-10, pre=2, post=2, status="CPR_OK"),
    dict(id="restart2", restart=2, max_restarts=100, tol=1e-10, pre=2, post=2, status="CPR_OK"),
    dict(id="restart6", restart=6, max_restarts=100, tol=1e-10, pre=2, post=2, status="CPR_OK"),
    dict(id="long-cycle", restart=30, max_restarts=100, tol=1e-6, pre=0, post=0, status="CPR_OK"),
    dict(id="restart30-crossed", restart=30, max_restarts=100, tol=1e-10, pre=0, post=0, status="CPR_OK"),
    dict(id="not-converged", restart=4, max_restarts=1, tol=1e-12, pre=2, post=2, status="CPR_NOT_CONVERGED"),
]


@pytest.mark.parametrize("c", CASES, ids=lambda c: c["id"])
def test_fgmres_branch_matches_oracle(small, c):
    from paper_2201_01970_amd import Params, Solver

    case, b = small
    A = cpr.Bsr.from_case(case)
    B = cpr.setup(A, amg.AmgParams(pre_sweeps=c["pre"], post_sweeps=c["post"]))
    ref = fgmres.fgmres(lambda v: cpr.bsr_matvec(A, v), B.apply, b, tol=c["tol"], m=c["restart"],
                        max_restarts=c["max_restarts"])
    S = Solver(_dev(case.row_ptr), _dev(case.col), _dev(case.vals.reshape(-1)),
               Params(restart=c["restart"], max_restarts=c["max_restarts"], pre_sweeps=c["pre"],
                      post_sweeps=c["post"]))
    x, info = S.solve(_dev(b), tol=c["tol"], allow_not_converged=True)
    x = x.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"[{c['id']}] gpu its={info['iterations']} restarts={info['restarts']} {info['status']} | oracle "
          f"its={ref.iterations} restarts={ref.restarts} converged={ref.converged} | rel diff {err:.2e}", flush=True)
    assert info["status"] == c["status"]
    assert ref.converged == (c["status"] == "CPR_OK")
    assert info["iterations"] == ref.iterations
    assert info["restarts"] == ref.restarts
    assert err <= 1e-10
    if c["id"] == "long-cycle":
        assert ref.iterations >= 17 and ref.restarts == 0
    if c["id"] == "restart30-crossed":
        assert ref.iterations > 30 and ref.restarts >= 1
    if c["id"].startswith("restart") and c["restart"] < 30:
        assert ref.restarts >= 1
    S.close()
