"""The serving runtime (include/cpr_serve.h) on the GPU.

* Every result is bit-identical whether its case's requests run alone
  (one slot, only that case) or mixed with other cases on four slots, with
  repeat Newton steps reusing the resident hierarchy.
* Results equal those of a plain handle with the same parameters and agree
  with the true residual.
* Every served request matches the oracle: each case's request stream is the
  oracle's Newton sequence (Algorithm "ASCPR", relative rule 1.3, float32
  preconditioner model): same rebuild decisions, same iteration counts, true
  relres < 1e-6, and an iterate no further from the oracle's float32-model
  iterate than five times the oracle's own float32-vs-float64 gap on that
  request (at least 1e-8).  Two float32 roundings of the same operator differ
  by about as much as float32 differs from float64: the library factors the
  3x3 diagonal blocks with its own FP64 routine before the cast, which moves
  single float32 values by an ulp; on requests solved with a reused B the
  oracle's own gap reaches 1e-7.
* A budget smaller than one case rejects the request (CPR_ERR_OOM); a budget
  for about one case evicts idle cases and still serves everything.
"""
import numpy as np
import pytest

from oracle import ascpr, cpr
from workloads import blackoil as bo

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests():
    descs = [
        dict(case_id=1, shape=(18, 16, 6), sigma=1.5, seed=11, drift_seed=None),
        dict(case_id=2, shape=(30, 12, 9), sigma=2.0, seed=12, drift_seed=None),
        dict(case_id=3, shape=(10, 10, 4), sigma=1.0, seed=13, drift_seed=None),
        dict(case_id=1, shape=(18, 16, 6), sigma=1.5, seed=11, drift_seed=101),
        dict(case_id=4, shape=(25, 25, 8), sigma=2.5, seed=14, drift_seed=None),
        dict(case_id=2, shape=(30, 12, 9), sigma=2.0, seed=12, drift_seed=102),
        dict(case_id=1, shape=(18, 16, 6), sigma=1.5, seed=11, drift_seed=103),
        dict(case_id=3, shape=(10, 10, 4), sigma=1.0, seed=13, drift_seed=104),
    ]
    out = []
    for d in descs:
        case, b = bo.serving_case(d)
        out.append((d["case_id"], case, b))
    return out


def _run(reqs, slots, budget=2 ** 34, params=None):
    from paper_2201_01970_amd import Params, Server

    S = Server(budget, slots, params or Params(precond_fp32=True))
    tickets = [S.submit(cid, c.row_ptr, c.col, c.vals, b) for cid, c, b in reqs]
    results = [S.wait(t) for t in tickets]
    stats = S.stats()
    S.close()
    return results, stats


def test_alone_vs_mix_bit_identical():
    reqs = _requests()
    mixed, stats = _run(reqs, slots=4)
    for (cid, c, b), (x, info) in zip(reqs, mixed):
        print(f"[serve mix] case {cid} n_b={c.n_b}: {info['status']} {info.get('error', '')} "
              f"its={info['iterations']} rebuilt={info['rebuilt']} latency={info['latency_ms']:.1f} ms", flush=True)
    print("[serve mix] stats", stats, flush=True)
    assert all(info["status"] == "CPR_OK" for _, info in mixed)
    assert stats["completed"] == len(reqs) and stats["rejected"] == 0
    assert stats["setups"] == 4 and stats["reuses"] == 4
    for cid in sorted({r[0] for r in reqs}):
        idx = [k for k, r in enumerate(reqs) if r[0] == cid]
        alone, _ = _run([reqs[k] for k in idx], slots=1)
        for k, (xa, ia) in zip(idx, alone):
            xm, im = mixed[k]
            assert im["status"] == "CPR_OK" and ia["status"] == "CPR_OK"
            assert np.array_equal(xm, xa), (cid, k)
            assert im["iterations"] == ia["iterations"] and im["rebuilt"] == ia["rebuilt"]
    for (cid, c, b), (x, info) in zip(reqs, mixed):
        rel = np.linalg.norm(cpr.bsr_residual(cpr.Bsr.from_case(c), x, b)) / np.linalg.norm(b)
        assert rel < 1e-6
        assert info["latency_ms"] > 0


def test_server_equals_plain_handle():
    from paper_2201_01970_amd import Params, Solver

    reqs = _requests()[:3]
    served, _ = _run(reqs, slots=2)
    for (cid, c, b), (x, info) in zip(reqs, served):
        S = Solver(c.row_ptr, c.col, c.vals, Params(precond_fp32=True))
        xs, _ = S.solve(torch.as_tensor(b, device="cuda"))
        assert np.array_equal(xs.cpu().numpy(), x)
        S.close()


def test_budget_rejection_and_eviction():
    reqs = _requests()
    res, stats = _run(reqs[:1], slots=2, budget=1 << 20)
    assert res[0][1]["status"] == "CPR_ERR_OOM" and stats["rejected"] == 1
    # room for one or two cases at a time: idle cases get evicted, all requests served
    res, stats = _run(reqs, slots=2, budget=48 << 20)
    print("stats with a 48 MiB budget:", stats)
    assert all(info["status"] == "CPR_OK" for _, info in res)
    assert stats["evictions"] >= 1
    for (cid, c, b), (x, info) in zip(reqs, res):
        rel = np.linalg.norm(cpr.bsr_residual(cpr.Bsr.from_case(c), x, b)) / np.linalg.norm(b)
        assert rel < 1e-6


def test_served_requests_match_oracle():
    reqs = _requests()
    served, stats = _run(reqs, slots=4)
    assert stats["evictions"] == 0
    for cid in sorted({r[0] for r in reqs}):
        idx = [k for k, r in enumerate(reqs) if r[0] == cid]
        steps = [(cpr.Bsr.from_case(reqs[k][1]), reqs[k][2]) for k in idx]
        reps = ascpr.solve_sequence(steps, mode="factor", factor=1.3, dtype=np.float32)
        reps64 = ascpr.solve_sequence(steps, mode="factor", factor=1.3, dtype=np.float64)
        for n, (k, rep, rep64) in enumerate(zip(idx, reps, reps64)):
            x, info = served[k]
            d = np.linalg.norm(x - rep.x) / np.linalg.norm(rep.x)
            gap = np.linalg.norm(rep.x - rep64.x) / np.linalg.norm(rep64.x)
            print(f"[serve vs oracle] case {cid} request {k}: gpu its={info['iterations']} "
                  f"rebuilt={info['rebuilt']} relres={info['relres_true']:.2e} | oracle its={rep.iterations} "
                  f"rebuilt={rep.rebuilt} | diff {d:.2e}, oracle float32-vs-float64 gap {gap:.2e}", flush=True)
            assert info["status"] == "CPR_OK"
            assert info["relres_true"] < 1e-6
            assert info["iterations"] == rep.iterations, (cid, k)
            if n > 0:
                assert bool(info["rebuilt"]) == rep.rebuilt, (cid, k)
            assert d <= max(1e-8, 5.0 * gap), (cid, k)


def test_inverse_coarsest_alone_vs_mix_and_plain_handle():
    """The coarsest level solved by its explicit inverse (coarse_solver = 1,
    coarse_max = 400): each SETUP runs its own Gauss-Jordan elimination on its
    slot's stream, several at once on four slots (the 400-cell case is a
    single 400-row level).  Every result is bit-identical alone and in the
    mix, and equal to a plain handle's."""
    from paper_2201_01970_amd import Params, Solver

    params = Params(precond_fp32=True, coarse_solver=1, coarse_max=400)
    reqs = _requests()
    mixed, stats = _run(reqs, slots=4, params=params)
    print("[serve inverse] stats", stats, flush=True)
    assert all(info["status"] == "CPR_OK" for _, info in mixed)
    assert stats["setups"] == 4 and stats["reuses"] == 4
    for cid in sorted({r[0] for r in reqs}):
        idx = [k for k, r in enumerate(reqs) if r[0] == cid]
        alone, _ = _run([reqs[k] for k in idx], slots=1, params=params)
        for k, (xa, ia) in zip(idx, alone):
            xm, im = mixed[k]
            assert np.array_equal(xm, xa), (cid, k)
            assert im["iterations"] == ia["iterations"] and im["rebuilt"] == ia["rebuilt"]
    for k in range(3):  # first request of cases 1, 2, 3: a fresh SETUP each
        cid, c, b = reqs[k]
        S = Solver(c.row_ptr, c.col, c.vals, params)
        assert S.level_info(S.level_info(0)["n_levels"] - 1)["n"] <= 400
        xs, _ = S.solve(torch.as_tensor(b, device="cuda"))
        assert np.array_equal(xs.cpu().numpy(), mixed[k][0])
        S.close()
    for (cid, c, b), (x, info) in zip(reqs, mixed):
        rel = np.linalg.norm(cpr.bsr_residual(cpr.Bsr.from_case(c), x, b)) / np.linalg.norm(b)
        assert rel < 1e-6
