"""The serving runtime: every request's result is the same alone and in a
mix of concurrently running solves (batched requests: the same as batched
alone), admission respects the memory budget, and errors come back per
request."""
import time

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1109_5981_amd import lsrn
    lsrn.lib()  # raises if the library is missing: there is no CPU fallback
    return lsrn


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def mix(L):
    """Uneven requests: tall and fat dense, FP64 and the precision form,
    LSQR and Chebyshev, sparse with Tikhonov."""
    reqs = []
    shapes = [(3000, 60, 0, "fp64", "lsqr"), (5000, 200, 0, "mixed", "lsqr"), (80, 4000, 1, "fp64", "lsqr"),
              (12000, 130, 0, "fp64", "chebyshev"), (2500, 40, 0, "fp64", "lsqr"),
              (150, 3000, 1, "fp64", "chebyshev"), (7000, 300, 0, "mixed", "lsqr"),
              (4000, 100, 0, "fp64", "lsqr")]
    for i, (m, n, layout, prec, meth) in enumerate(shapes):
        rows, cols = (m, n) if layout == 0 else (n, m)        # stored array
        P = workloads.dense_problem(max(rows, cols), min(rows, cols), smin=10.0 ** -(3 + i % 4),
                                    seed=100 + i)
        A = P.A if layout == 0 else P.A                       # tall storage (rows >= cols)
        b = workloads.rhs_gauss(m, 100 + i)
        # one request asks for autotuning: a served solve never tunes, so its
        # result still equals the lone solve's without tuning
        reqs.append(("dense", dev(A), dev(b), dict(layout=layout, precision=prec, method=meth,
                                                     seed=7 + i, refine=10 if prec == "mixed" else 3,
                                                     autotune=1 if i == 4 else 0),
                     (orc_dense(A, layout), b)))
    S = workloads.sparse_problem(20000, 150, per_row=12, n_dense=3, fill=0.2, seed=9)
    b = workloads.rhs_gauss(S.m, 9)
    reqs.append(("csr", L.Csr.from_host(S.m, S.n, S.rowptr, S.colind, S.val),
                 dev(b), dict(lam=1e-3, seed=3, refine=2),
                 (("csr", S), b)))
    return reqs


def orc_dense(A, layout):
    return ("colmajor" if layout == 1 else "dense", A)


def oracle_ref(orc, spec, b, lam):
    kind, A = spec
    if kind == "csr":
        M = orc.Matrix.csr(A.m, A.n, A.rowptr, A.colind, A.val, lam=lam)
    elif kind == "colmajor":
        M = orc.Matrix.dense_colmajor(A, lam=lam)
    else:
        M = orc.Matrix.dense(A, lam=lam)
    return orc.lsrn_solve(M, b, seed=1, refine=3).x


def batchable(kind, opts):
    """The requests the server's batcher takes (the batched path's scope:
    dense row-major over-determined LSQR or Chebyshev, n <= 512, no lambda;
    precision-form requests run in FP64 there; every request of the mix is
    wide enough for the Chebyshev bounds)."""
    return (kind == "dense" and opts.get("layout", 0) == 0 and opts.get("lam", 0.0) == 0.0)


def solve_alone(L, kind, A, b, opts):
    """A request's result alone: the batched path with only this request for
    those the batcher takes, the one-problem solve for the rest."""
    if kind == "dense" and batchable(kind, opts) and A.shape[0] >= A.shape[1] and A.shape[1] <= 512:
        o = {k: v for k, v in opts.items() if k != "layout"}
        xs, infos = L.solve_batch([A], [b], allow_not_converged=True, per_problem=[o])
        return host(xs[0]), infos[0]
    if kind == "dense":
        x, info = L.solve_dense(A, b, allow_not_converged=True, **opts)
    else:
        x, info = L.solve_csr(A, b, **opts)
    return host(x), info


def test_results_alone_equal_results_in_mix(L, orc):
    """Each served result equals the same request solved alone bit for bit,
    and every one is within 1e-10 of the oracle's reference-mode solution
    (FP64 requests refined three steps; precision-form requests refined to
    their FP64 answer)."""
    reqs = mix(L)
    assert sum(batchable(kind, o) for kind, _, _, o, _ in reqs) == 6   # both queues are used
    L.tune_clear()
    alone = [solve_alone(L, kind, A, b, {k: v for k, v in o.items() if k != "autotune"})[0]
             for kind, A, b, o, _ in reqs]
    for (kind, A, b, opts, (spec, b_h)), x in zip(reqs, alone):
        ref = oracle_ref(orc, spec, b_h, opts.get("lam", 0.0))
        e = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        assert e <= 1e-10, (kind, opts, e)
    with L.Server(hbm_budget_bytes=64 << 30, streams=4) as srv:
        for rep in range(2):
            tickets = []
            for kind, A, b, opts, _ in reqs:
                if kind == "dense":
                    tickets.append(srv.submit_dense(A, b, **opts))
                else:
                    tickets.append(srv.submit_csr(A, b, **opts))
            for t, ref, (kind, _, _, opts, _) in zip(tickets, alone, reqs):
                x, info, tm = srv.wait(t, allow_not_converged=True)
                np.testing.assert_array_equal(host(x), ref)
                assert tm["latency_ms"] >= tm["run_ms"] >= 0.0
                assert (tm["batch_size"] >= 1) == batchable(kind, opts)
    assert L.tune_export() == ""     # no served request recorded a tuned shape


def test_admission_respects_budget(L):
    P = workloads.dense_problem(20000, 100, smin=1e-4, seed=5)
    A, b = dev(P.A), dev(workloads.rhs_gauss(20000, 5))
    need = L.workspace_bytes(20000, 100)
    budget = int(1.5 * need)   # one request at a time fits, two do not
    with L.Server(hbm_budget_bytes=budget, streams=4) as srv:
        t0 = time.perf_counter()
        tickets = [srv.submit_dense(A, b, seed=s) for s in range(6)]
        spans = []
        for t in tickets:
            _, _, tm = srv.wait(t)
            assert tm["footprint_bytes"] == need
            spans.append((tm["queue_ms"], tm["queue_ms"] + tm["run_ms"]))
    # admitted one after the other: each request starts after the previous
    # one finished (submissions were back to back, so queue times grow)
    spans.sort()
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        assert s1 >= e0 - 2.0


def test_request_errors_are_per_request(L):
    P = workloads.dense_problem(500, 20, smin=1e-3, seed=6)
    A, b = dev(P.A), dev(workloads.rhs_gauss(500, 6))
    with L.Server(hbm_budget_bytes=1 << 30, streams=2) as srv:
        good = srv.submit_dense(A, b)
        bad = srv.submit_dense(A, b, precision="mixed", method="chebyshev")
        # an invalid request of the batcher's kind among valid ones: it
        # fails alone, the others are batched and solved
        goods = [srv.submit_dense(A, b, seed=s) for s in range(3)]
        invalid = srv.submit_dense(A, b, tol=2.0)
        goods += [srv.submit_dense(A, b, seed=s) for s in range(3, 6)]
        _, info, _ = srv.wait(good)
        assert info["rank"] == 20
        with pytest.raises(L.LSRNError) as e:
            srv.wait(bad)
        assert e.value.status == 5
        with pytest.raises(L.LSRNError) as e:
            srv.wait(invalid)
        assert e.value.status == 1
        for t in goods:
            _, info, tm = srv.wait(t)
            assert info["rank"] == 20 and tm["batch_size"] >= 1
