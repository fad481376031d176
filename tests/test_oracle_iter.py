"""Pins for the oracle's iterative solvers (Alg. 1/2 step 6, Alg. 3)."""
import json
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from scipy.sparse.linalg import lsqr as scipy_lsqr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _diag_op(sig):
    m = sig.size
    return m, m, (lambda x: sig * x), (lambda y: sig * y)


def _eps_for(k, sl, su):
    """A tolerance for which Alg. 3 runs exactly k iterations."""
    rate = (su - sl) / (su + sl)
    return 2.0 * rate ** (k - 1.5)


def test_cs_is_chebyshev_polynomial(orc):
    """After k steps the error in the component with singular value sigma is
    T_k((d - sigma^2)/c) / T_k(d/c) times the initial one (Golub-Varga):
    this fixes every alpha and beta of Alg. 3, including the k = 1 step."""
    sl, su = 0.5, 2.0
    sig = np.linspace(sl, su, 41)
    d, c = (su ** 2 + sl ** 2) / 2, (su ** 2 - sl ** 2) / 2
    b = np.random.default_rng(0).standard_normal(sig.size)
    xstar = b / sig
    for k in range(1, 9):
        eps = _eps_for(k, sl, su)
        assert orc.cs_iterations(sl, su, eps) == k
        x, it = orc.cs(*_diag_op(sig), b, sl, su, eps)
        assert it == k
        Tk = npcheb.Chebyshev.basis(k)
        p = Tk((d - sig ** 2) / c) / Tk(d / c)
        np.testing.assert_allclose(x, (1 - p) * xstar, rtol=0, atol=1e-12 * np.abs(xstar).max())


def test_cs_one_step_is_exact_when_bounds_meet(orc):
    sig = np.full(10, 1.7)
    b = np.arange(1.0, 11.0)
    x, it = orc.cs(*_diag_op(sig), b, 1.7, 1.7, 1e-14)
    assert it == 1
    np.testing.assert_allclose(x, b / 1.7, rtol=1e-15)


def test_table3_cs_iteration_count(orc):
    """Table 3: CS with gamma = 2 (s = 2048, r = 1024) takes 106 iterations at
    tolerance 1e-14; the count follows from Theorem 3's bounds with t = 1."""
    g = json.load(open(os.path.join(GOLDEN, "table3_cs_iterations.json")))
    sl, su = orc.cs_bounds(g["s"], g["r"], 1.0)
    assert orc.cs_iterations(sl, su, g["eps"]) == g["cs_iterations"]
    # Theorem 4 bound for LSQR with alpha -> 0 is above the printed LSQR count
    bound = (np.log(g["eps"]) - np.log(2)) / np.log(np.sqrt(g["r"] / g["s"]))
    assert g["lsqr_iterations"] <= bound


def test_kappa_estimate_below_six(orc):
    g = json.load(open(os.path.join(GOLDEN, "kappa_bound.json")))
    q = np.sqrt(g["ratio_r_over_s_max"])
    assert (1 + q) / (1 - q) < g["kappa_estimate_max"]


def test_lsqr_iterates_match_scipy(orc):
    """Oracle LSQR after k steps equals SciPy's LSQR after k steps."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((80, 30)) @ np.diag(np.linspace(1, 3, 30))
    b = rng.standard_normal(80)
    for k in (1, 2, 5, 10, 20):
        x, it, _ = orc.lsqr(80, 30, lambda v: A @ v, lambda u: A.T @ u, b, 1e-300, k)
        ref = scipy_lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert it == k
        assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_lsqr_converges_to_min_length_solution(orc):
    rng = np.random.default_rng(6)
    U = np.linalg.qr(rng.standard_normal((60, 8)))[0]
    V = np.linalg.qr(rng.standard_normal((20, 8)))[0]
    A = U @ np.diag(np.linspace(1, 2, 8)) @ V.T          # rank 8 of 20
    b = rng.standard_normal(60)
    x, it, ok = orc.lsqr(60, 20, lambda v: A @ v, lambda u: A.T @ u, b, 1e-14, 200)
    assert ok
    np.testing.assert_allclose(x, np.linalg.pinv(A) @ b, rtol=1e-12, atol=1e-13)


def test_lsqr_zero_rhs(orc):
    x, it, ok = orc.lsqr(5, 3, lambda v: np.ones(5) * v.sum(), lambda u: np.ones(3) * u.sum(),
                         np.zeros(5), 1e-14, 10)
    assert ok and it == 0 and not x.any()


def test_cs_bounds_reject_small_sketch(orc):
    with pytest.raises(ValueError):
        orc.cs_bounds(4, 4, 1.0)


@pytest.mark.parametrize("fat", [False, True])
def test_cs_check_catches_violated_bounds(orc, fat):
    """Theorem 3's bounds hold only with a probability (Lemma 3).  With the
    margin t made negative the interval [sigma_L, sigma_U] misses most of
    the spectrum of A N, the Chebyshev run diverges, the check after it
    fails and LSQR continues: the result is still the pseudoinverse
    solution.  With the default margin the check passes (no restart)."""
    import workloads
    P = workloads.dense_problem(1200, 60, smin=1e-3, seed=41)
    if fat:
        M = orc.Matrix.dense_colmajor(P.A)            # A = P.A^T, 60 x 1200
        A = P.A.T
        b = workloads.rhs_gauss(60, 41)
    else:
        M = orc.Matrix.dense(P.A)
        A = P.A
        b = workloads.rhs_gauss(1200, 41)
    ref = np.linalg.pinv(A) @ b
    ok = orc.lsrn_solve(M, b, seed=2, method=orc.CS)
    assert ok.cs_fallbacks == 0 and ok.converged
    bad = orc.lsrn_solve(M, b, seed=2, method=orc.CS, t_margin=-4.0)
    assert bad.cs_fallbacks == 1 and bad.converged
    # the divergent Chebyshev run alone is far off; the restarted result is not
    assert np.linalg.norm(bad.x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(ok.x - ref) <= 1e-9 * np.linalg.norm(ref)
