"""Parity at the full sizes of the benchmark workloads, on sampled targets.

The CPU oracle cannot run the plain EIFMM at 1e6 points in test time, so these
tests compare the HIP pass, in the configuration the benchmark times, with the
oracle's FP64 direct sum (eq. (1)) evaluated one target at a time on a seeded
random sample of 2000 targets, and check properties that hold at any size:

  * accuracy: sampled rel-L2 <= the requested 1e-6 (the sample estimates the
    full rel-L2 to a few percent; every measured value is far below the bound);
  * exact linearity: scaling sigma by 2 scales every rounding step by 2, so
    f(2 sigma) == 2 f(sigma) bit for bit, in FP64 and in mixed precision;
  * permutation invariance: the pass sorts by (key, input index), so permuting
    the input changes only the order of additions inside a leaf (<= 1e-12);
  * monotone accuracy in tau (Sec. 5.2 reports the error falling with d).
"""
import os

import numpy as np
import pytest

from paper_1408_0210_amd import workloads as W

pytestmark = pytest.mark.gpu

NS = 2000                    # sampled targets
THREADS = min(os.cpu_count() or 1, 16)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def E():
    from paper_1408_0210_amd import eifmm
    eifmm.lib()
    return eifmm


class Case:
    """Points, sigma, a sampled direct-sum reference and the device copies."""

    def __init__(self, name, torch_dev, oracle_lib):
        torch, dev = torch_dev
        self.w = dict(W.WORKLOADS[name])
        self.x = W.make_points(self.w)
        self.s = W.make_sigma(self.w)
        self.n = self.w["n"]
        rng = np.random.default_rng(2024)
        self.idx = np.sort(rng.choice(self.n, NS, replace=False))
        self.xd = torch.from_numpy(self.x).to(dev)
        self._ref = {}
        self.oracle = oracle_lib

    def ref(self, col=None):
        s = self.s if col is None else self.s[:, col]
        key = col
        if key not in self._ref:
            self._ref[key] = self.oracle.direct(self.w["kernel"], self.w["param"],
                                                self.x[:, self.idx].copy(), self.x,
                                                np.ascontiguousarray(s), threads=THREADS)
        return self._ref[key]


@pytest.fixture(scope="module")
def c2(torch_dev, oracle_lib):
    return Case("uniform1m_laplace_d5", torch_dev, oracle_lib)


@pytest.fixture(scope="module")
def c3(torch_dev, oracle_lib):
    return Case("cluster1m_yukawa", torch_dev, oracle_lib)


def _plan(E, case, depth=None, tau=None, precision="fp64", compress_tol=None, max_rhs=1):
    w = case.w
    if compress_tol is None:
        compress_tol = w.get("compress_tol", 1e-6)  # the benchmark's setting
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, case.n,
                  depth if depth is not None else w["depth"], tau if tau else w["tau"],
                  max_rhs=max_rhs, precision=precision, compress_tol=compress_tol)
    plan.set_points(case.xd)
    return plan


def _eval(torch_dev, plan, s):
    torch, dev = torch_dev
    f = plan.evaluate(torch.from_numpy(np.ascontiguousarray(s)).to(dev))
    torch.cuda.synchronize()
    return f.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uniform1m_sampled(precision, E, torch_dev, c2):
    """1e6 uniform points, 1/r, depth 5, tau 1e-6, M2L compressed as the timed run."""
    plan = _plan(E, c2, precision=precision)
    f = _eval(torch_dev, plan, c2.s)
    err = _rel(f[c2.idx], c2.ref())
    print(f"uniform1m {precision}: sampled rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-6
    f2 = _eval(torch_dev, plan, 2.0 * c2.s)
    np.testing.assert_array_equal(f2, 2.0 * f)
    plan.close()


def test_uniform1m_uncompressed_matches_compressed(E, torch_dev, c2):
    plan = _plan(E, c2, compress_tol=0.0)
    f0 = _eval(torch_dev, plan, c2.s)
    plan.close()
    plan = _plan(E, c2)
    f1 = _eval(torch_dev, plan, c2.s)
    plan.close()
    assert _rel(f0[c2.idx], c2.ref()) <= 1e-6
    assert _rel(f1, f0) <= 1e-6


def test_uniform1m_tau_sweep(E, torch_dev, c2):
    """tau in {1e-4, 1e-6, 1e-8} (compression at the same tolerance): the sampled
    error falls with tau and stays below tau."""
    errs = []
    for tau in (1e-4, 1e-6, 1e-8):
        plan = _plan(E, c2, tau=tau, compress_tol=tau)
        f = _eval(torch_dev, plan, c2.s)
        errs.append(_rel(f[c2.idx], c2.ref()))
        print(f"tau {tau:.0e}: d={plan.stats()['d']} rank={plan.stats()['rank']} "
              f"sampled rel-L2 {errs[-1]:.3e}", flush=True)
        plan.close()
    assert errs[0] > errs[1] > errs[2]
    for tau, e in zip((1e-4, 1e-6, 1e-8), errs):
        assert e <= tau


def test_uniform1m_permutation_invariance(E, torch_dev, c2):
    torch, dev = torch_dev
    plan = _plan(E, c2)
    f = _eval(torch_dev, plan, c2.s)
    p = np.random.default_rng(77).permutation(c2.n)
    plan.set_points(torch.from_numpy(np.ascontiguousarray(c2.x[:, p])).to(dev))
    fp = _eval(torch_dev, plan, c2.s[p])
    assert _rel(fp, f[p]) <= 1e-12
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cluster1m_yukawa_sampled(precision, E, torch_dev, c3):
    """16 Gaussian clusters (width 0.03), exp(-r)/r, depth 5 (crowded leaves of a
    few thousand points), tau 1e-6."""
    plan = _plan(E, c3, precision=precision)
    f = _eval(torch_dev, plan, c3.s)
    err = _rel(f[c3.idx], c3.ref())
    print(f"cluster1m {precision}: d={plan.stats()['d']} sampled rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-6
    f2 = _eval(torch_dev, plan, 2.0 * c3.s)
    np.testing.assert_array_equal(f2, 2.0 * f)
    plan.close()


@pytest.mark.parametrize("depth", [7, 8])
def test_cluster1m_deep_tree(depth, E, torch_dev, c3):
    """Deeper trees for the clustered cloud, up to the largest depth the library
    accepts (8: 16.8 million leaves, most of them empty)."""
    plan = _plan(E, c3, depth=depth, precision="mixed")
    f = _eval(torch_dev, plan, c3.s)
    err = _rel(f[c3.idx], c3.ref())
    print(f"cluster1m depth {depth}: sampled rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-6
    plan.close()


def test_rhs64_batched_mixed(E, torch_dev, oracle_lib):
    """2^20 points, 64 sigma vectors, mixed precision: right-hand sides 0, 21, 42
    and 63 against the direct sum; every column against the FP64 single-RHS pass."""
    torch, dev = torch_dev
    case = Case("uniform1m_laplace_d5_rhs64", torch_dev, oracle_lib)
    S = case.s  # (n, 64), column-major
    plan = _plan(E, case, precision="mixed", max_rhs=64)
    F = _eval(torch_dev, plan, S.T)
    plan.close()
    for r in (0, 21, 42, 63):
        err = _rel(F[r][case.idx], case.ref(r))
        print(f"rhs {r}: sampled rel-L2 {err:.3e}", flush=True)
        assert err <= 1e-6
    single = _plan(E, case)
    for r in range(64):
        f1 = _eval(torch_dev, single, S[:, r])
        assert _rel(F[r], f1) <= 1e-6, r
    single.close()


@pytest.mark.parametrize("name", ["uniform1m_cosr_d5", "uniform1m_gauss1_d5", "uniform1m_mq_d5"])
def test_paper_kernels_1m(name, E, torch_dev, oracle_lib):
    """The paper's inhomogeneous kernels on its 1e6-point cube (Sec. 5.4), depth 5,
    tau = 1e-6 with compression at the same tolerance: sampled rel-L2 <= 1e-6; for
    exp(-r^2) and sqrt(r^2+1) the number of interpolation points falls with depth."""
    case = Case(name, torch_dev, oracle_lib)
    plan = _plan(E, case, compress_tol=case.w["tau"])
    f = _eval(torch_dev, plan, case.s)
    err = _rel(f[case.idx], case.ref())
    d = plan.stats()["d"]
    print(f"{name}: d={d} sampled rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-6
    if case.w["kernel"] in ("gauss", "mq"):
        assert d[5] < d[4] < d[3] < d[2]
    plan.close()


def test_uniform100m_gauss(E, torch_dev, oracle_lib):
    """The paper's largest case (Table 4): 1e8 points in the cube, exp(-r^2), depth 7,
    tau 1e-6, mixed precision: 100 sampled targets against the direct sum."""
    torch, dev = torch_dev
    w = W.WORKLOADS["uniform100m_gauss1_d7"]
    x, s = W.make_points(w), W.make_sigma(w)
    idx = np.sort(np.random.default_rng(5).choice(w["n"], 100, replace=False))
    ref = oracle_lib.direct(w["kernel"], w["param"], x[:, idx].copy(), x, s, threads=THREADS)
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  precision="mixed", compress_tol=1e-6)
    xd = torch.from_numpy(x).to(dev)
    plan.set_points(xd)
    f = plan.evaluate(torch.from_numpy(s).to(dev))
    torch.cuda.synchronize()
    err = _rel(f.cpu().numpy()[idx], ref)
    print(f"uniform100m gauss: d={plan.stats()['d']} sampled rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-6
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_targets1m_sampled(precision, E, torch_dev, oracle_lib):
    """1e6 sources and 1e6 separate targets in the cube (the benchmark's targets
    run): 2000 sampled targets against the direct sum, and exact linearity."""
    torch, dev = torch_dev
    w = W.WORKLOADS["uniform1m_targets1m_laplace_d5"]
    xs, xt, s = W.make_points(w), W.make_targets(w), W.make_sigma(w)
    idx = np.sort(np.random.default_rng(17).choice(w["n_targets"], NS, replace=False))
    ref = oracle_lib.direct(w["kernel"], w["param"], xt[:, idx].copy(), xs, s, threads=THREADS)
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  precision=precision, compress_tol=w["compress_tol"], n_targets=w["n_targets"])
    plan.set_points(torch.from_numpy(xs).to(dev), targets=torch.from_numpy(xt).to(dev))
    sd = torch.from_numpy(s).to(dev)
    f = plan.evaluate(sd).cpu().numpy()
    err = _rel(f[idx], ref)
    print(f"targets1m {precision}: sampled rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-6
    np.testing.assert_array_equal(plan.evaluate(2.0 * sd).cpu().numpy(), 2.0 * f)
    plan.close()


@pytest.mark.parametrize("precision,ctol", [("fp64", 0.0), ("fp64", 5e-6), ("mixed", 5e-6)])
def test_advdiff1m_sampled(precision, ctol, E, torch_dev, oracle_lib):
    """The advection-diffusion kernel exp(z_x - r)/r (two EIMs per level) on the
    1e6-point cube, depth 5, tau 1e-6, with and without M2L compression: sampled
    targets against the direct sum."""
    case = Case("uniform1m_advdiff1_d5", torch_dev, oracle_lib)
    plan = _plan(E, case, precision=precision, compress_tol=ctol)
    f = _eval(torch_dev, plan, case.s)
    err = _rel(f[case.idx], case.ref())
    print(f"advdiff1m {precision} compress {ctol}: d={plan.stats()['d']} "
          f"d2={plan.stats()['d2']} rank={plan.stats()['rank']} sampled rel-L2 {err:.3e}",
          flush=True)
    assert err <= 1e-6
    plan.close()
