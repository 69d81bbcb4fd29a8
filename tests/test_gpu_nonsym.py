"""A kernel that is not symmetric: exp(a (z_x - r))/r (steady advection-diffusion
with the flow along x), two EIMs per level (Sec. 3.1).  The GPU pass against
the oracle's two-EIM pass (same setup, bit for bit: tests/test_abi.py) on the
same inputs, stage by stage, and against the direct sum; the general form on
1/r against the one-EIM pass; the same with the M2L compression of Sec. 4.2
(both stages), the oracle counting its own ranks and the library's checked
against them."""
import numpy as np
import pytest

from paper_1408_0210_amd import workloads as W
from parity_util import assert_close, rel as _rel

pytestmark = pytest.mark.gpu


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


def _eval(E, torch_dev, kernel, param, x, s, depth, tau, **kw):
    torch, dev = torch_dev
    plan = E.Plan(kernel, param, [0, 0, 0], 1.0, x.shape[1], depth, tau, **kw)
    plan.set_points(torch.from_numpy(x).to(dev))
    f = plan.evaluate(torch.from_numpy(np.ascontiguousarray(s)).to(dev))
    torch.cuda.synchronize()
    return plan, f.cpu().numpy()


@pytest.fixture(scope="module")
def c1(oracle_lib):
    x, s = W.uniform_points(2000, 1), W.potentials(2000, 2)
    O = oracle_lib.Plan("advdiff", 1.0, [0, 0, 0], 1.0, 3, 1e-6)
    fo, D = O.evaluate(x, s, dumps=True)
    return x, s, O, fo, D, oracle_lib.direct("advdiff", 1.0, x, x, s)


def test_advdiff_vs_oracle(E, torch_dev, c1):
    x, s, O, fo, D, fd = c1
    plan, f = _eval(E, torch_dev, "advdiff", 1.0, x, s, 3, 1e-6)
    st = plan.stats()
    assert st["d"] == {k: O.levels[k]["d"] for k in (2, 3)}
    assert st["d2"] == {k: O.levels2[k]["d"] for k in (2, 3)}
    assert_close(f, fo, 1e-10, "vs oracle two-EIM EIFMM")
    assert_close(f, fd, 1e-6, "vs direct sum", max_tol=1e-5)
    plan.close()


def test_advdiff_stages_vs_oracle(E, torch_dev, c1):
    """W, What (first EIM's size); g, l, lhat (second EIM's size)."""
    x, s, O, fo, D, fd = c1
    plan, f = _eval(E, torch_dev, "advdiff", 1.0, x, s, 3, 1e-6)
    tol = {"W": 1e-12, "What": 1e-5, "g": 1e-10, "l": 1e-10}
    for k in (2, 3):
        for name in ("W", "What", "g", "l"):
            e = _rel(plan.export_expansion(name, k), D[name][k])
            assert e < tol[name], (name, k, e)
    assert _rel(plan.export_expansion("lhat", 3), D["lhat"]) < 1e-5
    plan.close()


def test_advdiff_mixed_and_multi_rhs(E, torch_dev, c1):
    torch, dev = torch_dev
    x, s, O, fo, D, fd = c1
    plan, f = _eval(E, torch_dev, "advdiff", 1.0, x, s, 3, 1e-6, precision="mixed")
    assert _rel(f, fd) < 1e-6
    plan.close()
    S = np.stack([s, -2.0 * s])
    plan, F = _eval(E, torch_dev, "advdiff", 1.0, x, S, 3, 1e-6, max_rhs=2)
    assert _rel(F[0], fo) < 1e-10
    np.testing.assert_array_equal(F[1], -2.0 * F[0])
    plan.close()


def test_two_eim_form_on_laplace(E, torch_dev, oracle_lib):
    """The general form forced on 1/r: equal to the oracle's two-EIM pass and to
    the library's own one-EIM pass."""
    x, s = W.uniform_points(2000, 1), W.potentials(2000, 2)
    plan2, f2 = _eval(E, torch_dev, "laplace", 0.0, x, s, 3, 1e-6, two_eim=True)
    assert plan2.stats()["d2"][3] == plan2.stats()["d"][3]
    plan2.close()
    plan1, f1 = _eval(E, torch_dev, "laplace", 0.0, x, s, 3, 1e-6)
    plan1.close()
    O = oracle_lib.Plan("laplace", 0.0, [0, 0, 0], 1.0, 3, 1e-6, two_eim=True)
    assert _rel(f2, O.evaluate(x, s)) < 1e-10
    assert _rel(f2, f1) < 1e-10


def test_advdiff_clustered_and_targets(E, torch_dev, oracle_lib):
    """Clustered sources with separate uniform targets (depth 4), against the
    direct sum; a = 2 (stronger drift)."""
    torch, dev = torch_dev
    xs = W.cluster_points(5000, 3, 0.05, 111, 112)
    xt = W.uniform_points(3000, 113)
    s = W.potentials(5000, 114)
    plan = E.Plan("advdiff", 2.0, [0, 0, 0], 1.0, 5000, 4, 1e-6, n_targets=3000)
    plan.set_points(torch.from_numpy(xs).to(dev), targets=torch.from_numpy(xt).to(dev))
    f = plan.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    plan.close()
    assert _rel(f, oracle_lib.direct("advdiff", 2.0, xt, xs, s)) < 1e-6


@pytest.fixture(scope="module")
def c1c(E, torch_dev, oracle_lib):
    """The compressed pass (Sec. 4.2 with two EIMs: U from K_fat, V from K_thin):
    the oracle counts the rank of each level itself (the larger of the two
    filtered ranks) and the library must keep the same."""
    x, s = W.uniform_points(2000, 1), W.potentials(2000, 2)
    plan, f = _eval(E, torch_dev, "advdiff", 1.0, x, s, 3, 1e-6, compress_tol=1e-6)
    ranks = plan.stats()["rank"]
    O = oracle_lib.Plan("advdiff", 1.0, [0, 0, 0], 1.0, 3, 1e-6, compress_tol=1e-6)
    assert ranks == {k: O.levels[k]["r"] for k in (2, 3)}
    fo, D = O.evaluate(x, s, dumps=True)
    yield x, s, plan, f, ranks, O, fo, D
    plan.close()


def test_advdiff_compressed_vs_oracle(c1c, c1):
    x, s, plan, f, ranks, O, fo, D = c1c
    fd = c1[5]
    assert all(0 < ranks[k] < plan.stats()["d"][k] for k in (2, 3))
    assert_close(f, fo, 1e-10, "vs oracle compressed two-EIM EIFMM")
    assert_close(f, fd, 1e-6, "vs direct sum", max_tol=1e-5)
    for k in (2, 3):
        for name in ("g", "l"):
            assert_close(plan.export_expansion(name, k), D[name][k], 1e-10, f"{name} level {k}")


def test_advdiff_compressed_mixed_and_multi_rhs(E, torch_dev, c1c, c1):
    x, s, plan, f, ranks, O, fo, D = c1c
    fd = c1[5]
    pm, fm = _eval(E, torch_dev, "advdiff", 1.0, x, s, 3, 1e-6, compress_tol=1e-6,
                   precision="mixed")
    assert _rel(fm, fd) < 1e-6
    pm.close()
    S = np.stack([s, 0.5 * s + W.potentials(2000, 3)])
    p2, F = _eval(E, torch_dev, "advdiff", 1.0, x, S, 3, 1e-6, compress_tol=1e-6, max_rhs=2)
    assert _rel(F[0], f) < 1e-13
    assert _rel(F[1], O.evaluate(x, S[1])) < 1e-10
    p2.close()


def test_two_eim_compressed_laplace_equals_one_eim(E, torch_dev):
    x, s = W.uniform_points(2000, 1), W.potentials(2000, 2)
    p2, f2 = _eval(E, torch_dev, "laplace", 0.0, x, s, 3, 1e-6, two_eim=True, compress_tol=1e-6)
    p1, f1 = _eval(E, torch_dev, "laplace", 0.0, x, s, 3, 1e-6, compress_tol=1e-6)
    assert p2.stats()["rank"] == p1.stats()["rank"]
    p1.close()
    p2.close()
    assert _rel(f2, f1) < 1e-10


def test_advdiff_compressed_stage2_vs_oracle(E, torch_dev, oracle_lib):
    x, s = W.uniform_points(2000, 1), W.potentials(2000, 2)
    plan, f = _eval(E, torch_dev, "advdiff", 1.0, x, s, 3, 1e-6, compress_tol=1e-6,
                    compress_tol2=1e-6)
    ranks = plan.stats()["rank"]
    s2 = {k: plan.compression2(k) for k in ranks}
    assert all(s2[k].max() > 0 for k in ranks)
    plan.close()
    O = oracle_lib.Plan("advdiff", 1.0, [0, 0, 0], 1.0, 3, 1e-6, compress_tol=1e-6,
                        compress_tol2=1e-6)
    assert ranks == {k: O.levels[k]["r"] for k in (2, 3)}
    for k in ranks:
        np.testing.assert_array_equal(s2[k], O.levels[k]["s2"], err_msg=f"level {k}")
    assert_close(f, O.evaluate(x, s), 1e-10, "vs oracle stage-2 two-EIM EIFMM")


def test_two_eim_not_in_batches(E):
    with pytest.raises(E.EifmmError):
        E.Batch([dict(kernel="advdiff", param=1.0, n=100, tau=1e-4, depth=2)])
