"""Batches of independent problems (eifmm_batch_*): the fused, graph-replayed pass.

  * each problem of a batch equals its own plan at the same depth, built on the
    same level tables (with the absolute stopping rule, the scale level the
    batch reports): the fused launches do per problem what the plan does, except that a gathered-GEMM tile split across workgroups may be summed
    in another order, so the bound is 1e-12 rather than bit equality;
  * every problem against the oracle's direct sum: the requested 1e-6 (rel-L2);
  * graph replays, changed buffers and new points give the same results.
"""
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


def _small_problems():
    """Ten problems of uneven size: 1/r and exp(-r^2/0.01), uniform and clustered,
    fixed and autotuned depths, one problem large enough for Stream-K splits."""
    spec = [  # n, kernel, dist, depth
        (1000, "laplace", "uniform", None), (3000, "gauss", "cluster", None),
        (700, "laplace", "cluster", 2), (12000, "laplace", "uniform", 3),
        (5000, "gauss", "uniform", 3), (1, "laplace", "uniform", 2),
        (2500, "laplace", "cluster", None), (8000, "gauss", "cluster", None),
        (40000, "laplace", "uniform", 4), (1500, "gauss", "uniform", 2)]
    out = []
    for i, (n, kern, dist, depth) in enumerate(spec):
        x = (W.uniform_points(n, 500 + i) if dist == "uniform"
             else W.cluster_points(n, 4, 0.03, 600 + i, 700 + i))
        out.append(dict(n=n, kernel=kern, param=0.01 if kern == "gauss" else 0.0, depth=depth,
                        points=x, sigma=W.potentials(n, 800 + i), **W.BATCH_TOLERANCES[kern]))
    return out


@pytest.fixture(scope="module")
def small(E, torch_dev):
    torch, dev = torch_dev
    probs = _small_problems()
    B = E.Batch(probs)
    xs = [torch.from_numpy(q["points"]).to(dev) for q in probs]
    B.set_points(xs)
    ss = [torch.from_numpy(q["sigma"]).to(dev) for q in probs]
    F = [f.cpu().numpy() for f in B.evaluate(ss)]
    torch.cuda.synchronize()
    yield B, probs, xs, ss, F
    B.close()


def test_batch_matches_plans(E, torch_dev, small):
    torch, dev = torch_dev
    B, probs, xs, ss, F = small
    info = B.info()
    print("batch info", info, flush=True)
    assert info["graph_nodes"] > 0 and info["m2l_rbt"] in (3, 4, 5, 6)
    for p, q in enumerate(probs):
        st = B.stats(p)
        if q["depth"] is not None:
            assert st["depth"] == q["depth"]
        else:
            assert 2 <= st["depth"] <= 8
        # with the absolute stopping rule the shared tables take their scale from
        # their deepest level, which the problem's stats name: the plan uses it too
        assert (st["scale_level"] >= st["depth"]) if q["tol_mode"] == 1 else st["scale_level"] == 0
        plan = E.Plan(q["kernel"], q["param"], [0, 0, 0], 1.0, q["n"], st["depth"], q["tau"],
                      tol_mode=q["tol_mode"], compress_tol=q["compress_tol"],
                      scale_level=st["scale_level"])
        assert plan.stats()["d"] == st["d"]
        plan.set_points(xs[p])
        f1 = plan.evaluate(ss[p]).cpu().numpy()
        plan.close()
        if q["n"] == 1:
            np.testing.assert_array_equal(F[p], f1)
        else:
            assert _rel(F[p], f1) <= 1e-12, p


def test_batch_mixed_vs_direct(E, torch_dev, oracle_lib, small):
    """The same ten problems as one mixed-precision batch (FP32 M2L and near field):
    every problem within 1e-6 of the direct sum, and of the FP64 batch."""
    torch, dev = torch_dev
    _, probs, xs, ss, F = small
    B = E.Batch(probs, precision="mixed")
    B.set_points(xs)
    G = [f.cpu().numpy() for f in B.evaluate(ss)]
    again = [f.cpu().numpy() for f in B.evaluate(ss)]
    B.close()
    for p, q in enumerate(probs):
        np.testing.assert_array_equal(again[p], G[p])
        if q["n"] == 1:
            assert G[p][0] == 0.0
            continue
        fd = oracle_lib.direct(q["kernel"], q["param"], q["points"], q["points"], q["sigma"])
        err = _rel(G[p], fd)
        print(f"mixed problem {p}: n={q['n']} {q['kernel']} rel-L2 {err:.3e}", flush=True)
        assert err <= 1e-6, p
        assert _rel(G[p], F[p]) <= 1e-6, p


def test_batch_vs_direct(oracle_lib, small):
    B, probs, xs, ss, F = small
    for p, q in enumerate(probs):
        fd = oracle_lib.direct(q["kernel"], q["param"], q["points"], q["points"], q["sigma"])
        if q["n"] == 1:
            assert F[p][0] == 0.0 and fd[0] == 0.0
            continue
        err = _rel(F[p], fd)
        print(f"problem {p}: n={q['n']} {q['kernel']} depth={B.stats(p)['depth']} "
              f"rel-L2 {err:.3e}", flush=True)
        assert err <= 1e-6, p


def test_batch_replay_and_buffers(torch_dev, small):
    torch, dev = torch_dev
    B, probs, xs, ss, F = small
    again = [f.cpu().numpy() for f in B.evaluate(ss)]
    for a, b in zip(again, F):
        np.testing.assert_array_equal(a, b)
    # new sigma values in the same tensors, results into new tensors: linearity
    for t in ss:
        t.mul_(-2.0)
    out = [torch.full_like(t, np.nan) for t in ss]
    B.evaluate(ss, out)
    for o, b in zip(out, F):
        np.testing.assert_array_equal(o.cpu().numpy(), -2.0 * b)
    for t in ss:
        t.mul_(-0.5)
    # the unfused path (each problem's own pass) gives the same values
    U = [f.cpu().numpy() for f in B.evaluate_unfused(ss)]
    for p, (u, b) in enumerate(zip(U, F)):
        if probs[p]["n"] > 1:
            assert _rel(u, b) <= 1e-12, p


def test_batch_new_points(E, torch_dev, oracle_lib, small):
    torch, dev = torch_dev
    B, probs, xs, ss, F = small
    depths = [B.stats(p)["depth"] for p in range(len(probs))]
    new = [W.uniform_points(q["n"], 900 + p) for p, q in enumerate(probs)]
    B.set_points([torch.from_numpy(x).to(dev) for x in new])
    assert [B.stats(p)["depth"] for p in range(len(probs))] == depths
    G = [f.cpu().numpy() for f in B.evaluate(ss)]
    for p, q in enumerate(probs):
        if q["n"] < 2:
            continue
        fd = oracle_lib.direct(q["kernel"], q["param"], new[p], new[p], q["sigma"])
        assert _rel(G[p], fd) <= 1e-6, p
    B.set_points(xs)  # restore for the other tests of the module


def test_uneven_batch_256(E, torch_dev, oracle_lib):
    """256 problems, N log-uniform in [1e3, 2e5], half uniform / half 4 clusters,
    half 1/r / half exp(-r^2/0.01), depths autotuned, tolerances per kernel chosen
    for rel-L2 1e-6: 200 sampled targets of every problem against the direct sum."""
    torch, dev = torch_dev
    probs = W.uneven_batch()
    for q in probs:
        q.update(W.BATCH_TOLERANCES[q["kernel"]], depth=None)
    B = E.Batch(probs)
    B.set_points([torch.from_numpy(q["points"]).to(dev) for q in probs])
    F = [f.cpu().numpy() for f in
         B.evaluate([torch.from_numpy(q["sigma"]).to(dev) for q in probs])]
    info = B.info()
    print("uneven batch:", info, flush=True)
    rng = np.random.default_rng(3)
    worst = 0.0
    for p, q in enumerate(probs):
        idx = np.sort(rng.choice(q["n"], min(200, q["n"]), replace=False))
        fd = oracle_lib.direct(q["kernel"], q["param"], q["points"][:, idx].copy(),
                               q["points"], q["sigma"], threads=16)
        err = _rel(F[p][idx], fd)
        worst = max(worst, err)
        assert err <= 1e-6, (p, q["n"], q["kernel"], q["dist"], err)
    print(f"uneven batch: worst sampled rel-L2 {worst:.3e}", flush=True)
    B.close()
