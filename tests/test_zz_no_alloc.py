"""eifmm_evaluate_noalloc (no device allocation in the call; Stream-K partial
tiles in the library's static scratch array) against eifmm_evaluate, through
the C ABI.  The two passes run the same kernels; only the number of workgroups
that share a Stream-K tail differs (the scratch holds fewer pieces than a plan's
workspace), which changes the order of a few FP64 additions: bound 1e-12
(rel-L2 and max norm).  Two calls in a row, the second on a smaller input, then
the first input again, so that the scratch's previous contents cannot leak."""
import numpy as np
import pytest

from paper_1408_0210_amd import workloads as W
from parity_util import assert_close

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


def _case(E, torch_dev, n, depth, nrhs, precision, dist, seed):
    torch, dev = torch_dev
    x = (W.uniform_points(n, seed) if dist == "uniform"
         else W.cluster_points(n, 4, 0.05, seed, seed + 1))
    S = np.stack([W.potentials(n, seed + 2 + r) for r in range(nrhs)])
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, n, depth, 1e-6, max_rhs=nrhs,
                  precision=precision, compress_tol=6e-6)
    plan.set_points(torch.from_numpy(x).to(dev))
    sd = torch.from_numpy(S).to(dev)
    ref = plan.evaluate(sd).cpu().numpy()
    return plan, sd, ref


def test_noalloc_matches_evaluate(E, torch_dev):
    torch, dev = torch_dev
    print("noalloc: 100k uniform points, depth 4, 2 RHS, FP64", flush=True)
    pa, sa, ra = _case(E, torch_dev, 100_000, 4, 2, "fp64", "uniform", 301)
    print("noalloc: 5000 clustered points, depth 3, 1 RHS, mixed", flush=True)
    pb, sb, rb = _case(E, torch_dev, 5000, 3, 1, "mixed", "cluster", 311)
    fa = torch.full((2, 100_000), np.nan, dtype=torch.float64, device=dev)
    fb = torch.full((1, 5000), np.nan, dtype=torch.float64, device=dev)
    for rep in range(2):
        pa.evaluate_noalloc(sa, fa)
        a = fa.cpu().numpy()
        pb.evaluate_noalloc(sb, fb)  # the smaller input second
        b = fb.cpu().numpy()
        for r in range(2):
            assert_close(a[r], ra[r], 1e-12, f"large input, RHS {r}, call {rep}")
        assert_close(b[0], rb[0], 1e-12, f"small input, call {rep}")
    # repeated calls leave the device's free memory unchanged
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev)[0]
    for _ in range(3):
        pa.evaluate_noalloc(sa, fa)
        pb.evaluate_noalloc(sb, fb)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(dev)[0] == free0
    np.testing.assert_array_equal(fa.cpu().numpy(), a)
    pa.close()
    pb.close()


def test_noalloc_argument_errors(E, torch_dev):
    torch, dev = torch_dev
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, 1000, 3, 1e-4)
    s = torch.zeros(1000, dtype=torch.float64, device=dev)
    f = torch.empty(1000, dtype=torch.float64, device=dev)
    with pytest.raises(E.EifmmError) as e:
        plan.evaluate_noalloc(s, f)
    assert e.value.code == -3  # before set_points
    plan.close()
    x = torch.from_numpy(W.uniform_points(1000, 5)).to(dev)
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, 1000, 3, 1e-6, compress_tol=1e-6,
                  compress_tol2=1e-6)
    plan.set_points(x)
    with pytest.raises(E.EifmmError) as e:
        plan.evaluate_noalloc(s, f)
    assert e.value.code == -1  # the second compression stage keeps its own workspace
    plan.close()
