"""Algorithm 1 on the GPU: a device plan runs the greedy's iterations (argmax
and rank-1 update of the training residual) on the device.  Products and
differences are separately rounded and the quotient is a correctly rounded
division, as on the host, so the device plan selects the same training points
and gets the same factors as the host setup (itself pinned to the oracle's
Algorithm 1 by tests/test_abi.py), bit for bit.

The M2M and L2L operators (Sec. 4.1) of a device plan are solved on the device
by the pass's blocked MFMA solves; with EIFMM_FLAG_HOST_SETUP by substitution on
the host.  Both are backward-stable solves of the same systems, so the passes
agree to rounding; every parity test against the oracle runs device plans, so
the device-solved operators are the ones checked there."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_0210_amd import eifmm
    eifmm.lib()
    return eifmm


@pytest.mark.parametrize("kernel,param,depth,tau,tol_mode",
                         [("laplace", 0.0, 5, 1e-6, 0), ("yukawa", 1.0, 3, 1e-5, 0),
                          ("gauss", 1.0, 4, 1e-6, 0), ("gauss", 0.01, 4, 5e-7, 1),
                          ("cosr", 20.0, 3, 1e-4, 0), ("mq", 1.0, 3, 1e-6, 0),
                          ("sqdist", 0.0, 3, 1e-8, 0)])
def test_gpu_greedy_equals_host(kernel, param, depth, tau, tol_mode, E):
    G = E.Plan(kernel, param, [0, 0, 0], 1.0, 100, depth, tau, tol_mode=tol_mode)
    H = E.Plan(kernel, param, [0, 0, 0], 1.0, 100, depth, tau, tol_mode=tol_mode,
               host_only=True)
    sg, sh = G.stats(), H.stats()
    print(f"{kernel} depth {depth}: d={sg['d']} setup device {sg['setup_ms']:.0f} ms, "
          f"host {sh['setup_ms']:.0f} ms", flush=True)
    assert sg["d"] == sh["d"]
    assert sg["eim_err"] == sh["eim_err"]
    for k in range(2, depth + 1):
        a, b = G.level(k), H.level(k)
        for key in ("ia", "ib", "X", "Y", "G", "B"):
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"{key} level {k}")
    G.close()
    H.close()


def test_gpu_greedy_dmax(E):
    """Reaching dmax is the same error on the device."""
    with pytest.raises(E.EifmmError) as e:
        E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 3, 1e-6, dmax=30)
    assert e.value.code == -4


def test_host_setup_flag(E):
    """EIFMM_FLAG_HOST_SETUP keeps the iterations on the host: same tables."""
    G = E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 3, 1e-6)
    H = E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 3, 1e-6, host_setup=True)
    for k in (2, 3):
        np.testing.assert_array_equal(G.level(k)["G"], H.level(k)["G"])
    G.close()
    H.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kernel,param,depth,ctol", [("laplace", 0.0, 4, 0.0),
                                                     ("laplace", 0.0, 4, 1e-6),
                                                     ("yukawa", 1.0, 4, 0.0),
                                                     ("advdiff", 1.0, 4, 0.0),
                                                     ("advdiff", 1.0, 3, 1e-6)])
def test_device_operator_solves(kernel, param, depth, ctol, E):
    import torch
    from paper_1408_0210_amd import workloads as W
    dev = torch.device("cuda:0")
    x, s = W.uniform_points(6000, 91), W.potentials(6000, 92)
    out = {}
    for host in (False, True):
        P = E.Plan(kernel, param, [0, 0, 0], 1.0, 6000, depth, 1e-6, compress_tol=ctol,
                   host_setup=host)
        P.set_points(torch.from_numpy(x).to(dev))
        out[host] = (P.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy(), P.stats()["rank"])
        P.close()
    assert out[False][1] == out[True][1]
    assert _rel(out[False][0], out[True][0]) < 1e-11
