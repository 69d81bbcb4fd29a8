import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def c1_inputs():
    from paper_1408_0210_amd import workloads as W
    w = W.WORKLOADS["uniform2k_laplace_d3"]
    return W.make_points(w), W.make_sigma(w), w


@pytest.fixture(scope="session")
def c1_plan(oracle_lib, c1_inputs):
    _, _, w = c1_inputs
    return oracle_lib.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["depth"], w["tau"])


@pytest.fixture(scope="session")
def c1_direct(oracle_lib, c1_inputs):
    x, s, w = c1_inputs
    return oracle_lib.direct(w["kernel"], w["param"], x, x, s)
