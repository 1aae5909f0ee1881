import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def params_path():
    import sdinputs
    return sdinputs.default_params_path()


@pytest.fixture(scope="session")
def oparams(params_path):
    import oracle
    return oracle.Params(params_path)


@pytest.fixture(scope="session")
def weights():
    import sdinputs
    return sdinputs.codon_weights(2026)
