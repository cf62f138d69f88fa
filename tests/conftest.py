import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_DICT = os.path.join(ROOT, "paper_2404_19391_amd", "data", "default.zsd")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size parity cases")


@pytest.fixture(scope="session")
def odict():
    import oracle
    d = oracle.Dict.load(DEFAULT_DICT)
    assert d.valid
    return d
