import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def weights_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("weights")


@pytest.fixture(scope="session")
def net_files(weights_dir):
    """Seeded weight files for the three network shapes."""
    import synth
    from synth import netcfg
    out = {}
    for name, kw in netcfg.DEFAULTS.items():
        path = str(weights_dir / f"{name}.hbw")
        synth.write_weights(path, name, **kw)
        out[name] = path
    return out
