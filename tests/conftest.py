import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) device and the built device library")
    # the CPU-side libraries are cheap to build; build them only when absent
    from oracle import build as ob
    from sccg_gen import build as gb
    if not os.path.exists(os.path.join(ROOT, "oracle", "libsccg_oracle.so")):
        ob.build()
    if not os.path.exists(os.path.join(ROOT, "sccg_gen", "libsccg_gen.so")):
        gb.build()


@pytest.fixture(scope="session")
def cfg1():
    import sccg_gen
    return sccg_gen.pairs(1)
