import os
import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture
def write_mech(tmp_path):
    """Write mechanism text to a temporary file and return its path."""
    def _w(text, name="tiny.mech"):
        p = tmp_path / name
        p.write_text(text)
        return str(p)
    return _w


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
