import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# tuned tile budgets persist in a file between processes; the tests keep
# theirs in a file of their own session (tests that need another set it)
if "VDWNL_TUNE_CACHE" not in os.environ:
    import tempfile
    os.environ["VDWNL_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="vdwnl_tune_"), "tuning.json")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def table():
    """The oracle's FP64 kernel table (N_q = 20 log mesh, q_c = 5, m_c = 12)."""
    from oracle import kernel_table as kt
    t = kt.kernel_table()
    t = dict(t)
    t["mc"] = 12
    return t
