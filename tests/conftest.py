import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _ensure_built():
    """Build the HIP library and the oracle only if nothing is built yet."""
    lib = os.path.join(ROOT, "paper_1312_2880_amd", "libhmg.so")
    if not os.path.exists(lib):
        from paper_1312_2880_amd import build as hb
        hb.build()


_ensure_built()
