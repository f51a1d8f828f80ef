import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (oracle on larger meshes)")

# Tests run with the default launch choices unless they load a tuning table themselves;
# an explicitly set MTP_TUNE_FILE is kept.
os.environ.setdefault("MTP_TUNE_FILE", "")
