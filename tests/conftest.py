import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: runs HIP kernels on an MI355X (gfx950)")
    config.addinivalue_line("markers", "slow: long CPU-only check")


def pytest_sessionstart(session):
    # report the device the GPU tests will use (visible in the run log)
    if session.config.getoption("-m", default="") == "gpu":
        import torch
        ok = torch.cuda.is_available()
        name = torch.cuda.get_device_name(0) if ok else "none"
        print(f"[session] torch {torch.__version__} cuda available={ok} device={name}", flush=True)
