import os
import sys

# the oracle's OpenMP threads sleep instead of spinning while they wait, so
# tests stay fast on a host that is busy with other work
os.environ.setdefault("OMP_WAIT_POLICY", "passive")
# concurrent runs (ns_run_many) need a hardware queue per stream; read by the
# HIP runtime when it starts, before any test touches the GPU
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long statistical runs")
