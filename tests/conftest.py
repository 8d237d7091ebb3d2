import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_ERRORS = []


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    if not any("gpu" in it.keywords for it in items):
        return
    import torch

    if torch.cuda.is_available():
        p = torch.cuda.get_device_properties(0)
        print(f"\n[device] {p.name} {getattr(p, 'gcnArchName', '?')} "
              f"{p.total_memory >> 20} MiB, {p.multi_processor_count} CUs", flush=True)
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture
def record_error(request):
    """Records the error of a GPU result against the FP64 oracle (printed, and written as
    JSON to the file named by the SMOE_PARITY_ERRORS environment variable, if set)."""

    def rec(what: str, value: float, bound: float):
        entry = {"test": request.node.name, "what": what, "error": float(value),
                 "bound": float(bound)}
        _ERRORS.append(entry)
        print(f"[parity] {request.node.name} {what}: {value:.3e} (bound {bound:.1e})", flush=True)
        return value

    return rec


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("SMOE_PARITY_ERRORS")
    if _ERRORS and path:
        with open(path, "w") as f:
            json.dump(_ERRORS, f, indent=1)
