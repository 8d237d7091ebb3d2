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
    """Records the error of a GPU result against the FP64 oracle (printed and, when a
    gpurun_out/ folder exists, written to gpurun_out/parity_errors.json)."""

    def rec(what: str, value: float, bound: float):
        entry = {"test": request.node.name, "what": what, "error": float(value),
                 "bound": float(bound)}
        _ERRORS.append(entry)
        print(f"[parity] {request.node.name} {what}: {value:.3e} (bound {bound:.1e})", flush=True)
        return value

    return rec


def pytest_sessionfinish(session, exitstatus):
    out = os.path.join(ROOT, "gpurun_out")
    if _ERRORS and os.path.isdir(out):
        with open(os.path.join(out, "parity_errors.json"), "w") as f:
            json.dump(_ERRORS, f, indent=1)
