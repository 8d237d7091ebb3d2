"""CPU checks of the C ABI: the library loads, exports what include/smoe.h declares, the
ctypes structures match the C compiler's layout, and host-side validation rejects bad
arguments before anything is launched.  No compute call is made."""
import ctypes as ct
import re
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "smoe.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smoe_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2510_05814_amd import _capi

    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(_capi.lib, n), f"{n} declared in smoe.h but not exported"
    assert sorted(_capi.EXPORTED) == names
    out = subprocess.run(["nm", "-D", "--defined-only", str(_capi._LIB_PATH)], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (smoe_\w+)$", out, flags=re.M))
    assert set(names) <= exported


def test_struct_layouts_match_c(tmp_path):
    from paper_2510_05814_amd import _capi as C

    structs = {"smoe_model": C.SmoeModel, "smoe_grid": C.SmoeGrid, "smoe_bins": C.SmoeBins,
               "smoe_adam_config": C.SmoeAdamConfig, "smoe_fit_state": C.SmoeFitState,
               "smoe_segment": C.SmoeSegment, "smoe_batch": C.SmoeBatch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "smoe.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", f"-I{ROOT / 'include'}", str(src), "-o", str(exe)])
    got = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        s, f, v = ln.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ct.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_workspace_layout_host_only():
    from paper_2510_05814_amd import _capi as C

    n = C.smoe_bins_workspace_bytes(100, 3, 1, 64, 1000)
    assert n > 1000 * 15 * 4
    assert C.smoe_bins_workspace_bytes(-1, 3, 1, 64, 1000) == 0
    assert C.smoe_bins_workspace_bytes(10, 2, 1, 64, 1000) == 0
    base = 1 << 20  # a fake, 256-aligned address: layout only does pointer arithmetic
    b = C.SmoeBins()
    C.smoe_bins_layout(b, base, n, 100, 3, 1, 64, 1000)
    ptrs = [b.tile_rects, b.native_rects, b.counts, b.records, b.tile_counts, b.ranges, b.keys, b.vals,
            b.vals_alt, b.pair_grads, b.tile_loss, b.status]
    assert all(p % 256 == 0 for p in ptrs)
    assert ptrs == sorted(ptrs) and ptrs[-1] + 16 <= base + n
    assert b.record_stride == 16 and b.capacity == 1000 and b.max_tiles == 64
    # partial rows of NP = 15 floats padded to 16 (float4-aligned rows): 16 per kernel for the
    # fit step's kernel-major rows, then one per pair
    assert b.tile_loss - b.pair_grads >= (100 * 16 + 1000) * 16 * 4
    with pytest.raises(C.SmoeError):
        C.smoe_bins_layout(b, base, n - 1, 100, 3, 1, 64, 1000)
    with pytest.raises(C.SmoeError):
        C.smoe_bins_layout(b, base + 4, n, 100, 3, 1, 64, 1000)


def test_invalid_arguments_rejected_before_launch():
    """Each call validates on the host and returns SMOE_ERR_INVALID without touching a device."""
    from paper_2510_05814_amd import _capi as C

    lib = C.lib
    b = C.SmoeBins()
    n = C.smoe_bins_workspace_bytes(4, 3, 1, 16, 64)
    C.smoe_bins_layout(b, 1 << 20, n, 4, 3, 1, 16, 64)
    good_grid = C.SmoeGrid(64, 64, 1, 0, 0, 3.0)
    bad_models = [C.SmoeModel(4, 2, 1, 1 << 20), C.SmoeModel(4, 3, 2, 1 << 20),
                  C.SmoeModel(-1, 3, 1, 1 << 20), C.SmoeModel(4, 3, 1, None),
                  C.SmoeModel(5, 3, 1, 1 << 20)]  # K differs from the workspace
    for m in bad_models:
        assert lib.smoe_bin(ct.byref(m), ct.byref(good_grid), ct.byref(b), None) == C.SMOE_ERR_INVALID
    m = C.SmoeModel(4, 3, 1, 1 << 20)
    for g in [C.SmoeGrid(0, 64, 1, 0, 0, 3.0), C.SmoeGrid(64, 64, 0, 0, 0, 3.0),
              C.SmoeGrid(64, 64, 1, 0, 0, 0.0), C.SmoeGrid(64, 64, 1, 0, 0, float("nan")),
              C.SmoeGrid(64, 64, 1, 1 << 23, 0, 3.0), C.SmoeGrid(70000, 64, 1, 0, 0, 3.0),
              # the radius range [2^-30, 2^30]
              C.SmoeGrid(64, 64, 1, 0, 0, 2.0 ** -31), C.SmoeGrid(64, 64, 1, 0, 0, 2.0 ** 31),
              C.SmoeGrid(64, 64, 1, 0, 0, float("inf"))]:
        assert lib.smoe_bin(ct.byref(m), ct.byref(g), ct.byref(b), None) == C.SMOE_ERR_INVALID
    # the rule's variants: sharpening factor, box, regression mode, truncation reading
    for fields in [dict(sharpen=-1.0), dict(sharpen=float("nan")), dict(sharpen=float("inf")),
                   dict(box=2), dict(box=-1), dict(mode=2), dict(trunc=2), dict(trunc=-1)]:
        g = C.SmoeGrid(64, 64, 1, 0, 0, 3.0)
        for k, v in fields.items():
            setattr(g, k, v)
        assert lib.smoe_bin(ct.byref(m), ct.byref(g), ct.byref(b), None) == C.SMOE_ERR_INVALID, fields
    for ok in [dict(sharpen=2.5), dict(box=1), dict(mode=1), dict(trunc=1)]:
        g = C.SmoeGrid(80, 80, 1, 0, 0, 3.0)
        for k, v in ok.items():
            setattr(g, k, v)
        # valid fields: the call gets as far as the size check (80x80 needs 25 blocks, the
        # workspace holds 16), still before any launch
        assert lib.smoe_bin(ct.byref(m), ct.byref(g), ct.byref(b), None) == C.SMOE_ERR_TOO_LARGE, ok
    # the backward (and the fit step) take no sharpening
    sharp = C.SmoeGrid(64, 64, 1, 0, 0, 3.0)
    sharp.sharpen = 2.0
    q = 1 << 20
    assert lib.smoe_render_backward(ct.byref(m), ct.byref(sharp), ct.byref(b), q, q, q, None, q,
                                    None) == C.SMOE_ERR_INVALID
    # more blocks than the workspace holds (16): 80x80 needs 25
    big = C.SmoeGrid(80, 80, 1, 0, 0, 3.0)
    assert lib.smoe_bin(ct.byref(m), ct.byref(big), ct.byref(b), None) == C.SMOE_ERR_TOO_LARGE
    # render needs an image; backward needs exactly one of grad_image / target
    assert lib.smoe_render(ct.byref(m), ct.byref(good_grid), ct.byref(b), None, None, None, None,
                           None) == C.SMOE_ERR_INVALID
    p = 1 << 20
    assert lib.smoe_render_backward(ct.byref(m), ct.byref(good_grid), ct.byref(b), p, p, None,
                                    None, p, None) == C.SMOE_ERR_INVALID
    assert lib.smoe_render_backward(ct.byref(m), ct.byref(good_grid), ct.byref(b), p, p, p, p, p,
                                    None) == C.SMOE_ERR_INVALID
    assert lib.smoe_materialize(4, 3, 1, None, None, None) == C.SMOE_ERR_INVALID
    assert lib.smoe_fit_step(None, p, None, None) == C.SMOE_ERR_INVALID
    # window fusion: the displacement must divide the window; sizes and pointers checked
    for args in [(p, 3, 40, 40, 16, 3, p), (p, 3, 40, 40, 16, 0, p), (p, 2, 40, 40, 16, 4, p),
                 (p, 3, 0, 40, 16, 4, p), (p, 3, 40, 40, 2048, 4, p), (None, 3, 40, 40, 16, 4, p),
                 (p, 3, 40, 40, 16, 4, None), (p, 3, 40, 70000, 16, 4, p)]:
        assert lib.smoe_fuse_windows(*args, None) == C.SMOE_ERR_INVALID, args
    # the issue-rate probe
    for args in [(3, 16, 8, p), (-1, 16, 8, p), (0, 0, 8, p), (0, 16, 0, p), (0, 16, 8, None),
                 (0, 16, (1 << 20) + 1, p)]:
        assert lib.smoe_issue_probe(*args, None) == C.SMOE_ERR_INVALID, args


def test_segments_layout_host_only():
    from paper_2510_05814_amd import _capi as C

    segs = (C.SmoeSegment * 3)()
    for i, (w, h, k, sc) in enumerate([(33, 17, 5, 1), (16, 16, 0, 2), (100, 40, 7, 3)]):
        segs[i].width, segs[i].height, segs[i].num_kernels, segs[i].scale = w, h, k, sc
    K, T, px = C.smoe_segments_layout(segs)
    assert (K, T, px) == (12, 3 * 2 + 1 + 7 * 3, 33 * 17 + 256 + 4000)
    assert [s.kernel_offset for s in segs] == [0, 5, 5]
    assert [s.tile_offset for s in segs] == [0, 6, 7]
    assert [s.pixel_offset for s in segs] == [0, 561, 817]
    segs[1].scale = 0
    with pytest.raises(C.SmoeError):
        C.smoe_segments_layout(segs)


def test_one_hip_runtime_per_process():
    """Importing the package before torch must not load a second HIP runtime: the library
    binds to the libamdhip64 torch loads."""
    code = ("import paper_2510_05814_amd.serve, torch\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "libs = {ln.split()[-1] for ln in maps if 'libamdhip64' in ln}\n"
            "print(len(libs), sorted(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                         check=True).stdout
    assert out.startswith("1 "), out


def test_python_rule_settings_validated():
    """make_grid takes the rule's settings by name and refuses unknown ones (host only)."""
    import paper_2510_05814_amd as smoe
    from paper_2510_05814_amd import _capi as C

    g = smoe.make_grid(32, 16, 2, 1, 3, 3.0, sharpen=1.5, box="tight", mode="rbf",
                       trunc="render")
    assert (g.box, g.mode, g.trunc) == (C.SMOE_BOX_TIGHT, C.SMOE_MODE_RBF, C.SMOE_TRUNC_RENDER)
    assert abs(g.sharpen - 1.5) < 1e-7 and g.scale == 2 and g.origin_y == 3
    d = smoe.make_grid(8, 8)
    assert (d.sharpen, d.box, d.mode, d.trunc) == (1.0, C.SMOE_BOX_SQUARE, C.SMOE_MODE_SMOE,
                                                   C.SMOE_TRUNC_GRADIENT)
    for bad in (dict(box="round"), dict(mode="gauss"), dict(trunc="both")):
        with pytest.raises(ValueError):
            smoe.make_grid(8, 8, **bad)
