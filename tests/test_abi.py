"""Host-side checks of the C ABI: the library loads and exports every
symbol include/drr.h declares, and argument validation rejects bad input
before any device work (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_2208_12737_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "drr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(drr_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for n in ("drr_render", "drr_volume_pack", "drr_render_backward", "drr_ncc_forward",
              "drr_plan_create", "drr_plan_execute"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_version_and_status_strings():
    lib = _lib.load()
    assert lib.drr_version() >= 10000
    assert lib.drr_status_string(0) == b"ok"
    assert b"invalid" in lib.drr_status_string(_lib.DRR_EINVAL)


def test_packed_bytes_includes_zero_border():
    lib = _lib.load()
    d = _lib.volume_desc((4, 5, 6), (1, 1, 1), (0, 0, 0))
    assert lib.drr_volume_packed_bytes(ctypes.byref(d)) == 6 * 7 * 8 * 4


@pytest.mark.parametrize("shape,spacing", [((0, 5, 6), (1, 1, 1)), ((4, 5, 6), (1, 0, 1)),
                                           ((4, 5, 6), (1, float("nan"), 1))])
def test_invalid_volume_rejected(shape, spacing):
    lib = _lib.load()
    d = _lib.volume_desc(shape, spacing, (0, 0, 0))
    assert lib.drr_volume_packed_bytes(ctypes.byref(d)) == 0
    st = lib.drr_volume_pack(None, None, ctypes.byref(d), None)
    assert st == _lib.DRR_EINVAL
    assert lib.drr_last_error()


def test_render_validation_before_launch():
    lib = _lib.load()
    v = _lib.volume_desc((4, 4, 4), (1, 1, 1), (-2, -2, -2))
    good = _lib.detector_desc(8, 8, 1.0, 1.0)
    bad = _lib.detector_desc(0, 8, 1.0, 1.0)
    assert lib.drr_render(None, ctypes.byref(v), ctypes.byref(bad), None, 1, None, None,
                          None) == _lib.DRR_EINVAL
    assert lib.drr_render(None, ctypes.byref(v), ctypes.byref(good), None, -1, None, None,
                          None) == _lib.DRR_EINVAL
    # n_poses == 0 is a valid no-op, even with NULL buffers
    assert lib.drr_render(None, ctypes.byref(v), ctypes.byref(good), None, 0, None, None,
                          None) == _lib.DRR_OK
    # workspace queries
    assert lib.drr_backward_workspace_bytes(ctypes.byref(good), 3) >= 3 * 7 * 8
    assert lib.drr_ncc_workspace_bytes(2, 100) >= 2 * 5 * 8
    assert lib.drr_backward_workspace_bytes(ctypes.byref(bad), 3) == 0


def test_workspace_too_small_rejected():
    lib = _lib.load()
    det = _lib.detector_desc(16, 16, 1.0, 1.0)
    st = lib.drr_render_backward(ctypes.byref(det), 2, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), ctypes.c_void_p(16), 8, None)
    assert st == _lib.DRR_ENOMEM


def test_plan_rejects_bad_descriptors():
    lib = _lib.load()
    desc = _lib.PlanDesc()
    desc.max_items = 0
    out = ctypes.c_void_p()
    assert lib.drr_plan_create(ctypes.byref(desc), None, 0, None,
                               ctypes.byref(out)) == _lib.DRR_EINVAL
    assert lib.drr_plan_execute(None, None, 0, None) == _lib.DRR_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    """Without libdrr.so the first call raises; nothing falls back to a CPU
    path."""
    import subprocess
    import sys
    code = ("import paper_2208_12737_amd._lib as L; L.LIB_PATH = %r\n"
            "try:\n    L.load()\nexcept ImportError as e:\n    print('raised', e)\n"
            % str(tmp_path / "absent.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("raised"), r.stdout + r.stderr


def test_product_never_reaches_the_oracle():
    """The package neither imports nor loads anything from oracle/."""
    pkg = os.path.join(ROOT, "paper_2208_12737_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "liboracle" not in text and "drr_oracle" not in text, f


def test_plan_item_workspace_covers_every_launch_shape():
    """Scratch of an objective item: the most tiles any plan launch shape
    cuts the detector into (8 x 8 px tiles are the smallest), times 26
    float64 moment sums per tile."""
    lib = _lib.load()
    for (h, w), tiles in (((64, 64), 64), ((37, 53), 5 * 7), ((1, 1), 1), ((256, 256), 1024)):
        det = _lib.detector_desc(h, w, 1.0, 1.0)
        assert lib.drr_plan_item_workspace_bytes(ctypes.byref(det)) == tiles * 26 * 8
    bad = _lib.detector_desc(0, 8, 1.0, 1.0)
    assert lib.drr_plan_item_workspace_bytes(ctypes.byref(bad)) == 0
    assert lib.drr_plan_item_workspace_bytes(None) == 0


def test_work_item_layout_matches_header():
    """The binding's drr_work_item has the C struct's size and field offsets
    (LP64: 6 pointers of the original layout plus 4 for objective items)."""
    W = _lib.WorkItem
    assert W.det.offset == 8
    assert W.pose.offset == 8 + ctypes.sizeof(_lib.DetectorDesc)
    assert W.partials.offset == W.pose.offset + 7 * 8
    assert ctypes.sizeof(W) == W.partials.offset + 8


def test_packed_copy_size_limit():
    """Gathers address one zero-bordered copy with 32-bit byte offsets: a
    copy must stay below 4 GiB; the per-axis layout holds three copies."""
    lib = _lib.load()
    ok = _lib.volume_desc((1021, 1021, 1021), (1, 1, 1), (0, 0, 0))
    assert lib.drr_volume_packed_bytes(ctypes.byref(ok)) == 1023 ** 3 * 4
    ok3 = _lib.volume_desc((1021, 1021, 1021), (1, 1, 1), (0, 0, 0), _lib.DRR_LAYOUT_PER_AXIS)
    assert lib.drr_volume_packed_bytes(ctypes.byref(ok3)) == 3 * 1023 ** 3 * 4
    big = _lib.volume_desc((1022, 1022, 1022), (1, 1, 1), (0, 0, 0))
    assert lib.drr_volume_packed_bytes(ctypes.byref(big)) == 0
    assert lib.drr_volume_pack(None, None, ctypes.byref(big), None) == _lib.DRR_ENOTSUP
    assert b"4 GiB" in lib.drr_last_error()


def test_header_is_plain_c(tmp_path):
    """include/drr.h compiles as strict C99, and a C program links against
    libdrr.so and calls its host-only entry points (no GPU needed)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "use_drr.c"
    src.write_text(r"""
#include <stdio.h>
#include "drr.h"
int main(void)
{
    drr_detector_desc det = {64, 64, 1.0, 1.0, 0.0, 0.0};
    drr_volume_desc vol = {4, 5, 6, {1.0, 1.0, 1.0}, {0.0, 0.0, 0.0}, DRR_LAYOUT_INPUT};
    if (drr_version() < 10000) return 1;
    if (drr_plan_item_workspace_bytes(&det) != (size_t)64 * 26 * 8) return 2;
    if (drr_volume_packed_bytes(&vol) != (size_t)6 * 7 * 8 * 4) return 3;
    det.height = 0;
    if (drr_render(NULL, &vol, &det, NULL, 1, NULL, NULL, NULL) != DRR_EINVAL) return 4;
    if (drr_last_error()[0] == '\0') return 5;
    puts(drr_status_string(DRR_OK));
    return 0;
}
""")
    libdir = os.path.join(root, "paper_2208_12737_amd")
    exe = tmp_path / "use_drr"
    res = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                          "-I", os.path.join(root, "include"), str(src), "-L", libdir, "-ldrr",
                          f"-Wl,-rpath,{libdir}", "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, (run.returncode, run.stderr)
    assert run.stdout.strip() == "ok"


def test_noalloc_scratch_limit_matches_header_and_is_checked_on_the_host():
    src = open(os.path.join(ROOT, "include", "drr.h")).read()
    m = re.search(r"#define DRR_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.DRR_NOALLOC_SCRATCH_BYTES
    lib = _lib.load()
    vol = _lib.volume_desc((8, 8, 8), (1, 1, 1), (-4, -4, -4))
    det = _lib.detector_desc(256, 256, 1.0, 1.0)
    per_pose = lib.drr_ncc_grad_workspace_bytes(ctypes.byref(det), 1)
    n = _lib.DRR_NOALLOC_SCRATCH_BYTES // per_pose + 1
    # rejected before any device work: the pointers are never dereferenced
    st = lib.drr_render_ncc_grad_noalloc(8, ctypes.byref(vol), ctypes.byref(det), 8, n, 8, 0,
                                         None, 8, 8, None)
    assert st == _lib.DRR_ENOMEM
    assert b"scratch" in lib.drr_last_error()
