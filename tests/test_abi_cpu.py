"""The C ABI on the CPU: the library loads, exports every declared entry
point, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "r360.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(r360_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2208_02705_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    from paper_2208_02705_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_field_params(L):
    assert L.r360_field_params(32, 10, 4) == 6212
    assert L.r360_field_params(64, 10, 4) == 18564
    assert L.r360_field_params(0, 10, 4) == -1


def test_status_strings(L):
    for s in (0, -1, -2, -3, -4, -5):
        assert L.r360_status_string(s)
    assert L.r360_status_string(7) == b"unknown status"


def test_null_arguments_rejected_before_launch(L):
    from paper_2208_02705_amd import _lib
    out = C.c_void_p()
    g = _lib.GridDesc(); m = _lib.MlpDesc()
    assert L.r360_scene_create(None, None, None, None, None, None, C.byref(out)) == _lib.R360_EINVAL
    assert b"NULL" in L.r360_last_error()
    assert L.r360_scene_create(C.byref(g), None, None, C.byref(m), None, None, None) == _lib.R360_EINVAL
    assert L.r360_equirect_create(0, 16, C.byref(out)) == _lib.R360_EINVAL
    assert L.r360_workspace_bytes(None, 10, 4) == 0
    opts = _lib.RenderOpts(0.0, 1.0, 4, 0)
    assert L.r360_render_rays(None, None, None, 4, C.byref(opts), None, None, None, None, 0, None) == _lib.R360_EINVAL
    assert L.r360_render_rays_noalloc(None, None, None, 4, C.byref(opts), None, None, None, None) == _lib.R360_EINVAL
    assert L.r360_adam_step(None, None, None, None, 4, 1, 1e-3, 0.9, 0.99, 1e-8, None) == _lib.R360_EINVAL
    assert L.r360_train_step(None, None, None, 4, None, C.byref(opts), None, None, None, None, 0, None) == _lib.R360_EINVAL


def test_bad_grid_and_network_rejected(L):
    """Descriptor checks run before any allocation: non power-of-two voxel,
    unsupported widths, out-of-range field counts."""
    from paper_2208_02705_amd import _lib
    out = C.c_void_p()
    dummy = C.c_void_p(0x1000)  # never dereferenced: the checks fail first
    g = _lib.GridDesc(); g.n[:] = [4, 4, 4]; g.lo[:] = [-4, -4, -4]; g.voxel = 0.3; g.threshold = 0.5
    m = _lib.MlpDesc(); m.n_fields = 2; m.hidden = 32; m.L_xyz = 10; m.L_dir = 4; m.half_extent = 4.0
    assert L.r360_scene_create(C.byref(g), dummy, dummy, C.byref(m), dummy, None, C.byref(out)) == _lib.R360_EINVAL
    g.voxel = 2.0
    m.hidden = 48
    assert L.r360_scene_create(C.byref(g), dummy, dummy, C.byref(m), dummy, None, C.byref(out)) == _lib.R360_EUNSUPPORTED
    m.hidden = 32; m.L_xyz = 8
    assert L.r360_scene_create(C.byref(g), dummy, dummy, C.byref(m), dummy, None, C.byref(out)) == _lib.R360_EUNSUPPORTED
    m.L_xyz = 10; m.n_fields = 0
    assert L.r360_scene_create(C.byref(g), dummy, dummy, C.byref(m), dummy, None, C.byref(out)) == _lib.R360_EINVAL
    m.n_fields = 2; m.half_extent = 0.0
    assert L.r360_scene_create(C.byref(g), dummy, dummy, C.byref(m), dummy, None, C.byref(out)) == _lib.R360_EINVAL


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2208_02705_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_occupancy_arguments_rejected(L):
    from paper_2208_02705_amd import _lib
    assert L.r360_occupancy_workspace_bytes(None) == 0
    g = _lib.OccDesc()
    g.n[:] = [8, 8, 8]; g.lo[:] = [-4.0] * 3; g.voxel = 1.0
    g.near_, g.far_ = 0.0, float("inf")
    g.l_hit, g.l_miss, g.l_min, g.l_max, g.min_opacity = 0.85, -0.4, -2.0, 3.5, 0.5
    assert L.r360_occupancy_workspace_bytes(C.byref(g)) == 2048 + 512
    for field, bad in (("voxel", 0.3), ("l_hit", -1.0), ("l_miss", 0.2), ("min_opacity", 2.0), ("far_", 0.0)):
        h = _lib.OccDesc.from_buffer_copy(g)
        setattr(h, field, bad)
        assert L.r360_occupancy_workspace_bytes(C.byref(h)) == 0, field
        assert L.r360_occupancy_update(C.byref(h), None, None, None, None, 1, None, None, None, None, 0,
                                       None) == _lib.R360_EINVAL
    assert L.r360_occupancy_update(C.byref(g), None, None, None, None, 1, None, None, None, None, 0,
                                   None) == _lib.R360_EINVAL
    assert L.r360_depth_uncertainty(None, None, None, 4, 4, None, None, None, None) == _lib.R360_EINVAL
    gd = _lib.GlobalDesc()
    assert L.r360_global_field_measure(C.byref(gd), None, None, None, 4, None, None, None, None, 0,
                                       None) == _lib.R360_EUNSUPPORTED


def test_assignment_arguments_rejected(L):
    from paper_2208_02705_amd import _lib
    n = (C.c_int32 * 3)(8, 8, 8)
    assert L.r360_assign_workspace_bytes(None) == 0
    assert L.r360_assign_workspace_bytes((C.c_int32 * 3)(0, 8, 8)) == 0
    assert L.r360_assign_workspace_bytes(n) > 512 * 13
    S = C.c_int64(0)
    assert L.r360_assign_fields(n, None, 0.5, 4, None, C.byref(S), None, 0, None) == _lib.R360_EINVAL
    b = (C.c_int32 * 3)(2, 2, 2)
    assert L.r360_assign_uniform_workspace_bytes(b) > 0
    assert L.r360_assign_uniform_workspace_bytes((C.c_int32 * 3)(0, 1, 1)) == 0
    nf = C.c_int32(0)
    assert L.r360_assign_uniform(n, None, 0.5, b, None, C.byref(nf), None, 0, None) == _lib.R360_EINVAL


def test_frames_arguments_rejected(L):
    from paper_2208_02705_amd import _lib
    assert L.r360_field_frames_workspace_bytes(0) == 0
    assert L.r360_field_frames_workspace_bytes(5) == 256
    g = _lib.GridDesc()
    assert L.r360_field_frames(C.byref(g), None, 4, None, None, None, 0, None) == _lib.R360_EINVAL
    assert L.r360_scene_set_frames(None, None, None, None) == _lib.R360_EINVAL


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's ctypes mirrors of the header's descriptor structs have
    the same size and field offsets as the C compiler gives them (a field
    added on one side only would be read as garbage by the other)."""
    import shutil
    import subprocess
    from paper_2208_02705_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = {"r360_grid_desc": _lib.GridDesc, "r360_mlp_desc": _lib.MlpDesc, "r360_render_opts": _lib.RenderOpts,
             "r360_global_desc": _lib.GlobalDesc, "r360_occ_desc": _lib.OccDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "r360.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c11", "-I", include, str(src), "-o", str(exe)], check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_host_helpers(L):
    """The learning-rate schedule (Sec. 6.3: 1e-3 decaying to 5e-5) and the
    update description's sensor logits are computed by the library."""
    import math
    from paper_2208_02705_amd import _lib
    assert L.r360_lr_schedule(0, 1000, 1e-3, 5e-5) == 1e-3
    assert abs(L.r360_lr_schedule(1000, 1000, 1e-3, 5e-5) - 5e-5) < 1e-18
    assert abs(L.r360_lr_schedule(5000, 1000, 1e-3, 5e-5) - 5e-5) < 1e-18
    assert abs(L.r360_lr_schedule(500, 1000, 1e-3, 5e-5) - math.sqrt(1e-3 * 5e-5)) < 1e-15
    assert math.isnan(L.r360_lr_schedule(-1, 1000, 1e-3, 5e-5))
    g = _lib.OccDesc()
    assert L.r360_occ_desc_init(C.byref(g), 128, -4.0, 0.0625, 0.0, float("inf"), 0.7, 0.4, -2.0, 3.5, 0.5) == 0
    assert list(g.n) == [128] * 3 and list(g.lo) == [-4.0] * 3
    assert g.l_hit == C.c_float(math.log(0.7 / 0.3)).value
    assert g.l_miss == C.c_float(math.log(0.4 / 0.6)).value
    assert (g.l_min, g.l_max, g.min_opacity) == (-2.0, 3.5, 0.5)
    assert L.r360_occ_desc_init(C.byref(g), 128, -4.0, 0.0625, 0.0, 1.0, 0.4, 0.4, -2.0, 3.5, 0.5) == _lib.R360_EINVAL
    assert L.r360_occ_desc_init(C.byref(g), 128, -4.0, 0.0625, 0.0, 1.0, 0.7, 0.5, -2.0, 3.5, 0.5) == _lib.R360_EINVAL
    o = C.c_void_p(1)
    c2w = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    assert L.r360_pinhole_rays(0, 4, 2.0, 2.0, c2w, o, o, None) == _lib.R360_EINVAL
    assert L.r360_pinhole_rays(4, 4, 0.0, 2.0, c2w, o, o, None) == _lib.R360_EINVAL
    assert L.r360_pinhole_rays(4, 4, 2.0, 2.0, c2w, None, o, None) == _lib.R360_EINVAL
