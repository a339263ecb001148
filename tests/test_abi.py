"""The C-ABI library loads and exports every symbol its header declares (CPU only)."""
import ctypes
import os
import re

import pytest

pa = pytest.importorskip("paper_2604_07170_amd")


def test_library_exports_every_declared_symbol():
    lib = pa.load_library()
    decls = re.findall(r"\b(wfp2d_[a-z_0-9]+)\s*\(", open(pa.HEADER_PATH).read())
    assert len(set(decls)) >= 9
    for name in set(decls):
        assert hasattr(lib, name), name


def test_errors_are_status_codes_without_a_device():
    lib = pa.load_library()
    plan = ctypes.c_void_p()
    xy = (ctypes.c_double * 2)(0.0, 0.0)
    # bad arguments are rejected before any device call
    assert lib.wfp2d_init(ctypes.byref(plan), 0, xy, 1, xy, 0.1, 16, 1e-7, None) == -1   # no sources
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 0, xy, 0.1, 16, 1e-7, None) == -1   # no targets
    assert lib.wfp2d_init(ctypes.byref(plan), 1, None, 1, xy, 0.1, 16, 1e-7, None) == -1  # no coordinates
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, -0.1, 16, 1e-7, None) == -1
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, 0.1, 16, 0.5, None) == -1
    far = (ctypes.c_double * 2)(1.5, 0.0)
    assert lib.wfp2d_init(ctypes.byref(plan), 1, far, 1, xy, 0.01, 24, 1e-7, None) == -2
    # W too small for the tolerance: pi - 2b/W <= 0 (eq. dt)
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, 0.01, 8, 1e-7, None) == -3
    assert plan.value is None
    assert b"pi - 2b/W" in lib.wfp2d_last_error(None)
    assert lib.wfp2d_step(None, None) == -6
    assert lib.wfp2d_destroy(None) == 0
    with pytest.raises(pa.Wfp2dError):
        pa.host_eval(99, [], 1)


def test_graph_and_batch_entry_points_reject_without_a_device():
    lib = pa.load_library()
    assert lib.wfp2d_graph_capture(None, None, None) == -6
    assert lib.wfp2d_graph_launch(None) == -6
    b = ctypes.c_void_p()
    assert lib.wfp2d_batch_create(ctypes.byref(b), 0, None, None, None, 1, None) == -1
    assert b.value is None
    assert lib.wfp2d_batch_launch(None) == -6
    assert lib.wfp2d_batch_destroy(None) == 0


def test_spread_tile_entry_points_reject_without_a_device():
    lib = pa.load_library()
    ms = ctypes.c_double(0.0)
    assert lib.wfp2d_set_spread_tile(None, 3) == -6
    assert lib.wfp2d_time_spread(None, 3, 1, ctypes.byref(ms)) == -6
    o = pa.Opts()
    lib.wfp2d_default_opts(ctypes.byref(o))
    assert o.spread_tile == 0
    o.spread_tile = 9
    plan = ctypes.c_void_p()
    xy = (ctypes.c_double * 2)(0.0, 0.0)
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, 0.01, 24, 1e-7, ctypes.byref(o)) == -1
    o.spread_tile = 0
    o.nufft_tol = 1e-17
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, 0.01, 24, 1e-7, ctypes.byref(o)) == -1


def test_adjoint_and_state_entry_points_reject_without_a_device():
    lib = pa.load_library()
    h = ctypes.c_void_p()
    n = ctypes.c_int64(0)
    assert lib.wfp2d_adjoint_init(ctypes.byref(h), None) == -6
    assert lib.wfp2d_adjoint_init(None, None) == -1
    assert lib.wfp2d_evaluate_dot(None, None, None) == -6
    assert lib.wfp2d_state_bytes(None, ctypes.byref(n)) == -6
    assert lib.wfp2d_save_state(None, None, 0) == -6
    assert lib.wfp2d_load_state(None, None, 0) == -6
    assert lib.wfp2d_reset(None) == -6


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of wfp2d_opts and wfp2d_info have the header's field offsets
    and sizes (a C program built against include/wfp2d.h prints them)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "wfp2d.h"', "int main(void) {"]
    for cname, cls in (("wfp2d_opts", pa.Opts), ("wfp2d_info", pa.Info)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.dirname(pa.HEADER_PATH), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in (("wfp2d_opts", pa.Opts), ("wfp2d_info", pa.Info)):
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_boundary_options_default_off_and_are_validated():
    lib = pa.load_library()
    o = pa.Opts()
    lib.wfp2d_default_opts(ctypes.byref(o))
    assert o.host_pointers == 0 and o.check_finite == 0
    plan = ctypes.c_void_p()
    xy = (ctypes.c_double * 2)(0.0, 0.0)
    o.host_pointers = 2
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, 0.05, 24, 1e-7, ctypes.byref(o)) == -1
    o.host_pointers, o.check_finite = 0, 5
    assert lib.wfp2d_init(ctypes.byref(plan), 1, xy, 1, xy, 0.05, 24, 1e-7, ctypes.byref(o)) == -1
    assert b"check_finite" in lib.wfp2d_last_error(None)
    assert pa.STATUS[-7] == "ERR_NONFINITE"
