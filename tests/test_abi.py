"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/jacobi.h declares, and rejects bad descriptors with negative
status codes (validation happens before any HIP call)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header, prefix):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(%s[a-z_0-9]+)\s*\(" % prefix, src)))


def test_library_exports_every_declared_symbol():
    import paper_1006_3148_amd as pkg
    from paper_1006_3148_amd import guess
    names = _declared("jacobi.h", "jacobi_")
    assert "jacobi_create" in names and "jacobi_batch_sweep" in names
    for n in names:
        assert hasattr(pkg.lib, n), n
    assert set(names) == set(pkg._lib.EXPORTED)
    gnames = _declared("jacobi_guess.h", "jg_")
    assert "jg_forward" in gnames
    for n in gnames:
        assert hasattr(pkg.lib, n), n
    assert set(gnames) == set(guess.EXPORTED)


def test_guess_sizes_and_errors():
    from paper_1006_3148_amd import lib, param_count
    from oracle import conv as cv
    for L in (2, 3, 4):
        assert param_count(L) == sum(int(np.prod(s)) for _, s in cv.param_shapes(L))
    n = ctypes.c_size_t()
    assert lib.jg_workspace_size(12, 4, ctypes.byref(n)) == -1   # 12 % 8 != 0
    assert lib.jg_workspace_size(16, 7, ctypes.byref(n)) == -1   # levels
    assert lib.jg_workspace_size(16, 4, ctypes.byref(n)) == 0 and n.value > 0
    h = ctypes.c_void_p()
    assert lib.jg_create(16, 4, None, None, None, None, None, 0, None, ctypes.byref(h)) == -1


def test_conv_layer_argument_errors():
    """The single-layer entry points reject bad sizes, strides, null buffers
    and short workspaces before touching the GPU."""
    from paper_1006_3148_amd import guess
    lib = guess.lib
    n = ctypes.c_size_t()
    assert lib.jg_conv3_workspace_size(7, 2, ctypes.byref(n)) == -1    # 7 % 2
    assert lib.jg_conv3_workspace_size(8, 3, ctypes.byref(n)) == -1    # stride
    assert lib.jg_conv3_workspace_size(0, 1, ctypes.byref(n)) == -1
    assert lib.jg_conv3_workspace_size(16, 2, ctypes.byref(n)) == 0 and n.value > 27 * 512
    assert lib.jg_conv3_forward(None, 8, 1, 1, 1, 1, None) == -1
    assert lib.jg_conv3_forward(1, 9, 1, 1, 2, 1, None) == -1
    assert lib.jg_conv3_backward_data(1, 8, 1, 1, 1, None, 0, None) == -3
    assert lib.jg_conv3_backward_weight(1, 8, 1, 1, 1, None, 0, None) == -3


def _desc(**kw):
    from paper_1006_3148_amd._lib import JacobiDesc
    d = JacobiDesc()
    d.nx, d.ny, d.nz = kw.pop("dims", (8, 8, 8))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _rc(fn, *args):
    return fn(*args)


@pytest.mark.parametrize("kw,code", [
    (dict(dims=(0, 8, 8)), -1),
    (dict(dims=(8, -1, 8)), -1),
    (dict(dims=(70000, 8, 8)), -1),
    (dict(dtype=7), -1),
    (dict(layout=3), -1),
    (dict(t=9), -2),
    (dict(t=-1), -2),
    (dict(inner_sweeps=-3), -1),
    (dict(tile_rows=33, rows_per_wave=4), -1),
    (dict(tile_rows=24, rows_per_wave=4), -2),
    (dict(stencil=5), -1),
    (dict(stencil=27, dtype=1), -2),
    (dict(stencil=27, layout=1), -2),
    (dict(stencil=27, teams=2), -2),
    (dict(stencil=27, t=5), -2),
    (dict(stencil=27, t=3, tile_rows=48, rows_per_wave=4), -2),
])
def test_bad_descriptors_are_rejected(kw, code):
    from paper_1006_3148_amd import lib
    d = _desc(**kw)
    n = ctypes.c_size_t()
    assert lib.jacobi_workspace_size(ctypes.byref(d), ctypes.byref(n)) == code
    h = ctypes.c_void_p()
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == code
    assert h.value is None
    assert lib.jacobi_last_error().decode() != ""


def test_stencil27_descriptors_plan_without_a_gpu():
    from paper_1006_3148_amd import lib
    n = ctypes.c_size_t()
    for t in (0, 1, 2, 3, 4):
        d = _desc(dims=(100, 70, 30), stencil=27, t=t)
        assert lib.jacobi_workspace_size(ctypes.byref(d), ctypes.byref(n)) == 0
    # every compiled 27-point shape is accepted for its t
    for t, rows, rpw in ((1, 32, 4), (2, 32, 4), (2, 36, 3), (2, 32, 2), (3, 24, 3),
                         (3, 32, 4), (4, 24, 3)):
        d = _desc(dims=(100, 70, 30), stencil=27, t=t, tile_rows=rows, rows_per_wave=rpw)
        assert lib.jacobi_workspace_size(ctypes.byref(d), ctypes.byref(n)) == 0, (t, rows)


def test_create_checks_buffers_before_touching_the_gpu():
    from paper_1006_3148_amd import lib
    d = _desc()
    h = ctypes.c_void_p()
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == -1  # grid0 null
    d.grid0 = 4096
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == -1  # grid1 null
    d.grid1 = 4096
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == -1  # same grid
    d.grid1 = 8192 + 8
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == -1  # misaligned
    d.grid1 = 8192
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == -3  # workspace
    d.workspace = 1 << 20
    d.workspace_bytes = 16
    assert lib.jacobi_create(ctypes.byref(d), ctypes.byref(h)) == -3
    assert lib.jacobi_create(ctypes.byref(d), None) == -1


def test_sizes():
    from paper_1006_3148_amd import lib
    d = _desc(dims=(10, 6, 4))
    n = ctypes.c_size_t()
    assert lib.jacobi_grid_bytes(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value == 12 * 8 * 6 * 8
    d.layout = 1
    d.t = 3
    assert lib.jacobi_grid_bytes(ctypes.byref(d), ctypes.byref(n)) == 0
    # box plus 2t shift planes in i and j, 2t + 2E in k with E = 2t
    assert n.value == 18 * 14 * (6 + 6 + 12) * 8
    d.seg_len = 8  # caps E at seg_len - 2t = 2
    assert lib.jacobi_grid_bytes(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value == 18 * 14 * (6 + 6 + 4) * 8
    d.seg_len = 0
    d.dtype = 1
    assert lib.jacobi_workspace_size(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value >= 3 * 12 * 8 * 6 * 4


def test_null_handle_calls_fail_cleanly():
    from paper_1006_3148_amd import lib
    assert lib.jacobi_sweep(None, 1) == -1
    l2 = ctypes.c_double()
    assert lib.jacobi_residual(None, ctypes.byref(l2), None) == -1
    assert lib.jacobi_sync(None) == -1
    assert lib.jacobi_destroy(None) == 0
    from paper_1006_3148_amd import guess
    assert guess.lib.jg_set_low_mode_weight(None, 1.0) == -1


def test_tile_menu():
    from paper_1006_3148_amd import tile_supported
    assert tile_supported(1, 64, 4)
    assert tile_supported(4, 32, 4)
    assert not tile_supported(4, 24, 4)
    assert not tile_supported(9, 32, 4)


def test_multigrid_shape_errors():
    """The multigrid dtype needs the A/B layout and an n^3 interior with
    n = 2^k - 1; other shapes are rejected before anything is allocated."""
    from paper_1006_3148_amd import lib
    n = ctypes.c_size_t()
    for dims, layout, rc in (((31, 31, 31), 0, 0), ((32, 32, 32), 0, -2),
                             ((31, 31, 15), 0, -2), ((31, 31, 31), 1, -2)):
        d = _desc(dims=dims, dtype=2, layout=layout)
        assert lib.jacobi_workspace_size(ctypes.byref(d), ctypes.byref(n)) == rc, dims
