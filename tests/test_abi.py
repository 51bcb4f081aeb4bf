"""Host-side checks of the C ABI: the library loads, exports every symbol
include/eed4.h declares, and rejects bad arguments before any GPU work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eed4.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eed4_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2006_10406_amd import _lib
    return _lib.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("eed4_inpaint", "eed4_fsi_cycle", "eed4_backward", "eed4_inpaint_batched",
              "eed4_workspace_size", "eed4_strerror", "eed4_radius"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2006_10406_amd import _lib
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in _lib.EXPORTED


def test_radius(lib):
    assert lib.eed4_radius(0.0) == 0
    assert lib.eed4_radius(1.0) == 3
    assert lib.eed4_radius(1.5) == 5
    assert lib.eed4_radius(2.0) == 6
    assert lib.eed4_radius(2.66) == 8
    assert lib.eed4_radius(2.7) == -1
    assert lib.eed4_radius(-0.5) == -1
    assert lib.eed4_radius(float("nan")) == -1


def test_workspace_size(lib):
    import paper_2006_10406_amd as e
    p = e.params(0.05, 1.0, 0.05, 10, 20)
    n1 = e.eed4_workspace_size(e.EED4_OP_INPAINT, 1, 64, 64, p)
    assert n1 >= 2 * 64 * 64 * 4
    assert e.eed4_workspace_size(e.EED4_OP_INPAINT, 2, 64, 64, p) > n1
    assert e.eed4_workspace_size(e.EED4_OP_CYCLE, 1, 64, 64, p) >= 2 * 64 * 64 * 4
    assert e.eed4_workspace_size(e.EED4_OP_BACKWARD, 1, 64, 64, p) > 0
    assert e.eed4_workspace_size(e.EED4_OP_INPAINT, 0, 64, 64, p) == 0
    bad = e.params(-1.0, 1.0, 0.05, 10, 20)
    assert e.eed4_workspace_size(e.EED4_OP_INPAINT, 1, 64, 64, bad) == 0
    assert e.eed4_workspace_size(99, 1, 64, 64, p) == 0


def _call_inpaint(lib, p, ws=0x1000, wsz=1 << 40, B=1, H=8, W=8, ptr=0x2000):
    from paper_2006_10406_amd import _lib
    st = _lib.eed4_stats()
    return lib.eed4_inpaint(ptr, ptr, ptr, B, H, W, ctypes.byref(p), None, ws, wsz, None,
                            ctypes.byref(st), None)


def test_argument_errors_before_any_gpu_work(lib):
    import paper_2006_10406_amd as e
    ok = e.params(0.05, 1.0, 0.05, 10, 2)
    assert _call_inpaint(lib, e.params(0.05, 1.0, 0.07, 10, 2)) == e._lib.EED4_EUNSTABLE
    assert _call_inpaint(lib, e.params(0.0, 1.0, 0.05, 10, 2)) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, e.params(0.05, 3.0, 0.05, 10, 2)) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, e.params(0.05, 1.0, 0.05, 0, 2)) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, e.params(0.05, 1.0, 0.05, 10, 0)) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, e.params(0.05, 1.0, -0.01, 10, 2)) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, e.params(0.05, 1.0, 0.05, 10, 2, tol=-1.0)) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, ok, H=0) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, ok, H=1, W=(1 << 21) + 1) == e._lib.EED4_EINVAL   # width bound
    assert _call_inpaint(lib, ok, H=(1 << 24) + 1, W=1) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, ok, ptr=0) == e._lib.EED4_EINVAL
    assert _call_inpaint(lib, ok, ws=0) == e._lib.EED4_EWORKSPACE
    assert _call_inpaint(lib, ok, ws=0x1001) == e._lib.EED4_EWORKSPACE
    assert _call_inpaint(lib, ok, wsz=16) == e._lib.EED4_EWORKSPACE
    big = e.params(0.05, 1.0, 0.07, 10, 2, flags=e.EED4_ALLOW_LARGE_TAU)
    assert _call_inpaint(lib, big, ws=0) == e._lib.EED4_EWORKSPACE


def test_shape_families_partition_the_shape_ids():
    # every shape id is a tile or a strip shape, never both (results are bitwise equal within a
    # family); the names follow the family
    import paper_2006_10406_amd as e
    ids = set(range(len(e.SHAPE_NAMES)))
    assert set(e.TILE_SHAPES) | set(e.STRIP_SHAPES) == ids
    assert not set(e.TILE_SHAPES) & set(e.STRIP_SHAPES)
    assert all(e.SHAPE_NAMES[i].startswith("tile") for i in e.TILE_SHAPES)
    assert all(e.SHAPE_NAMES[i].startswith("strip") for i in e.STRIP_SHAPES)


def test_step_shape_query_without_tuning(lib):
    # no device work: forced shapes, the tile flag and the size rule used
    # before any tuning (strips when they give enough waves, else 32x32 tiles)
    import ctypes
    import paper_2006_10406_amd as e
    q = lambda B, H, W, p: lib.eed4_step_shape(B, H, W, ctypes.byref(p))
    for sh in range(len(e.SHAPE_NAMES)):
        assert q(1, 300, 200, e.params(0.05, 1.0, 0.05, 10, 2, flags=e.EED4_FORCE_SHAPE(sh))) == sh
    assert q(1, 300, 200, e.params(0.05, 1.0, 0.05, 10, 2, flags=e.EED4_TILE_KERNEL)) == 0
    assert q(1, 4096, 4096, e.params(0.02, 2.0, 0.05, 15, 2)) == 3
    assert q(1, 64, 64, e.params(0.05, 1.0, 0.05, 10, 2)) == 2
    assert q(1, 0, 64, e.params(0.05, 1.0, 0.05, 10, 2)) == e._lib.EED4_EINVAL
    assert q(1, 64, 64, e.params(0.05, 1.0, 0.05, 10, 2, flags=e.EED4_FORCE_SHAPE(99))) == \
        e._lib.EED4_EINVAL


def test_tensor_variant_flags(lib):
    # the variants of Table 7 / Sec. 3.1 run the 28-row strip kernels; bad fields and other
    # shapes are rejected before any device work, in every entry point
    import ctypes
    import paper_2006_10406_amd as e
    q = lambda p, B=1, H=300, W=200: lib.eed4_step_shape(B, H, W, ctypes.byref(p))
    EINVAL = e._lib.EED4_EINVAL
    for d in range(len(e.DIFFUSIVITY_NAMES)):
        for r in range(len(e.MU3_NAMES)):
            fl = e.EED4_DIFFUSIVITY(d) | e.EED4_MU3(r)
            p = e.params(0.05, 1.0, 0.05, 10, 2, flags=fl)
            want = 3 if fl == 0 else 5
            assert q(p, 1, 4096, 4096) == want
            if fl:
                assert q(p, 1, 40, 30) == 5
                assert e.eed4_workspace_size(e.EED4_OP_INPAINT, 1, 64, 64, p) > 0
                assert e.eed4_workspace_size(e.EED4_OP_BACKWARD, 1, 64, 64, p) > 0
    var = e.EED4_DIFFUSIVITY(e.EED4_PERONA_MALIK_EXP) | e.EED4_MU3(e.EED4_MU3_ARITHMETIC)
    assert q(e.params(0.05, 1.0, 0.05, 10, 2, flags=var | e.EED4_FORCE_SHAPE(5))) == 5
    assert q(e.params(0.05, 1.0, 0.05, 10, 2, flags=var | e.EED4_FORCE_SHAPE(3))) == EINVAL
    assert q(e.params(0.05, 1.0, 0.05, 10, 2, flags=var | e.EED4_TILE_KERNEL)) == EINVAL
    assert q(e.params(0.05, 1.0, 0.05, 10, 2, flags=e.EED4_DIFFUSIVITY(4))) == EINVAL
    assert q(e.params(0.05, 1.0, 0.05, 10, 2, flags=e.EED4_MU3(3))) == EINVAL
    assert _call_inpaint(lib, e.params(0.05, 1.0, 0.05, 10, 2, flags=e.EED4_MU3(3))) == EINVAL
    pv = e.params(0.05, 1.0, 0.05, 10, 2, flags=var)
    fake = 0x2000
    bad = e.params(0.05, 1.0, 0.05, 10, 2, flags=var | e.EED4_FORCE_SHAPE(3))
    assert lib.eed4_backward(fake, fake, fake, 1, 8, 8, ctypes.byref(bad), 2, fake, fake, fake,
                             fake, 0x1000, 1 << 40, None) == EINVAL
    img = e._lib.eed4_image(fake, fake, fake, 8, 8, 0.05)
    assert lib.eed4_inpaint_batched(ctypes.byref(img), 1, ctypes.byref(bad), 0x1000, 1 << 40,
                                    None, None) == EINVAL
    assert lib.eed4_batched_workspace_size(ctypes.byref(img), 1, ctypes.byref(pv)) > 0
    assert lib.eed4_batched_workspace_size(ctypes.byref(img), 1, ctypes.byref(bad)) == 0


def test_strerror(lib):
    import paper_2006_10406_amd as e
    for c in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(e.eed4_strerror(c), str) and e.eed4_strerror(c)


def test_static_cycle_size_limit_before_any_gpu_work(lib):
    # eed4_fsi_cycle_static rejects a problem whose cycle workspace exceeds its static
    # scratch with EED4_ETOOLARGE before touching the device (dummy pointers here)
    import paper_2006_10406_amd as e
    p = e.params(0.03, 1.5, 0.05, 10, 1)
    limit = e._lib.EED4_STATIC_SCRATCH_BYTES
    assert e.eed4_workspace_size(e.EED4_OP_CYCLE, 1, 3000, 3000, p) > limit
    assert e.eed4_workspace_size(e.EED4_OP_CYCLE, 1, 2048, 2048, p) <= limit
    ptr = 0x2000
    rc = lib.eed4_fsi_cycle_static(ptr, ptr, ptr, 1, 3000, 3000, ctypes.byref(p), None, ptr)
    assert rc == e._lib.EED4_ETOOLARGE
    assert b"static scratch" in lib.eed4_strerror(rc)
    bad = e.params(-1.0, 1.5, 0.05, 10, 1)
    assert lib.eed4_fsi_cycle_static(ptr, ptr, ptr, 1, 8, 8, ctypes.byref(bad), None,
                                     ptr) == e._lib.EED4_EINVAL
    assert lib.eed4_fsi_cycle_static(ptr, ptr, ptr, 1, 8, 8, ctypes.byref(p), None,
                                     None) == e._lib.EED4_EINVAL
