"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/lb.h declares, reports its constants (pinned to the
oracle's quadrature solve) and rejects invalid configurations before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1804_01918_amd import lb

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "lb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lb_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("lb_init", "lb_propagate", "lb_collide", "lb_step", "lb_moments"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_binding_knows_every_entry_point(name):
    """Every declared call has a ctypes signature in the binding, and the
    step calls are also Python functions of the same name."""
    assert name in lb._SIGNATURES, name
    if name in ("lb_buffer_bytes", "lb_scratch_bytes", "lb_init", "lb_propagate", "lb_collide", "lb_step",
                "lb_moments", "lb_audit", "lb_destroy"):
        assert callable(getattr(lb, name)), name


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports(name):
    so = ctypes.CDLL(lb.LIB_PATH)
    assert hasattr(so, name), name


def test_constants_match_oracle(consts):
    r, w, c = lb.model_constants()
    assert np.array_equal(c, consts["c"])
    assert r == consts["r"]
    assert np.array_equal(w, consts["w"])


def test_buffer_and_scratch_sizes():
    assert lb.buffer_bytes(2048, 2048, "f64", "soa") == 2048 * 2048 * 37 * 8
    assert lb.buffer_bytes(2048, 2048, "f32s", "caosoa") == 2048 * 2048 * 37 * 4
    assert lb.buffer_bytes(8192, 8192, "f16s", "csoa") == 8192 * 8192 * 37 * 2
    assert lb.buffer_bytes(3, 5, "f64", "aos") % 256 == 0
    # clustered layouts need LY % VL == 0 (VL = 16/32/64 for f64/f32s/f16s)
    assert lb.buffer_bytes(4, 48, "f64", "csoa") > 0
    assert lb.buffer_bytes(4, 48, "f32s", "csoa") == 0
    assert lb.buffer_bytes(4, 64, "f16s", "caosoa") > 0
    # empty and oversized lattices
    assert lb.buffer_bytes(0, 8, "f64", "soa") == 0
    assert lb.buffer_bytes(8, 0, "f64", "soa") == 0
    assert lb.buffer_bytes(65536, 32768, "f64", "soa") == 0
    assert lb.scratch_bytes(0, 1) == 0
    assert lb.scratch_bytes(1, 1) >= 5 * 8


def test_scratch_holds_the_fallback_ring():
    """Scratch ends with the learned collide's fallback ring: 128 slots of
    160 bytes per wavefront, 8 wavefronts per workgroup, one workgroup per
    512-site tile up to 256 of them."""
    ring_wg = 8 * 128 * 160
    assert lb.scratch_bytes(1, 1) >= ring_wg
    assert lb.scratch_bytes(3, 1024) >= 6 * ring_wg
    assert lb.scratch_bytes(2048, 2048) >= 256 * ring_wg
    # capped at 256 workgroups: the ring part stops growing with the lattice
    big, bigger = lb.scratch_bytes(2048, 2048), lb.scratch_bytes(4096, 2048)
    assert bigger - big < 256 * ring_wg


# Rows longer than the kernels' 32-bit in-row byte offsets can address:
# ly * 37 * elem > 2^32 (AoS, CAoSoA) or ly * elem > 2^32 (SoA, CSoA).
ROW_LIMIT = [
    (8, 2 ** 24, "f64", "caosoa"),     # 8 x 2^24 FP64: two 39.7 GB buffers would fit the GPU
    (8, 2 ** 24, "f64", "aos"),
    (1, 60_000_000, "f16s", "aos"),    # 4.4 GB per buffer
    (1, 60_000_000, "f16s", "caosoa"),
    (3, 600_000_000, "f64", "soa"),    # 4.8e9 bytes in one population row
    (3, 600_000_000, "f64", "csoa"),
]


@pytest.mark.parametrize("lx,ly,prec,layout", ROW_LIMIT)
def test_buffer_bytes_rejects_rows_beyond_32bit_offsets(lx, ly, prec, layout):
    assert lb.buffer_bytes(lx, ly, prec, layout) == 0


def test_row_limit_boundary():
    # the largest accepted rows: ly * 37 * 8 <= 2^32 and ly * 8 <= 2^32
    last = (2 ** 32) // (37 * 8)
    assert lb.buffer_bytes(1, last, "f64", "aos") > 0
    assert lb.buffer_bytes(1, last + 1, "f64", "aos") == 0
    last_c = last - last % 16
    assert lb.buffer_bytes(1, last_c, "f64", "caosoa") > 0
    assert lb.buffer_bytes(1, last_c + 16, "f64", "caosoa") == 0
    assert lb.buffer_bytes(1, 2 ** 29, "f64", "soa") > 0
    assert lb.buffer_bytes(1, 2 ** 29 + 1, "f64", "soa") == 0
    # the same rows in SoA fit: only the interleaved layouts hit the limit
    assert lb.buffer_bytes(8, 2 ** 24, "f64", "soa") == 8 * 2 ** 24 * 37 * 8


def _cfg(**kw):
    c = lb.Config()
    c.lx, c.ly, c.tau = kw.get("lx", 8), kw.get("ly", 16), kw.get("tau", 0.8)
    c.precision, c.layout = kw.get("precision", 0), kw.get("layout", 0)
    c.compensated, c.audit = 1, 0
    c.buf[0], c.buf[1] = kw.get("b0", 0x10000), kw.get("b1", 0x20000)
    c.scratch = kw.get("scratch", 0x30000)
    c.scratch_bytes = kw.get("scratch_bytes", 1 << 20)
    c.stream = None
    c.gx, c.gy = kw.get("gx", 0.0), kw.get("gy", 0.0)
    c.walls = kw.get("walls", 0)
    c.t_bottom, c.t_top = kw.get("t_bottom", 1.0), kw.get("t_top", 1.0)
    return c


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), lb.LB_EINVAL),
    (dict(tau=0.3), lb.LB_EINVAL),
    (dict(tau=float("nan")), lb.LB_EINVAL),
    (dict(lx=0), lb.LB_EINVAL),
    (dict(ly=-4), lb.LB_EINVAL),
    (dict(lx=65536, ly=32768), lb.LB_EINVAL),
    (dict(precision=7), lb.LB_EUNSUPPORTED),
    (dict(layout=9), lb.LB_EUNSUPPORTED),
    (dict(layout=2, ly=24), lb.LB_EUNSUPPORTED),
    (dict(b0=0), lb.LB_EINVAL),
    (dict(b1=0x20008), lb.LB_EINVAL),
    (dict(b1=0x10000), lb.LB_EINVAL),
    (dict(scratch=0), lb.LB_EINVAL),
    (dict(scratch_bytes=8), lb.LB_EINVAL),
    (dict(gx=float("nan")), lb.LB_EINVAL),
    (dict(gy=1.5), lb.LB_EINVAL),
    (dict(walls=2), lb.LB_EINVAL),
    (dict(walls=1, t_bottom=0.0), lb.LB_EINVAL),
    (dict(walls=1, t_top=float("inf")), lb.LB_EINVAL),
    (dict(walls=1, t_top=-1.0), lb.LB_EINVAL),
])
def test_init_rejects_before_device_work(kw, code):
    """Every invalid configuration is refused by validation, before any HIP
    call (the fake device addresses here are never touched)."""
    ctx = ctypes.c_void_p()
    fake = 0x40000
    rc = lb.lib().lb_init(ctypes.byref(ctx), ctypes.byref(_cfg(**kw)), fake, fake, fake, fake)
    assert rc == code
    assert not ctx.value
    assert lb.lib().lb_last_error(None).decode()


@pytest.mark.parametrize("lx,ly,prec,layout", ROW_LIMIT)
def test_init_rejects_rows_beyond_32bit_offsets(lx, ly, prec, layout):
    """Refused by validation with LB_EUNSUPPORTED; the fake device
    addresses are never touched (no kernel is launched)."""
    ctx = ctypes.c_void_p()
    cfg = _cfg(lx=lx, ly=ly, precision=lb.PRECISIONS[prec], layout=lb.LAYOUTS[layout], scratch_bytes=1 << 40)
    fake = 0x40000
    rc = lb.lib().lb_init(ctypes.byref(ctx), ctypes.byref(cfg), fake, fake, fake, fake)
    assert rc == lb.LB_EUNSUPPORTED
    assert not ctx.value
    assert b"4 GiB" in lb.lib().lb_last_error(None)


def test_init_null_arguments():
    ctx = ctypes.c_void_p()
    assert lb.lib().lb_init(None, ctypes.byref(_cfg()), 1, 1, 1, 1) == lb.LB_EINVAL
    assert lb.lib().lb_init(ctypes.byref(ctx), None, 1, 1, 1, 1) == lb.LB_EINVAL
    assert lb.lib().lb_init(ctypes.byref(ctx), ctypes.byref(_cfg()), 0, 0x40000, 0x40000, 0x40000) == lb.LB_EINVAL


def test_null_context_calls():
    L = lb.lib()
    for fn in (L.lb_propagate, L.lb_collide):
        assert fn(None) == lb.LB_EINVAL
    assert L.lb_step(None, 1) == lb.LB_EINVAL
    assert L.lb_current_buffer(None) == -1
    L.lb_destroy(None)


def test_strerror():
    for code in (0, -1, -2, -3, -4):
        assert lb.lib().lb_strerror(code)
    assert lb.lib().lb_strerror(-99) == b"unknown error code"


def test_copy_rejects_misaligned():
    assert lb.lib().lb_copy(0x1000, 0x2008, 64, None) == lb.LB_EINVAL
    assert lb.lib().lb_copy(0x1000, 0x2000, 63, None) == lb.LB_EINVAL


def test_gelu16_rejects_bad_arguments():
    """Validated on the host before any launch: NULL pointers and negative
    counts are LB_EINVAL; n = 0 is a no-op."""
    L = lb.lib()
    assert L.lb_mlp_gelu16(None, 0x2000, 4, None) == lb.LB_EINVAL
    assert L.lb_mlp_gelu16(0x1000, None, 4, None) == lb.LB_EINVAL
    assert L.lb_mlp_gelu16(0x1000, 0x2000, -1, None) == lb.LB_EINVAL
    assert L.lb_mlp_gelu16(0x1000, 0x2000, 0, None) == lb.LB_OK
