"""GPU parity of the plain D2Q37 step (propagate, collide, fused step,
moments, audit) against the FP64 oracle, through the C ABI.

Tolerances:
* propagate and every layout/fusion comparison: bit-exact;
* FP64 collide / step / moments: |f_gpu - f_oracle| / w_p <= 1e-12 (the
  oracle and the kernels evaluate the same polynomial in different orders,
  so they differ by rounding only).
"""
import math

import numpy as np
import pytest

from oracle import lbm
from paper_1804_01918_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1804_01918_amd import lb  # noqa: E402

LAYOUTS = ["soa", "aos", "csoa", "caosoa"]
VL = {"f64": 16, "f32s": 32, "f16s": 64}


def _ok_shape(prec, layout, lx, ly):
    return layout in ("soa", "aos") or ly % VL[prec] == 0


def _w(consts):
    return consts["w"][:, None, None]


def _noneq(lx, ly, seed, consts, amp=1e-3):
    f = lbm.init(*inputs.random_equilibrium(lx, ly, seed=seed, amp=0.03))
    return f + amp * _w(consts) * inputs.perturbation(f.shape, seed + 77)


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.fixture(scope="module")
def config1_oracle():
    """Config 1: 128 x 64, tau 0.8, 100 steps from a random equilibrium (seed 0)."""
    fields = inputs.random_equilibrium(128, 64, seed=0)
    return fields, lbm.run(lbm.init(*fields), 0.8, 100)


# ---- init ------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(128, 64), (37, 32), (3, 16)])
def test_init_matches_oracle_equilibrium(consts, layout, shape):
    lx, ly = shape
    fields = inputs.random_equilibrium(lx, ly, seed=1, amp=0.05)
    with lb.Lattice(lx, ly, 0.8, fields, layout=layout) as lat:
        got = lat.get_populations().cpu().numpy()
    ref = lbm.init(*fields)
    assert np.max(np.abs(got - ref) / _w(consts)) < 1e-14


# ---- propagate ---------------------------------------------------------------

PROP_SHAPES = [(8, 8), (37, 29), (3, 5), (1, 1), (1, 7), (6, 1), (2, 2), (128, 64), (5, 16), (21, 48),
               (7, 64), (9, 96), (3, 128), (4, 192)]


@pytest.mark.parametrize("prec", ["f64", "f32s", "f16s"])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", PROP_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_propagate_bit_exact(consts, prec, layout, shape):
    lx, ly = shape
    if not _ok_shape(prec, layout, lx, ly):
        pytest.skip("clustered layout needs LY % VL == 0")
    f0 = _noneq(lx, ly, 5, consts, amp=0.3)
    with lb.Lattice(lx, ly, 0.8, inputs.random_equilibrium(lx, ly), precision=prec, layout=layout) as lat:
        lat.set_populations(f0)
        before = lat.get_populations().cpu().numpy()
        lat.propagate()
        after = lat.get_populations().cpu().numpy()
    assert np.array_equal(_bits(after), _bits(lbm.propagate(before)))


def test_propagate_preserves_nan_payloads_f64(consts):
    lx, ly = 16, 32
    f0 = _noneq(lx, ly, 6, consts)
    payload = np.frombuffer(np.uint64(0x7FF8DEADBEEF0001).tobytes(), dtype=np.float64)[0]
    f0[3, 2, 5] = payload
    f0[30, 15, 31] = -np.inf
    with lb.Lattice(lx, ly, 0.8, inputs.random_equilibrium(lx, ly)) as lat:
        lat.set_populations(f0)
        lat.propagate()
        got = lat.get_populations().cpu().numpy()
    assert np.array_equal(_bits(got), _bits(lbm.propagate(f0)))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_propagate_period_is_identity(layout):
    lx, ly = 6, 16
    period = lx * ly // math.gcd(lx, ly)
    with lb.Lattice(lx, ly, 0.8, inputs.random_equilibrium(lx, ly, amp=0.05), layout=layout) as lat:
        start = lat.get_populations().cpu().numpy()
        for _ in range(period):
            lat.propagate()
        end = lat.get_populations().cpu().numpy()
    assert np.array_equal(_bits(start), _bits(end))


# ---- collide -----------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 3.0])
def test_collide_f64_matches_oracle(consts, layout, tau):
    lx, ly = 37, 32
    f0 = _noneq(lx, ly, 7, consts, amp=1e-2)
    with lb.Lattice(lx, ly, tau, inputs.random_equilibrium(lx, ly), layout=layout) as lat:
        lat.set_populations(f0)
        lat.collide()
        got = lat.get_populations().cpu().numpy()
    # One collide: both sides round O(10)-sized bracket terms of the outer
    # shells at 2^-53, and the deviation from equilibrium is scaled by 1/tau.
    assert np.max(np.abs(got - lbm.collide(f0, tau)) / _w(consts)) < 1e-13


# ---- full step -----------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
def test_config1_f64_100_steps(consts, config1_oracle, layout):
    fields, ref = config1_oracle
    with lb.Lattice(128, 64, 0.8, fields, layout=layout) as lat:
        lat.step(100)
        got = lat.get_populations().cpu().numpy()
        rho, ux, uy, T = (t.cpu().numpy() for t in lat.moments())
    assert np.max(np.abs(got - ref) / _w(consts)) < 1e-12
    r_rho, r_ux, r_uy, r_T = lbm.moments(ref)
    assert np.max(np.abs(rho - r_rho)) < 1e-12
    assert np.max(np.abs(ux - r_ux)) < 1e-12
    assert np.max(np.abs(uy - r_uy)) < 1e-12
    assert np.max(np.abs(T - r_T)) < 1e-12


@pytest.mark.parametrize("shape,steps", [((1, 1), 7), ((1, 9), 5), ((9, 1), 5), ((3, 3), 6), ((37, 29), 10),
                                         ((2, 5), 4)])
def test_small_and_ragged_lattices(consts, shape, steps):
    lx, ly = shape
    fields = inputs.random_equilibrium(lx, ly, seed=3, amp=0.03)
    f0 = _noneq(lx, ly, 8, consts)
    with lb.Lattice(lx, ly, 0.7, fields) as lat:
        lat.set_populations(f0)
        lat.step(steps)
        got = lat.get_populations().cpu().numpy()
    assert np.max(np.abs(got - lbm.run(f0, 0.7, steps)) / _w(consts)) < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32s", "f16s"])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("compensated", [True, False])
def test_fused_equals_split_bitwise(consts, prec, layout, compensated):
    if prec == "f64" and not compensated:
        pytest.skip("FP64 has no compensation switch")
    lx, ly = 24, 64
    fields = inputs.random_equilibrium(lx, ly, seed=2, amp=0.03)
    outs = []
    for fused in (True, False):
        with lb.Lattice(lx, ly, 0.8, fields, precision=prec, layout=layout, compensated=compensated) as lat:
            if fused:
                lat.step(6)
            else:
                for _ in range(6):
                    lat.propagate()
                    lat.collide()
            assert lat.steps_done() == 6
            outs.append(lat.get_populations().cpu().numpy())
    assert np.array_equal(_bits(outs[0]), _bits(outs[1]))


@pytest.mark.parametrize("prec", ["f64", "f32s", "f16s"])
def test_layouts_bitwise_identical(prec):
    lx, ly = 20, 128
    fields = inputs.shear_wave(lx, ly, seed=1)
    outs = []
    for layout in LAYOUTS:
        with lb.Lattice(lx, ly, 0.8, fields, precision=prec, layout=layout) as lat:
            lat.step(9)
            outs.append(lat.get_populations().cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(_bits(outs[0]), _bits(o))


def test_nsteps_zero_is_noop():
    fields = inputs.random_equilibrium(8, 16)
    with lb.Lattice(8, 16, 0.8, fields) as lat:
        a = lat.get_populations().cpu().numpy()
        lat.step(0)
        assert lat.steps_done() == 0 and lat.current_buffer() == 0
        b = lat.get_populations().cpu().numpy()
    assert np.array_equal(_bits(a), _bits(b))


@pytest.mark.parametrize("prec", ["f64", "f32s", "f16s"])
@pytest.mark.parametrize("layout", ["soa", "caosoa"])
def test_every_site_written_over_poisoned_buffer(prec, layout):
    lx, ly = 33, 64
    with lb.Lattice(lx, ly, 0.8, inputs.random_equilibrium(lx, ly), precision=prec, layout=layout) as lat:
        lat.bufs[1].fill_(0xFF)   # all-ones bytes: NaN in every precision
        lat.step(1)
        assert lat.current_buffer() == 1
        f = lat.get_populations().cpu().numpy()
    assert np.isfinite(f).all()


# ---- checkpoint / resume -----------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32s", "f16s"])
def test_checkpoint_resume_bitwise(prec):
    lx, ly = 16, 64
    fields = inputs.shear_wave(lx, ly, seed=4)
    with lb.Lattice(lx, ly, 0.8, fields, precision=prec) as lat:
        lat.step(50)
        raw = lat.raw_state()
        lat.step(50)
        a = lat.get_populations().cpu().numpy()
    with lb.Lattice(lx, ly, 0.8, fields, precision=prec) as lat2:
        lat2.load_raw_state(raw)
        lat2.step(50)
        b = lat2.get_populations().cpu().numpy()
    assert np.array_equal(_bits(a), _bits(b))


def test_checkpoint_through_canonical_f64():
    lx, ly = 16, 64
    fields = inputs.shear_wave(lx, ly, seed=4)
    with lb.Lattice(lx, ly, 0.8, fields) as lat:
        lat.step(50)
        f = lat.get_populations()
        lat.step(50)
        a = lat.get_populations().cpu().numpy()
    with lb.Lattice(lx, ly, 0.8, fields) as lat2:
        lat2.set_populations(f)
        lat2.step(50)
        b = lat2.get_populations().cpu().numpy()
    assert np.array_equal(_bits(a), _bits(b))


# ---- audit -----------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
def test_audit_matches_oracle_and_is_conserved(consts, layout):
    lx, ly = 64, 48
    fields = inputs.random_equilibrium(lx, ly, seed=9, amp=0.02)
    with lb.Lattice(lx, ly, 0.8, fields, layout=layout) as lat:
        a0 = lat.audit()
        lat.step(100)
        a1 = lat.audit()
        f = lat.get_populations().cpu().numpy()
    ref = lbm.audit(f)
    scale = np.array([a0[0], a0[0], a0[0], a0[3]])
    assert np.all(np.abs(a1 - ref) <= 1e-13 * scale)
    assert np.all(np.abs(a1 - a0) <= 1e-13 * scale)


@pytest.mark.parametrize("prec", ["f64", "f32s", "f16s"])
def test_fused_audit_equals_standalone(prec):
    lx, ly = 32, 64
    fields = inputs.random_equilibrium(lx, ly, seed=10, amp=0.02)
    with lb.Lattice(lx, ly, 0.8, fields, precision=prec, audit=True) as lat:
        lat.step(3)
        fused = lat.audit()
    with lb.Lattice(lx, ly, 0.8, fields, precision=prec, audit=False) as lat2:
        lat2.step(3)
        standalone = lat2.audit()
    assert np.array_equal(fused, standalone)


def test_audit_reports_nonfinite(consts):
    lx, ly = 8, 16
    f0 = _noneq(lx, ly, 1, consts)
    f0[4, 3, 3] = np.nan
    with lb.Lattice(lx, ly, 0.8, inputs.random_equilibrium(lx, ly)) as lat:
        lat.set_populations(f0)
        with pytest.raises(lb.LBNonFinite) as ei:
            lat.audit()
    assert np.isnan(ei.value.totals[0])


def test_misaligned_buffer_rejected():
    fields = inputs.random_equilibrium(8, 16)
    lat = lb.Lattice(8, 16, 0.8, fields)
    cfg = lb.Config.from_buffer_copy(lat.cfg)
    cfg.buf[1] = lat.bufs[1].data_ptr() + 8
    import ctypes
    ctx = ctypes.c_void_p()
    rc = lb.lib().lb_init(ctypes.byref(ctx), ctypes.byref(cfg), *[a.data_ptr() for a in lat._fields_keepalive])
    assert rc == lb.LB_EINVAL
    lat.close()


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48, 3 * 256 * 16 + 16])
def test_copy_kernel_bytes(nbytes):
    """The bandwidth-reference copy moves exactly the given bytes (one 16-byte
    word per thread, ragged last workgroup) and nothing past them."""
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.full((nbytes + 256,), 0xA5, dtype=torch.uint8, device="cuda")
    lb.device_copy(dst[:nbytes], src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert bool((dst[nbytes:] == 0xA5).all())
