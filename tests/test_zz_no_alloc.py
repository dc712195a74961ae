"""lb_audit_static: the audit without the caller's scratch (for callers that
cannot allocate device memory) against lb_audit on the same lattice, and
against the oracle's lattice totals (paper, Section 3: the quantities the
collide conserves)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lattice(lx, ly, precision, layout, steps, seed):
    from paper_1804_01918_amd import inputs, lb
    fields = inputs.random_equilibrium(lx, ly, seed=seed)
    lat = lb.Lattice(lx, ly, 0.8, fields, precision=precision, layout=layout, audit=False)
    lat.step(steps)
    return lat, fields


def _oracle_totals(fields, steps):
    from oracle import lbm
    return lbm.audit(lbm.run(lbm.init(*fields), 0.8, steps))


@pytest.mark.parametrize("first,second", [
    ((96, 640, "f64", "soa", 3), (24, 64, "f32s", "caosoa", 2)),
    ((80, 512, "f32s", "csoa", 2), (7, 33, "f64", "aos", 4)),
])
def test_audit_static_equals_audit(first, second):
    """Two calls in a row, the second on a smaller lattice (fewer partials in
    the library's array than the first call left there): each equals
    lb_audit of the same state bit for bit (same kernels, same order) and
    the oracle's totals within 1e-13 of the mass."""
    import torch
    from paper_1804_01918_amd import lb
    for seed, (lx, ly, prec, layout, steps) in enumerate((first, second)):
        print(f"lb_audit_static: {lx}x{ly} {prec} {layout}, {steps} steps", flush=True)
        lat, fields = _lattice(lx, ly, prec, layout, steps, seed)
        try:
            got = lb.lb_audit_static(lat.ctx)
            ref = lb.lb_audit(lat.ctx)
            torch.cuda.synchronize()
        finally:
            lat.close()
        assert np.array_equal(got, ref), (got, ref)
        if prec == "f64":
            orc = _oracle_totals(fields, steps)
            assert np.all(np.abs(got - orc) <= 1e-13 * orc[0]), (got, orc)


def test_audit_static_after_fused_audit():
    """A lattice whose last lb_step fused its audit: lb_audit takes the fused
    partials, lb_audit_static reduces the buffer again; equal bit for bit."""
    import torch
    from paper_1804_01918_amd import inputs, lb
    fields = inputs.random_equilibrium(64, 256, seed=3)
    lat = lb.Lattice(64, 256, 0.8, fields, precision="f64", layout="caosoa", audit=True)
    try:
        lat.step(2)
        ref = lb.lb_audit(lat.ctx)
        got = lb.lb_audit_static(lat.ctx)
        torch.cuda.synchronize()
    finally:
        lat.close()
    assert np.array_equal(got, ref), (got, ref)


def test_audit_static_rejects_lattices_beyond_its_array():
    """2^18 + 1 row tiles (a 262145 x 1 lattice, 19 MB of FP16 populations)
    exceed the library's array: LB_EINVAL, nothing launched."""
    from paper_1804_01918_amd import inputs, lb
    lx, ly = (1 << 18) + 1, 1
    lat = lb.Lattice(lx, ly, 0.8, inputs.random_equilibrium(lx, ly, seed=0), precision="f16s", layout="soa")
    try:
        with pytest.raises(lb.LBError) as e:
            lb.lb_audit_static(lat.ctx)
        assert e.value.code == lb.LB_EINVAL
        # the context stays usable
        assert np.isfinite(lat.audit()).all()
    finally:
        lat.close()
