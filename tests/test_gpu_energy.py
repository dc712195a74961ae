"""The energy meter on the GPU (the paper's second figure of merit, energy
to solution, Section 5 and Fig. 4): the package energy counter is there,
the package power while the fused step runs lies between the idle power
and the board's power cap, and the energy of a loop scales with its length
(2N calls take twice the energy of N calls, within 10 %). The graphics
clock and power-throttle share read beside it are in range."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1804_01918_amd import inputs, lb  # noqa: E402
from paper_1804_01918_amd.energy import EnergyMeter  # noqa: E402


def _loop_energy(meter, lat, calls, chunk=10):
    """(watts, GPU seconds, joules) of `calls` fused steps."""
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nchunks = calls // chunk
    state = {"i": 0}

    def launch():
        if state["i"] == 0:
            start.record(lat.stream)
        lat.step(chunk)
        state["i"] += 1
        if state["i"] == nchunks:
            stop.record(lat.stream)

    torch.cuda.synchronize()
    watts, span, refreshes = meter.power_during(launch, nchunks, stop.query)
    stop.synchronize()
    secs = start.elapsed_time(stop) / 1e3
    assert watts is not None and refreshes >= 2, (watts, refreshes)
    return watts, secs, watts * secs


def test_energy_meter_on_the_fused_step():
    meter = EnergyMeter(0)
    assert meter.available, meter.reason
    L = 2048
    fields = [torch.from_numpy(a).cuda() for a in inputs.shear_wave(L, L, seed=0)]
    with lb.Lattice(L, L, 0.8, fields, precision="f64", layout="caosoa") as lat:
        lat.step(20)
        torch.cuda.synchronize()
        idle, _, nidle = meter.idle_power(2.5)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(lat.stream)
        lat.step(200)
        t1.record(lat.stream)
        t1.synchronize()
        per_step = t0.elapsed_time(t1) / 1e3 / 200
        n = int(2.5 / per_step) // 10 * 10
        w1, s1, j1 = _loop_energy(meter, lat, n)
        clk, thr = meter.last_clock_mhz, meter.last_power_throttled
        w2, s2, j2 = _loop_energy(meter, lat, 2 * n)
    cap = meter.power_limit_watts()
    meter.close()
    print(f"idle {idle} W ({nidle} refreshes); loop {w1:.0f} W for {s1:.2f} s, {w2:.0f} W for {s2:.2f} s; "
          f"cap {cap} W; J(2N)/2J(N) = {j2 / (2 * j1):.3f}; {j1 / (n * L * L) * 1e9:.1f} nJ per lattice update; "
          f"graphics clock {clk} MHz, power-throttled share {thr}")
    assert idle is not None and idle > 0
    assert idle < w1 and idle < w2
    if cap is not None:
        assert w1 <= 1.05 * cap and w2 <= 1.05 * cap
    assert abs(j2 / (2 * j1) - 1) <= 0.10
    # the metrics table, where the device has one: a clock within the part's
    # range (nominal 2.4 GHz) and a throttled share between 0 and 1
    if clk is not None:
        assert 100 <= clk <= 2600
    if thr is not None:
        assert 0.0 <= thr <= 1.0 + 1e-9
