"""GPU energy from the accumulated-energy counter that the AMD SMI library
exposes for the device package (read only).

The paper's second figure of merit is energy to solution (its Section 5,
Fig. 4). Here the counterpart is the average package power while a kernel
loop runs, times the loop's GPU time: energy per lattice update or per
kernel call.

The counter is refreshed by the firmware at its own interval (about once a
second, each value stamped with the firmware's time), so a read just before
and just after a short region can both return stale samples. The meter
therefore enqueues the work, polls the counter while the GPU is busy, and
takes the power between the first and the last refresh it sees inside the
run, on the counter's own timestamps.

At each refresh it also reads the device's metrics table: the current
graphics clock and the firmware's residency counter for package-power
throttling. Kernels that draw the board's power cap run below the
nominal 2.4 GHz; `last_clock_mhz` and `last_power_throttled` say by how
much and for what share of the run.
"""
from __future__ import annotations

import time


class EnergyMeter:
    """Energy counter of the GPU that torch calls `device`, matched by PCI id.
    `available` is False (and `reason` says why) when the SMI library or the
    counter cannot be used."""

    def __init__(self, device: int = 0):
        self.available = False
        self.reason = ""
        self.last_clock_mhz = None        # mean graphics clock over the last power_during run
        self.last_power_throttled = None  # share of that run under package-power throttling
        self._smi = None
        self._h = None
        try:
            import torch
            import amdsmi
            props = torch.cuda.get_device_properties(device)
            want = (int(props.pci_domain_id), int(props.pci_bus_id), int(props.pci_device_id))
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            for h in amdsmi.amdsmi_get_processor_handles():
                dom, bus, rest = amdsmi.amdsmi_get_gpu_device_bdf(h).split(":")  # "dddd:bb:dd.f"
                if (int(dom, 16), int(bus, 16), int(rest.split(".")[0], 16)) == want:
                    self._h = h
                    break
            if self._h is None:
                self.reason = f"no SMI device with PCI id {want}"
                return
            self._read()
            self.available = True
        except Exception as e:  # no SMI library, no permission, no counter
            self.reason = f"{type(e).__name__}: {e}"

    def _read(self):
        """(joules accumulated, counter timestamp)."""
        r = self._smi.amdsmi_get_energy_count(self._h)
        return r["energy_accumulator"] * r["counter_resolution"] * 1e-6, r["timestamp"]

    def _metrics(self):
        """(graphics clock in MHz or None, package-power throttle residency,
        residency sample count) from the metrics table; the two counters
        accumulate in the same firmware samples, so the ratio of their
        differences is the throttled share of the time between two reads."""
        try:
            m = self._smi.amdsmi_get_gpu_metrics_info(self._h)
        except Exception:
            return None, None, None
        num = lambda v: v if isinstance(v, int) else None  # noqa: E731  ("N/A" where unsupported)
        return num(m.get("current_gfxclk")), num(m.get("ppt_residency_acc")), num(m.get("accumulation_counter"))

    def power_during(self, launch_chunk, nchunks: int, done, poll_s: float = 0.001):
        """Enqueue GPU work as nchunks calls of launch_chunk() (asynchronous;
        the counter is polled between chunks, since enqueueing blocks once
        the queue is full) and poll until done() is true. Returns (average
        watts between the first and the last counter refresh seen while the
        work ran, seconds between them on the counter's clock, refreshes
        seen), or (None, 0.0, n) with fewer than two refreshes in the run."""
        if not self.available:
            for _ in range(nchunks):
                launch_chunk()
            while not done():
                time.sleep(poll_s)
            return None, 0.0, 0
        _, ts = self._read()
        samples = []
        metrics = []

        def poll():
            nonlocal ts
            e, t = self._read()
            if t != ts:
                ts = t
                samples.append((e, t))
                metrics.append(self._metrics())

        for _ in range(nchunks):
            launch_chunk()
            poll()
        while not done():
            poll()
            time.sleep(poll_s)
        clocks = [c for c, _, _ in metrics if c]
        self.last_clock_mhz = sum(clocks) / len(clocks) if clocks else None
        self.last_power_throttled = None
        if len(metrics) >= 2 and None not in metrics[0][1:] + metrics[-1][1:]:
            dn = metrics[-1][2] - metrics[0][2]
            if dn > 0:
                self.last_power_throttled = (metrics[-1][1] - metrics[0][1]) / dn
        if len(samples) < 2:
            return None, 0.0, len(samples)
        (e0, t0), (e1, t1) = samples[0], samples[-1]
        span = (t1 - t0) * 1e-9  # counter timestamps are in ns
        return (e1 - e0) / span, span, len(samples)

    def idle_power(self, seconds: float = 2.5):
        """(average watts, seconds sampled, refreshes) with no work queued by
        this process, over about `seconds` of counter refreshes."""
        t_end = time.perf_counter() + seconds
        return self.power_during(lambda: None, 1, lambda: time.perf_counter() >= t_end)

    def power_limit_watts(self):
        """The board's power cap in watts as the SMI library reports it (read
        only), or None if it cannot be read."""
        if not self.available:
            return None
        try:
            info = self._smi.amdsmi_get_power_cap_info(self._h)
            cap = info.get("power_cap") or info.get("max_power_cap")
            return float(cap) * 1e-6 if cap else None  # reported in microwatts
        except Exception:
            return None

    def close(self):
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:
                pass
            self._smi = None
