"""GPU energy around a timed region, from the accumulated-energy counter that
the AMD SMI library exposes for the device (read only).

The paper's second figure of merit is energy to solution (its Section 5,
Fig. 4); here the counterpart is the energy per lattice update of the fused
step on the GPU package, read before and after a synchronised region.
"""
from __future__ import annotations


class EnergyMeter:
    """Reads the energy counter of the GPU that torch calls `device`,
    matched by PCI bus id. `available` is False (and `reason` says why) when
    the SMI library or the counter cannot be used; measurements are then None."""

    def __init__(self, device: int = 0):
        self.available = False
        self.reason = ""
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
                bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)  # "dddd:bb:dd.f"
                dom, bus, rest = bdf.split(":")
                dev = rest.split(".")[0]
                if (int(dom, 16), int(bus, 16), int(dev, 16)) == want:
                    self._h = h
                    break
            if self._h is None:
                self.reason = f"no SMI device with PCI id {want}"
                return
            self._read()
            self.available = True
        except Exception as e:  # no SMI library, no permission, no counter
            self.reason = f"{type(e).__name__}: {e}"

    def _read(self) -> float:
        """Accumulated energy in joules."""
        r = self._smi.amdsmi_get_energy_count(self._h)
        return r["energy_accumulator"] * r["counter_resolution"] * 1e-6

    def measure(self, fn):
        """Run fn() (which must synchronise the GPU before returning) and
        return (joules, seconds), or (None, seconds) without a counter."""
        import time
        e0 = self._read() if self.available else None
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        if e0 is None:
            return None, dt
        return self._read() - e0, dt

    def close(self):
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:
                pass
            self._smi = None
