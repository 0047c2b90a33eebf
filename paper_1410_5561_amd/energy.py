"""GPU energy to solution (the GPU counterpart of the paper's energy
measurements, Sec. IV-A and IV-C, Tables I-III, which read the CPU socket's
and the DRAM's energy through RAPL).

The meter reads the GPU's accumulated energy counter through the AMD SMI
library (``amdsmi_get_energy_count``: an accumulator in units of
``counter_resolution`` microjoules, kept by the firmware for the whole
socket), which comes with the time of its last update (ns).  A measurement
reads it before and after a region that ends with a device synchronisation;
the counter is updated in steps, so the energy difference is divided by the
difference of the counter's own timestamps (not by the wall time between the
reads) to give the region's average power, and the region's energy is that
power times its wall time.

    meter = EnergyMeter()          # None-safe: meter.ok tells whether it works
    j0 = meter.joules()
    ... run, synchronise ...
    j1 = meter.joules()
"""
from __future__ import annotations


class EnergyMeter:
    """Reads the accumulated energy of one GPU, in joules."""

    def __init__(self, index: int = 0):
        self.ok = False
        self.error = None
        self._smi = None
        self._h = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            handles = amdsmi.amdsmi_get_processor_handles()
            if not handles:
                raise RuntimeError("no GPU handle")
            self._smi = amdsmi
            self._h = handles[min(index, len(handles) - 1)]
            self.joules()  # probe once
            self.ok = True
        except Exception as e:  # library missing, no permission, no counter
            self.error = "%s: %s" % (type(e).__name__, e)

    def joules(self) -> float:
        return self.read()[0]

    def read(self):
        """(joules accumulated, seconds: the time of the counter's last update)."""
        e = self._smi.amdsmi_get_energy_count(self._h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6, e["timestamp"] * 1e-9

    def power_w(self):
        """The firmware's own average socket power in watts (a cross-check
        of the counter), or None."""
        try:
            info = self._smi.amdsmi_get_power_info(self._h)
            for k in ("average_socket_power", "current_socket_power", "socket_power"):
                v = info.get(k)
                if isinstance(v, (int, float)) and v > 0:
                    return float(v)
        except Exception:
            pass
        return None

    def clocks_mhz(self):
        """Current graphics (SYS) and memory clocks in MHz, or None."""
        try:
            t = self._smi.AmdSmiClkType
            sclk = self._smi.amdsmi_get_clock_info(self._h, t.SYS).get("clk")
            mclk = self._smi.amdsmi_get_clock_info(self._h, t.MEM).get("clk")
            if isinstance(sclk, (int, float)) and isinstance(mclk, (int, float)):
                return {"sclk": sclk, "mclk": mclk}
        except Exception:
            pass
        return None

    def close(self):
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:
                pass
            self._smi = None


def measure(meter: EnergyMeter, run, sync, min_seconds: float = 2.0, max_reps: int = 1000, on_sync=None):
    """Repeat ``run()`` until at least ``min_seconds`` have passed (after
    ``sync()``); return (repetitions, seconds, joules, mean of the firmware's
    power readings taken at the synchronisations, or None).  joules is the
    counter's average power over its own update times times the wall time.
    ``on_sync()``, if given, runs at each of those synchronisations."""
    import time
    sync()
    j0, ts0 = meter.read()
    t0 = time.perf_counter()
    reps = 0
    pw = []
    while True:
        run()
        reps += 1
        if reps % 4 == 0 or reps >= max_reps:
            sync()
            p = meter.power_w()
            if p is not None:
                pw.append(p)
            if on_sync is not None:
                on_sync()
            if time.perf_counter() - t0 >= min_seconds or reps >= max_reps:
                break
    sync()
    dt = time.perf_counter() - t0
    j1, ts1 = meter.read()
    joules = (j1 - j0) / (ts1 - ts0) * dt if ts1 > ts0 else j1 - j0
    return reps, dt, joules, (sum(pw) / len(pw) if pw else None)
