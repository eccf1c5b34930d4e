"""Performance model of Section VII-A/B (Eq. 1-5): when should a reduction
use fewer workers?

A "basic" configuration (one thread, one wavefront, one workgroup, ...) is
compared with a "more" configuration that has higher throughput but pays a
synchronization latency T_sync (Eq. 3: T_more = T + T_sync).  Concurrency
follows Little's law (Eq. 1: C = T * Thr).  With N bytes of input the basic
configuration wins when Eq. 2 holds:

    T_basic + max(0, N - C_basic) / Thr_basic < T_more + max(0, N - C_more) / Thr_more

which gives two switch points: N_m (Eq. 4) when N lies between the two
concurrencies, and N_l (Eq. 5) when N exceeds both.  All quantities share
one time unit (cycles in the paper) and bytes.

The library's default plan applies the same rule on MI355X: one workgroup
(no device-wide synchronization) below the switch point computed from
measured latencies and throughputs (``mi355x_single_workgroup_switch``),
the whole device above it.
"""
from __future__ import annotations

from dataclasses import dataclass


def concurrency(latency: float, throughput: float) -> float:
    """Eq. 1, Little's law: bytes in flight C = T * Thr."""
    return latency * throughput


def latency_more(t_basic: float, t_sync: float) -> float:
    """Eq. 3: the 'more' configuration pays the synchronization latency."""
    return t_basic + t_sync


def time_to_finish(n: float, latency: float, throughput: float, conc: float) -> float:
    """One side of Eq. 2: latency plus the bytes beyond the concurrency at
    the configuration's throughput."""
    return latency + max(0.0, n - conc) / throughput


def prefer_basic(n: float, t: float, t_sync: float, thr_basic: float, thr_more: float) -> bool:
    """Eq. 2: True when the basic configuration finishes first for n bytes."""
    c_basic = concurrency(t, thr_basic)
    t_m = latency_more(t, t_sync)
    c_more = concurrency(t, thr_more)  # concurrency is taken at the basic latency T
    return time_to_finish(n, t, thr_basic, c_basic) < time_to_finish(n, t_m, thr_more, c_more)


def switch_point_m(t: float, t_sync: float, thr_basic: float) -> float:
    """Eq. 4: N_m = (T + T_sync) * Thr_basic (n between the concurrencies)."""
    return (t + t_sync) * thr_basic


def switch_point_l(t_sync: float, thr_more: float, thr_basic: float) -> float:
    """Eq. 5: N_l = T_sync * Thr_more * Thr_basic / (Thr_more - Thr_basic)
    (n beyond both concurrencies)."""
    return t_sync * thr_more * thr_basic / (thr_more - thr_basic)


@dataclass
class Scenario:
    """One row pair of Tables III/IV: basic vs more."""
    name: str
    latency: float      # T (cycles)
    thr_basic: float    # bytes / cycle
    thr_more: float     # bytes / cycle
    t_sync: float       # cycles (the synchronization steps the 'more' side pays)

    def concurrency_basic(self) -> float:
        return concurrency(self.latency, self.thr_basic)

    def concurrency_more(self) -> float:
        return concurrency(self.latency, self.thr_more)

    def n_l(self) -> float:
        return switch_point_l(self.t_sync, self.thr_more, self.thr_basic)

    def n_m(self) -> float:
        return switch_point_m(self.latency, self.t_sync, self.thr_basic)

    def use_basic(self, n_bytes: float) -> bool:
        """Scenario rule of Section VII-A: (1) n within the basic
        concurrency -> basic; (2) n between the concurrencies -> compare
        with N_m; (3) beyond both -> compare with N_l."""
        if n_bytes <= self.concurrency_basic():
            return True
        if n_bytes <= self.concurrency_more():
            return n_bytes < self.n_m()
        return n_bytes < self.n_l()


def switch_point(t_basic: float, t_sync: float, thr_basic: float, thr_more: float) -> float:
    """Bytes below which the basic configuration wins, by the scenario rule
    of Section VII-A: within the basic concurrency always basic; between
    the concurrencies N_m (Eq. 4); beyond both N_l (Eq. 5).  Times and
    throughputs in any consistent units (e.g. us and bytes/us)."""
    c_basic = concurrency(t_basic, thr_basic)
    c_more = concurrency(t_basic, thr_more)
    n_m = switch_point_m(t_basic, t_sync, thr_basic)
    if c_basic < n_m <= c_more:
        return n_m
    return max(c_basic, switch_point_l(t_sync, thr_more, thr_basic))


# MI355X measurements (one GPU): one 1024-thread workgroup streaming fp32
# (fixed cost 4.2 us, 100 GB/s) against the device-wide atomic-ticket
# kernel (fixed cost 5.0 us, about 7000 GB/s) and the two-kernel relaunch
# path (6.9 us).  The library's default plan uses the same constants.
MI355X = {"t_single_us": 4.2, "thr_single_GBps": 100.0, "t_atomic_us": 5.0, "t_relaunch_us": 6.9,
          "thr_device_GBps": 7000.0}


def mi355x_single_workgroup_switch(versus: str = "atomic", m: dict = MI355X) -> float:
    """Bytes below which one workgroup beats the device-wide kernel on
    MI355X (scenario rule with the measured constants)."""
    t_more = m["t_atomic_us"] if versus == "atomic" else m["t_relaunch_us"]
    return switch_point(m["t_single_us"], t_more - m["t_single_us"], m["thr_single_GBps"] * 1e3,
                        m["thr_device_GBps"] * 1e3)
