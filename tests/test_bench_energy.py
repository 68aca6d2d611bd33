"""Host logic of bench.py's energy-to-solution measurement (no GPU).

The GPU package's energy accumulator advances in steps (about once per
second on MI355X); the mean power must be taken between two of its updates
that both fall inside the busy period.  A simulated counter with a known
idle and busy power checks that the idle time before the run never leaks
into the window, for several update periods and phases.
"""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


class FakeCounter:
    """Accumulator sampled every `period` s of a virtual clock; power is
    `idle_w` until `busy_from`, `busy_w` afterwards."""

    def __init__(self, period, phase, idle_w, busy_w, busy_from):
        self.period, self.phase = period, phase
        self.idle_w, self.busy_w, self.busy_from = idle_w, busy_w, busy_from
        self.t = 0.0

    def energy_at(self, t):
        if t <= self.busy_from:
            return self.idle_w * t
        return self.idle_w * self.busy_from + self.busy_w * (t - self.busy_from)

    def read(self):
        # last update at or before the current time
        k = int((self.t - self.phase) // self.period)
        ts = self.phase + k * self.period
        return self.energy_at(ts), ts


@pytest.mark.parametrize("period,phase,solve_s", [(1.0, 0.37, 0.058), (1.0, 0.99, 0.1), (0.25, 0.1, 0.031),
                                                  (1.0, 0.0, 1.55)])
def test_steady_power_excludes_idle_lead_in(period, phase, solve_s):
    c = FakeCounter(period, phase, idle_w=250.0, busy_w=1077.0, busy_from=10.0)
    c.t = 10.0   # the run starts here, right after an idle stretch

    def work():
        c.t += solve_s

    watts, window, calls = bench.steady_power(c.read, work, min_window_s=4.0, clock=lambda: c.t)
    assert watts == pytest.approx(1077.0, rel=1e-12)
    assert window >= 4.0
    assert calls * solve_s >= window


def test_steady_power_needs_two_updates():
    c = FakeCounter(100.0, 0.0, 250.0, 1000.0, 0.0)   # counter far slower than the run cap
    c.t = 1.0

    def work():
        c.t += 0.5

    with pytest.raises(RuntimeError):
        bench.steady_power(c.read, work, min_window_s=4.0, max_run_s=5.0, clock=lambda: c.t)
