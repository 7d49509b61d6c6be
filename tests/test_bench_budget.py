"""Host-only checks of the benchmark's wall-clock budget arithmetic (no GPU).

The driver's command (--steps 20 --warmup 5) must finish inside its time
limit when one step of the default workload takes close to a minute: the
budget allows at most one long warmup, whole timed steps while another one
fits, and always at least one timed step.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def simulate(budget_s, setup_s, cpu_s, step_s, steps, warmup, est_s=None, reserve=bench.POST_RESERVE_S):
    """Run the bench's warmup and timed loops against a fake clock; returns
    (warmups, timed steps, end time)."""
    clk = FakeClock()
    b = bench.StepBudget(budget_s, t0=0.0, clock=clk)
    clk.t = setup_s + cpu_s

    def step():
        clk.t += step_s
        return (0.0, 0.0, 0.0)

    real = bench.time.perf_counter
    bench.time.perf_counter = clk
    try:
        wn, ws, est = bench.run_warmup(step, b, warmup, step_s if est_s is None else est_s, reserve)
        n, secs, _ = bench.run_timed(step, b, steps, est, reserve, lambda: None)
    finally:
        bench.time.perf_counter = real
    return wn, n, clk.t + reserve


def test_driver_command_fits_with_one_minute_steps():
    wn, n, end = simulate(bench.DEFAULT_BUDGET_S, setup_s=120.0, cpu_s=65.0, step_s=54.0, steps=20, warmup=5)
    assert wn == 1
    assert n >= 3
    assert end <= bench.DEFAULT_BUDGET_S
    assert end <= 600.0 - 60.0


def test_short_steps_run_every_requested_step():
    wn, n, end = simulate(480.0, setup_s=20.0, cpu_s=5.0, step_s=0.5, steps=20, warmup=5)
    assert (wn, n) == (5, 20)


def test_first_timed_step_always_runs():
    # setup already overran the budget: no warmup, one timed step, still a line
    wn, n, _ = simulate(100.0, setup_s=150.0, cpu_s=0.0, step_s=54.0, steps=20, warmup=5)
    assert (wn, n) == (0, 1)


def test_underestimated_step_is_corrected_after_the_first():
    # the probe said 10 s but a step takes 54 s: the loop stops on the measured time
    wn, n, end = simulate(480.0, setup_s=120.0, cpu_s=65.0, step_s=54.0, steps=20, warmup=0, est_s=10.0)
    assert wn == 0
    assert end <= 480.0 + 54.0
    assert n == int((480.0 - bench.POST_RESERVE_S - 185.0) // 54.0)


def test_steps_and_warmup_are_upper_bounds():
    wn, n, _ = simulate(10_000.0, setup_s=0.0, cpu_s=0.0, step_s=1.0, steps=3, warmup=2)
    assert (wn, n) == (2, 3)


def test_whole_problem_weights():
    d, t = bench.whole_problem_weight(40)
    assert (d, t) == (9880, 1560)
    assert d + t == 40 * 41 * 42 // 6 - 40
