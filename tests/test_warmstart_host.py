"""Host logic of the learned warm start: the guard's decision rule and the summary of a
time-to-tolerance evaluation (no device needed)."""
import math

from paper_2202_08627_amd.warmstart import guard_choice, summarize


def test_guard_takes_network_only_when_no_worse():
    assert guard_choice({"zero": 10.0, "single_shot": 5.0, "unet": 4.0}) == "unet"
    assert guard_choice({"zero": 10.0, "single_shot": 5.0, "unet": 5.0}) == "unet"
    assert guard_choice({"zero": 10.0, "single_shot": 5.0, "unet": 6.0}) == "single_shot"
    assert guard_choice({"zero": 3.0, "single_shot": 5.0, "unet": 4.0}) == "zero"
    assert guard_choice({"zero": 3.0, "single_shot": 5.0}) == "zero"
    assert guard_choice({"zero": 10.0, "single_shot": 5.0}) == "single_shot"


def test_guard_rejects_non_finite_costs():
    assert guard_choice({"zero": 10.0, "single_shot": 5.0, "unet": math.nan}) == "single_shot"
    assert guard_choice({"zero": 10.0, "single_shot": math.inf, "unet": math.inf}) == "zero"
    assert guard_choice({"zero": 10.0, "single_shot": math.nan, "unet": 7.0}) == "unet"


def test_summary_medians_and_ratios():
    def rec(kz, kn, tz, tn):
        return {"zero": {"iters": kz, "t_total_s": tz, "err0": 1.0, "choice": "zero"},
                "unet": {"iters": kn, "t_total_s": tn, "err0": 0.2, "choice": "unet"}}
    s = summarize([rec(200, 150, 2.0, 1.0), rec(100, 100, 1.0, 1.0), rec(300, None, 3.0, None)])
    assert s["zero"]["median_iters"] == 200 and s["zero"]["reached"] == 3
    assert s["unet"]["reached"] == 2 and s["unet"]["median_iters"] == 125
    assert s["ratio_time_unet_vs_zero"] == 0.75
    assert s["ratio_iters_unet_vs_zero"] == 0.875
