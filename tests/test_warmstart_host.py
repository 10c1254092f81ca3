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


def test_stable_crossing_on_a_monotone_error():
    from paper_2202_08627_amd.warmstart import first_stable_crossing
    err = lambda k: 1.0 / (1.0 + k)          # <= 1e-2 from k = 99 on
    k, e, checks = first_stable_crossing(err, 1.0, 1e-2, 500)
    assert k == 99 and e == err(99)
    assert checks["err_k_minus_1"] > 1e-2
    assert all(v <= 1e-2 for v in checks["probes"].values())


def test_stable_crossing_skips_a_crossing_that_is_undone():
    """The error dips below the tolerance at 95-105, rises above it again and stays below from
    160 on. Bisection over [0, 200] alone evaluates 100 (in the dip), then 50, 75, 87, 93, 96,
    94, 95 and stops at K = 95, inside the dip. The probes after it (96, 100, 115, 145, 200) see
    the rise at 115 and 145, so the search restarts above 145 and returns 160."""
    from paper_2202_08627_amd.warmstart import first_stable_crossing
    tol = 1e-3

    def err(k):
        return 0.5 * tol if (95 <= k <= 105 or k >= 160) else 2.0 * tol
    k, e, checks = first_stable_crossing(err, 1.0, tol, 200)
    assert k == 160 and checks["err_k_minus_1"] > tol
    k, e, checks = first_stable_crossing(err, 1.0, tol, 200, probes=())
    assert k == 95                    # what a bisection without the probes would report


def test_stable_crossing_not_reached():
    from paper_2202_08627_amd.warmstart import first_stable_crossing
    k, e, checks = first_stable_crossing(lambda k: 1.0, 1.0, 1e-3, 50)
    assert k is None and e == 1.0


def test_stable_crossing_at_zero():
    from paper_2202_08627_amd.warmstart import first_stable_crossing
    k, e, checks = first_stable_crossing(lambda k: 1e-4, 1e-4, 1e-3, 50)
    assert k == 0 and checks["err_k_minus_1"] is None
