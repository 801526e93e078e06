"""Host logic of the warm-start pipeline (no GPU): the fallback combination,
the settled test and the capped median.  (Standardisation and folding run
in the library: tests/test_gpu_mlp.py.)"""
import numpy as np

from paper_2406_13191_amd import warmstart as W


def test_fallback_rule():
    # columns: cold hit, cold bound at the probe, warm hit, warm bound at the probe
    hc = np.array([500, 40, 500, -1, 300, 90])
    pc = np.array([10., 10., 10., 10., 10., 10.])
    hw = np.array([200, 500, 60, 150, -1, 80])
    pw = np.array([11., 12., 9., 12., 9., 9.])
    got, used = W.combine_with_fallback(hc, pc, hw, pw, 100)
    # 0: warm better at probe -> warm's 200; 1: cold certified at 40 (< probe)
    # 2: warm certified at 60 before the probe; 3: warm kept -> 150
    # 4: cold kept -> 300; 5: both certified before the probe -> 80
    np.testing.assert_array_equal(got, [200, 40, 60, 150, 300, 80])
    np.testing.assert_array_equal(used, [True, True, False, True, False, False])


def test_median_counts_unreached_at_cap():
    assert W.median_iters(np.array([10, -1, -1]), 5000) == 5000
    assert W.median_iters(np.array([10, 20, -1]), 5000) == 20


def test_settled_drops_rising_and_oversized_bounds():
    from paper_2406_13191_amd import warmstart as W
    bound = np.array([100.0, 100.0, 100.0, 5000.0, np.nan, 100.0])
    earlier = np.array([99.99, 90.0, 100.0, 4999.0, 100.0, np.inf])
    ok = W.settled(bound, earlier, cost_ub=1000.0, rel=1e-3)
    # settled; rose 10 %; flat; above the largest cost; NaN; infinite history
    assert ok.tolist() == [True, False, True, False, False, False]
