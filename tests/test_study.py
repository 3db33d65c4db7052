"""CPU checks of the leaf-size study's host logic (no GPU)."""
import numpy as np
import pytest

from paper_0810_0233_amd import study


def test_paper_rule_reproduces_worked_examples():
    """Sec. 4's three worked trees: (50^3, p=3) -> L=14; (40x40x10, p=4) -> L=10;
    (32^3, p=5) -> L=11, with s_o(p) = 0.74 p^2 for p > 3 and 8 below."""
    assert study.paper_s(3) == 8.0
    assert study.paper_s(4) == pytest.approx(11.84)
    assert study.paper_levels(50 ** 3, study.paper_s(3)) == 14
    assert study.paper_levels(40 * 40 * 10, study.paper_s(4)) == 10
    assert study.paper_levels(32 ** 3, study.paper_s(5)) == 11


def test_levels_rule_tie_takes_smaller_level():
    # N / 2^L = 12 and 6 straddle s = 9 equally: the smaller L wins
    assert study.paper_levels(24, 9.0) == 1


def test_optimum_of_a_parabola_in_log_s():
    xs = [4.0, 8.0, 16.0, 32.0, 64.0]
    pts = [{"s": s, "t": (np.log2(s) - np.log2(20.0)) ** 2 + 1.0} for s in xs]
    assert study.optimum_s(pts, "t") == pytest.approx(20.0, rel=1e-9)
    # the fastest point at the end of the sweep is returned as it is
    assert study.optimum_s(pts[:2], "t") == 8.0


def test_fit_of_c_in_s_equals_c_p_squared():
    recs = [{"order": p, "s_opt": 1.3 * p * p} for p in (2, 3, 4, 5, 6)]
    recs[0]["s_opt"] = 99.0  # orders up to 3 are not fitted (Eq. (so) sets 8 there)
    recs[1]["s_opt"] = 99.0
    assert study.fit_c(recs) == pytest.approx(1.3)


def test_error_estimate_reproduces_table_ii():
    """Sec. 3 estimate e = [theta/(2-theta)]^p at Table II's (p, alpha) pairs:
    about 0.05 for every pair (printed there as 0.048 ... 0.053)."""
    pairs = {(2, 0.36): 0.048, (3, 0.54): 0.051, (4, 0.64): 0.049, (5, 0.71): 0.050, (6, 0.76): 0.053,
             (7, 0.79): 0.051, (8, 0.81): 0.046}
    for (p, a), e in pairs.items():
        assert abs(study.paper_error_estimate(p, a) - e) <= 0.0006, (p, a)


def test_alpha_for_error_inverts_the_estimate():
    """alpha(p, e) solves [alpha/(2-alpha)]^p = e; Table II's pairs come back
    at e = 0.05 to the two printed digits of alpha."""
    for p in range(1, 9):
        for e in (0.1, 0.05, 0.001):
            a = study.alpha_for_error(p, e)
            assert 0 < a < 1 and abs(study.paper_error_estimate(p, a) - e) <= 1e-12 * e
    table = {2: 0.36, 3: 0.54, 4: 0.64, 5: 0.71, 6: 0.76, 7: 0.79, 8: 0.81}
    for p, a in table.items():
        assert abs(study.alpha_for_error(p, 0.05) - a) <= 0.01, p
