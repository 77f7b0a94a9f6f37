"""The seeded census draw (host only): reproducible, the documented
families and ranges, one placement seed per packing, and the span rule
(the largest sphere at phi = 0.8 spans at most span_max of the box edge)."""
import numpy as np
import pytest

import rcp_inputs as ri


@pytest.fixture(scope="module")
def draw():
    return ri.census_draw(64)


def test_census_draw_is_reproducible(draw):
    again = ri.census_draw(64)
    assert [w.name for w in again] == [w.name for w in draw]
    for a, b in zip(again, draw):
        assert np.array_equal(a.d0, b.d0) and a.L == b.L and a.seed == b.seed


def test_census_draw_families_and_ranges(draw):
    fams = ("lognormal", "powerlaw", "weibull")
    for k, w in enumerate(draw):
        assert w.family == fams[k % 3]
        S = w.params["S"]
        assert 2.0 <= S <= 100.0
        assert 1_000 <= w.n <= 200_000
        if w.family == "lognormal":
            assert 0.2 <= w.params["alpha"] <= 1.5
        elif w.family == "powerlaw":
            assert -4.0 <= w.params["p"] <= -2.0
        else:
            assert 0.5 <= w.params["k"] <= 3.0
        # equal-probability quantiles of the distribution truncated to [1, S]:
        # the realised ratio lies inside the truncation range
        assert 1.0 < w.S_realised <= S * (1.0 + 1e-12)
        assert w.phi0 == 0.05
        assert w.L == ri.box_for_phi(w.d0, 0.05)


def test_census_draw_span_rule_and_seeds(draw):
    for w in draw:
        assert (0.8 / w.phi0) ** (1.0 / 3.0) * w.d0.max() <= 0.4 * w.L
    seeds = [w.seed for w in draw]
    assert len(set(seeds)) == len(seeds)
