"""Host logic of the batch autotuner (CPU): the layouts it proposes are ones the
library accepts, and its knob search stays within what the library supports."""
import math

import pytest

import paper_2207_05152_amd as dl
from paper_2207_05152_amd import autotune


def _max_rows(h, g):
    return max((k + 1) * h // g - k * h // g for k in range(g))


@pytest.mark.parametrize("rows", [2, 12, 16, 24, 64, 96, 192, 256, 300, 1000])
@pytest.mark.parametrize("lanes", [1, 2, 4, 32, 64])
def test_coders_for_respects_format_limits(rows, lanes):
    sizes = [(1, 5), (2, 9), (3, 3), (17, 40), (256, 256), (384, 512), (768, 1024),
             (1536, 2048), (4097, 64), (60000, 8)]
    for (h, w), (g, l) in zip(sizes, autotune.coders_for(sizes, rows, lanes)):
        assert l == lanes
        assert 1 <= g <= 1024
        assert g == 1 or h >= 2 * g
        assert _max_rows(h, g) <= 256
        # as many groups as asked for unless a limit forces more or fewer
        want = max(1, math.ceil(h / rows))
        if want <= 1024 and (want == 1 or h >= 2 * want) and math.ceil(h / want) <= 256:
            assert g == want, (h, rows, g)
        # the library accepts the layout (host-only size query)
        assert dl.dlic_encode_bound(h, w, dl.dlic_coder(g, l)) > 0, (h, w, g, l)


def test_coders_for_refuses_impossible_heights():
    with pytest.raises(ValueError):
        autotune.coders_for([(1024 * 256 + 1, 4)], 256, 32)


def test_knob_search_space():
    assert set(autotune.DEFAULT) == {"rows_per_group", "lanes", "density_grid", "search_lanes",
                                     "decode_grid"}
    for rows, lanes in autotune.LAYOUTS:
        assert 1 <= lanes <= 64 and rows >= 2
        opts = autotune.search_options(lanes)
        assert 0 in opts
        # 16 lanes per pixel only for layouts of at most 4 lanes, the split search at most 32
        assert all(o in (0, 1, 2) for o in opts)
        if lanes > 32:
            assert opts == (0,)
    best = dict(autotune.DEFAULT, rows_per_group=12, lanes=4)
    trials = autotune.knob_trials(best)
    # one knob changed at a time, never the layout
    for t in trials:
        assert (t["rows_per_group"], t["lanes"]) == (12, 4)
        assert sum(t[k] != best[k] for k in best) == 1
    assert {t["search_lanes"] for t in trials} >= {2}
    assert {t["decode_grid"] for t in trials} >= set(autotune.DECODE_GRIDS) - {0}
