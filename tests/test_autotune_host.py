"""Tile lookup on the host (no GPU): the autotuner's cache is keyed by grid size, angle count
and detector width only, so a cached variant can be too narrow for another angle list of the
same size (angles over 360 degrees, irregular angles). The lookup must then return tiles the
library accepts for that geometry."""
import os

import numpy as np
import pytest

from paper_2202_08627_amd import _lib as L
from paper_2202_08627_amd import autotune, ops, synth

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")

SIZES = [(256, 360), (512, 720), (768, 1080), (1024, 1800)]


def _geo(n, nt, theta):
    return ops.Geometry(n, nt, n, 8, 10.0, theta, synth.mask_positions(8), np.ones(n),
                        np.zeros(n), np.full(n, 0.6))


def _angle_lists(n, nt):
    return {"180": synth.angles(nt),
            "360": np.arange(nt) * (2.0 * np.pi / nt),
            "irregular": np.sort(np.random.default_rng(n).uniform(0.0, np.pi, nt))}


@pytest.mark.parametrize("n,nt", SIZES)
def test_tiles_fit_every_angle_list(n, nt):
    cache = autotune.load_cache()
    for kind, th in _angle_lists(n, nt).items():
        geo = _geo(n, nt, th)
        t = autotune.tiling_for(geo)
        ops.inspect(geo, *t)                 # raises EitError if the library rejects the tiles
        if kind == "180" and autotune.size_key(geo) in cache:
            ent = cache[autotune.size_key(geo)]
            assert t == (ent["proj_variant"], ent["adj_variant"], ent["adj_splits"])


def test_360_degree_lookup_needed_the_fallback():
    """The case the fallback exists for: at 512^2 the tuned projector variant is rejected for
    angles over 360 degrees, and the lookup picks another interleaved variant, not the default."""
    geo = _geo(512, 720, np.arange(720) * (2.0 * np.pi / 720))
    ent = autotune.load_cache()[autotune.size_key(geo)]
    with pytest.raises(L.EitError) as e:
        ops.inspect(geo, ent["proj_variant"], ent["adj_variant"], ent["adj_splits"])
    assert e.value.code == L.EIT_ERR_SHAPE
    pv, av, ag = autotune.tiling_for(geo)
    assert pv != ent["proj_variant"] and pv >= 0
    assert (av, ag) == (ent["adj_variant"], ent["adj_splits"])
