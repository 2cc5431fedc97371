"""Golden fixtures: the paper's printed organisation constants, and the oracle's stored summary."""
import json
import os

import numpy as np
import pytest

from oracle import oracle
from paper_2605_17855_amd import scenes

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_paper_constants_tile_and_masks():
    c = _load("paper_constants.json")
    assert oracle.TILE == c["tile_size_px"]["value"]
    sc, cam = scenes.small_camera_space(n=512)
    rec = oracle.preprocess(sc, cam)
    for g, bits in c["mask_bits"]["value"].items():
        _, _, masks = oracle.lists(rec, cam, int(g))
        assert int(masks.max()) < (1 << bits)
        assert int(masks.max()) >= (1 << (bits - 1))   # the top member tile is used
    e = c["entry_bytes_fp16"]["value"]
    base = e["centre"] + e["conic_opacity"] + e["id"]
    assert e["mask"] / base == pytest.approx(c["mask_overhead_fraction"]["value"])
    k0, k1 = c["inner_dim_padding"]["value"]
    assert k1 == c["tensor_shape_mnk"]["value"][2] and k0 == 3


def test_oracle_matches_stored_summary():
    want = _load("oracle_small.json")
    sc, cam = scenes.small_camera_space()
    out = oracle.render(sc, cam)
    rec = out["records"]
    assert int(rec["visible"].sum()) == want["visible"]
    assert int(out["start"][-1]) == want["tile_entries"]
    assert int(out["e_pix"]) == want["e_pix"]
    assert np.allclose([out["image"][c].sum() for c in range(3)], want["image_channel_sums"], rtol=1e-12)
    assert float(out["tfinal"].sum()) == pytest.approx(want["tfinal_sum"], rel=1e-12)
    for g, v in want["load_reduction"].items():
        n_total, n_group, _ = oracle.load_reduction(rec, cam, int(g))
        assert (n_total, n_group) == (v["n_total"], v["n_group"])
