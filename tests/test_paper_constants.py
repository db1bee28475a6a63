"""The oracle's defaults carry the constants the paper prints (tests/golden)."""

import json
import os

from oracle import lddmm as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_defaults_match_paper_constants():
    g = json.load(open(GOLDEN))
    prm = O.Params()
    assert prm.gamma == g["gamma"]["value"]
    assert prm.sigma == g["sigma"]["value"]
    assert tuple(prm.weight) == tuple(g["mask_channel_weights"]["value"])
