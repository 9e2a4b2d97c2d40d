"""The oracle against its stored outputs on a fixed five-Gaussian scene
(tests/golden/oracle_tiny.json, written by tests/golden/make_oracle_tiny.py
from the oracle alone).  A regression guard for the oracle's arithmetic: the
independent pins of the method are in test_oracle_*.py."""
import json
import os

import numpy as np

from tests.golden.make_oracle_tiny import compute

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_reproduces_its_fixture():
    ref = json.load(open(os.path.join(HERE, "oracle_tiny.json")))
    got = compute()
    assert got["index"] == ref["index"]
    for k in ("color", "depth", "trans", "d_pos", "d_scale", "d_rot", "d_opacity", "d_color"):
        np.testing.assert_allclose(np.asarray(got[k]), np.asarray(ref[k]), rtol=1e-12, atol=1e-12, err_msg=k)
    # the fixture exercises every output: hits and misses, partial coverage
    idx = np.asarray(ref["index"])
    assert (idx >= 0).sum() > 100 and (idx == -1).sum() > 100
    assert np.abs(np.asarray(ref["d_pos"])).max() > 0
