"""Writes oracle_tiny.json: the FP64 oracle's outputs on a fixed five-Gaussian
scene (two poses, a 24x18 image), as a regression fixture for the oracle
itself.  It calls only oracle/ and the seeded scene below; the values are the
oracle's, not the paper's (the paper prints no worked example for the
rasterizer), so the fixture guards against unintended changes of the
oracle's arithmetic and is regenerated only with a change the paper
justifies.

    python tests/golden/make_oracle_tiny.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402
from rtg_synth import camera, look_at  # noqa: E402


def scene():
    pos = [[0.0, 0.0, 2.0], [0.05, -0.03, 2.2], [-0.06, 0.04, 1.9], [0.02, 0.05, 2.5], [-0.02, -0.05, 2.1]]
    scale = [[0.05, 0.04, 0.005], [0.03, 0.03, 0.003], [0.04, 0.02, 0.004], [0.08, 0.06, 0.008],
             [0.02, 0.05, 0.002]]
    rot = [[1.0, 0.0, 0.0, 0.0], [0.9, 0.1, -0.2, 0.3], [0.7, -0.3, 0.5, 0.1], [0.95, 0.05, 0.05, -0.2],
           [0.6, 0.4, 0.4, 0.5]]
    opacity = [0.97, 0.6, 0.95, 0.99, 0.05]
    color = [[0.9, 0.1, 0.1], [0.1, 0.8, 0.2], [0.2, 0.3, 0.9], [0.5, 0.5, 0.5], [0.7, 0.7, 0.1]]
    unstable = [1, 1, 0, 1, 1]
    f = lambda a: np.asarray(a, np.float32)  # noqa: E731
    return {"pos": f(pos), "scale": f(scale), "rot": f(rot), "opacity": f(opacity), "color": f(color),
            "unstable": np.asarray(unstable, np.uint8)}


def poses():
    p0 = np.concatenate([np.eye(3).reshape(-1), np.zeros(3)])
    p1 = look_at(np.array([0.1, -0.05, 0.0]), np.array([0.0, 0.0, 2.1]), up=np.array([0.0, -1.0, 0.0]))
    return np.stack([p0, p1])


def compute():
    cam = camera(24, 18, 200.0, 200.0)
    sc, ps = scene(), poses()
    P = orc.make_params(cam, tile=(8, 8))
    recs = orc.project(P, sc, ps)
    mask = np.ones((2, 18, 24), np.uint8)
    pix = orc.masked_pixels(mask)
    out = orc.render(P, recs, sc, pix)
    rng = np.random.default_rng(5)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    grads = orc.backward(P, recs, sc, ps, pix, gC, gD)
    return {"color": out["color"].tolist(), "depth": out["depth"].tolist(), "trans": out["trans"].tolist(),
            "index": out["index"].tolist(), **{"d_" + k: np.asarray(v).tolist() for k, v in grads.items()}}


if __name__ == "__main__":
    orc.build(force=False) if not os.path.exists(orc._LIB_PATH) else None
    with open(os.path.join(HERE, "oracle_tiny.json"), "w") as fh:
        json.dump({"about": "FP64 oracle outputs on the five-Gaussian scene of make_oracle_tiny.py "
                            "(regression fixture of the oracle, not paper values)", **compute()}, fh)
    print("wrote oracle_tiny.json")
