"""Host-side logic that needs no GPU: the benchmark's command-line contract
and profile parsing, the autotuner's workload key, and the determinism of
the synthetic workloads."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_parsing(tmp_path, monkeypatch):
    import bench
    src = open(os.path.join(ROOT, "paper_2404_19706_amd", "csrc", "raster.hip"), "rb").read()
    digest = hashlib.sha256(src).hexdigest()[:16]
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_k_raster_bwd_c9_16x16.txt").write_text("# comment: x\nhbm_bytes_per_launch: 1234\nsource_sha256_16: %s\n"
                                                      % digest)
    (prof / "traffic_k_raster_fwd_c9_16x16.txt").write_text("hbm_bytes_per_launch: 99\nsource_sha256_16: 0000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "paper_2404_19706_amd" / "csrc")
    (tmp_path / "paper_2404_19706_amd" / "csrc" / "raster.hip").write_bytes(src)
    assert bench.traffic_from_profile("k_raster_bwd", "c9", (16, 16)) == 1234.0
    assert bench.traffic_from_profile("k_raster_fwd", "c9", (16, 16)) is None   # stale: kernel changed since
    assert bench.traffic_from_profile("k_raster_bwd", "c8", (16, 16)) is None   # no summary
    assert bench.traffic_from_profile("k_raster_bwd", "c9", (32, 8)) is None    # other tile shape


def test_autotune_key_buckets():
    from paper_2404_19706_amd.autotune import _key
    cam = {"width": 640, "height": 480}
    m = torch.zeros((2, 480, 640), dtype=torch.uint8)
    m[:, :240] = 1
    k1 = _key(cam, 100_000, 2, m)
    k2 = _key(cam, 110_000, 2, m)           # same size bucket
    k3 = _key(cam, 1_000_000, 2, m)
    assert k1 == k2 and k1 != k3 and "m10" in k1


def test_workloads_are_seeded_and_shaped():
    from rtg_synth import make_config
    a, b = make_config("c1"), make_config("c1")
    for k in ("pos", "scale", "rot", "opacity", "color", "unstable"):
        assert np.array_equal(a["scene"][k], b["scene"][k])
    sc = a["scene"]
    assert sc["pos"].shape == (2000, 3) and sc["pos"].dtype == np.float32
    op = sc["opacity"]
    assert ((op >= 0.95) & (op <= 0.99)).mean() > 0.6 and ((op >= 0.02) & (op <= 0.1)).mean() > 0.2
    c2 = make_config("c2")
    s = c2["scene"]["scale"]
    # surface Gaussians: two equal in-plane scales in 1-5 cm, thin axis a tenth
    assert np.allclose(s[:, 0], s[:, 1]) and np.allclose(s[:, 2], 0.1 * s[:, 0], rtol=1e-5)
    assert s[:, 0].min() >= 0.0099 and s[:, 0].max() <= 0.0501
    assert c2["cam"]["width"] == 640 and c2["poses"].shape == (1, 12)
