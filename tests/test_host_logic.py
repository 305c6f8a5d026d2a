"""Host-side logic that needs no GPU: the local-BA request generator, the
Poisson arrival stream and the autotuner's database file."""
import collections

import numpy as np

from paper_2509_26581_amd import autotune, synth


def test_local_request_shapes_and_windows():
    for seed in range(12):
        r = synth.make_local_request(seed)
        K, npt = len(r["cams"]), len(r["pts"])
        assert 5 <= K <= 40 and 500 <= npt <= 20_000
        assert r["cam_fixed"][:2].all() and not r["cam_fixed"][2:].any()
        # fixed keyframes are not perturbed
        assert np.array_equal(r["cams"][:2], r["cams_true"][:2])
        tracks = collections.defaultdict(list)
        for c, p in zip(r["cam_idx"], r["pt_idx"]):
            tracks[int(p)].append(int(c))
        assert len(tracks) == npt                           # every point observed
        for cams in tracks.values():
            assert 2 <= len(cams) <= min(10, K)
            assert len(set(cams)) == len(cams)              # distinct keyframes
            assert max(cams) - min(cams) < len(cams) + 4    # inside a local window
        assert r["cam_idx"].min() >= 0 and r["cam_idx"].max() < K
        assert np.isfinite(r["uv"]).all()


def test_local_request_is_seeded():
    a, b = synth.make_local_request(3), synth.make_local_request(3)
    for k in ("cams", "pts", "cam_idx", "pt_idx", "uv"):
        assert np.array_equal(a[k], b[k])


def test_poisson_arrivals():
    t = synth.poisson_arrivals(20_000, 250.0, 1)
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 250.0) < 0.05 / 250.0
    assert abs(gaps.std() - 1 / 250.0) < 0.05 / 250.0      # exponential: std = mean


def test_tuning_database_file(tmp_path):
    path = str(tmp_path / "db.txt")
    autotune.write_db(path, "fp32", {"tiles_per_block": 8, "pcg_sync_every": 4}, 123.4, 96, 64)
    autotune.write_db(path, "fp64", {"tiles_per_block": 32}, 50.0, 96, 64)
    autotune.write_db(path, "fp32", {"tiles_per_block": 16}, 130.0, 96, 64)
    lines = open(path).read().splitlines()
    keys = [ln.split()[0] for ln in lines if not ln.startswith("#")]
    assert keys == ["fp64.tiles_per_block", "fp32.tiles_per_block"]
    assert "fp32.tiles_per_block 16" in lines and "fp64.tiles_per_block 32" in lines
