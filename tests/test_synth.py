"""Input generators: exact sizes, reproducibility, shape of the workloads."""

import numpy as np

import synth


def test_blobs_exact_and_reproducible():
    a = synth.blobs_cloud(seed=1)
    b = synth.blobs_cloud(seed=1)
    assert a.shape == (20000, 3) and a.dtype == np.float32
    assert a.tobytes() == b.tobytes()
    assert synth.blobs_cloud(seed=2).tobytes() != a.tobytes()
    x, truth = synth.blobs_cloud(seed=1, return_truth=True)
    assert np.array_equal(x, a)
    sizes = np.bincount(truth[truth >= 0])
    assert sizes.shape[0] == 40 and sizes.min() >= 300 and sizes.max() <= 700
    noise = x[truth < 0]
    assert (noise[:, 2] == 0).all() and noise.min() >= 0 and noise.max() <= 50


def test_lidar_frame_exact_and_plausible():
    a = synth.lidar_frame(seed=2)
    assert a.shape == (120000, 3) and a.dtype == np.float32
    assert a.tobytes() == synth.lidar_frame(seed=2).tobytes()
    r = np.hypot(a[:, 0], a[:, 1])
    assert r.max() < 81 and r.min() > 0.3
    ground = np.abs(a[:, 2]) < 0.1
    assert 0.5 < ground.mean() < 0.98          # mostly ground, some objects
    assert a[:, 2].max() < 8.5


def test_map_prefix_and_frames():
    two = synth.lidar_map(frames=[0, 1], cache=False)
    assert two.shape == (270000, 3)
    one = synth.lidar_map(frames=[1], cache=False)
    assert np.array_equal(two[135000:], one)
    cached = synth.lidar_map(frames=[0, 1])
    again = synth.lidar_map(frames=[0, 1])
    assert np.array_equal(cached, two) and np.array_equal(again, two)


def test_trajectory_length():
    xy, head, _ = synth.map_trajectory()
    steps = np.hypot(*np.diff(xy, axis=0).T)
    assert xy.shape == (200, 2) and np.allclose(steps, 10.0)


def test_near_threshold_pairs_straddle():
    x = synth.near_threshold_cloud(200, 0.5, seed=3, spread=3.0)
    p = x.astype(np.float64)
    dist = np.linalg.norm(p[0::2] - p[1::2], axis=1)
    assert np.all(np.abs(dist - 0.5) < 1e-6)
    assert (dist < 0.5).any() and (dist >= 0.5).any()
