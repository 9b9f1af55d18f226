"""The seeded scene generator is deterministic and matches its recipe."""
import numpy as np

from synth import batch_workloads, make_scene, make_workload_pair, workload


def test_same_seed_same_pair():
    a = make_scene(96, 64, (8.0, 0.0, 0.1), 2, 1, 5)
    b = make_scene(96, 64, (8.0, 0.0, 0.1), 2, 1, 5)
    assert np.array_equal(a.ref, b.ref) and np.array_equal(a.tar, b.tar)
    c = make_scene(96, 64, (8.0, 0.0, 0.1), 2, 1, 6)
    assert not np.array_equal(a.ref, c.ref)


def test_texture_statistics_and_ground_truth_range():
    w = workload("c1")
    sc = make_workload_pair(w)
    assert sc.ref.dtype == np.uint8 and sc.ref.shape == (240, 320)
    assert 4.5 < sc.ref.astype(float).std() < 7.5
    assert abs(sc.ref.astype(float).mean() - 128) < 2
    v = np.arange(240)[:, None]
    road = 8.0 + 0.1 * v
    assert np.all(sc.d_gt <= road + 1e-12)
    assert np.all(sc.d_gt >= road - 4.0 - 1e-12)   # potholes 1..4 px deep
    assert np.array_equal(sc.d_gt[sc.road_mask], np.broadcast_to(road, sc.d_gt.shape)[sc.road_mask])


def test_float_pairs_are_not_quantised():
    sc = make_scene(64, 48, (24.0, 0, 0.1), 1, 0, 5, float_images=True)
    assert sc.ref.dtype == np.float32
    assert np.any(sc.ref != np.rint(sc.ref))


def test_planar_target_is_the_shifted_texture():
    """Without damage, tar(x) = T(x + d_road) exactly for integer shifts."""
    sc = make_scene(80, 10, (6.0, 0.0, 0.0), 0, 0, 9, float_images=True)
    assert np.allclose(sc.tar[:, :70], sc.ref[:, 6:76], atol=1e-4)


def test_batch_recipe():
    b = batch_workloads()
    assert len(b) == 64
    sizes = [(w.width, w.height) for w in b]
    assert sizes.count((320, 240)) == 16 and sizes.count((640, 480)) == 24
    assert sizes.count((1280, 720)) == 16 and sizes.count((1920, 1080)) == 8
    for w in b:
        assert 32 <= w.num_disp <= 96 and w.delta_p == w.num_disp // 2
        c0, c1, c2 = w.plane
        a1 = np.hypot(c1, c2)
        assert 0.05 - 1e-12 <= a1 <= 0.2 + 1e-12
        assert abs(np.arctan2(-c1, c2)) <= np.deg2rad(10) + 1e-12
        corners = [c0 + c1 * u + c2 * v for u in (0, w.width - 1) for v in (0, w.height - 1)]
        assert abs(min(corners) - 4.0) < 1e-9
