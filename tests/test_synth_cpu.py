"""The seeded input generators against their stated recipes: the camera
paths of the animation workload (an orbit at constant distance with evenly
spaced azimuths, a far-to-near sweep), the random poses, the clustered set
and the blobs."""
import math

import numpy as np

from paper_1606_04427_amd import synth

C = np.array([0.5, 0.5, 0.5])


def _check_pose(p):
    eye, look, up = map(np.asarray, (p.eye, p.lookat, p.up))
    fwd = look - eye
    assert np.allclose(look, C)
    assert abs(np.linalg.norm(up) - 1.0) < 1e-12
    assert abs(np.dot(up, fwd)) < 1e-9 * np.linalg.norm(fwd)


def test_orbit_is_a_circle_around_the_centre():
    poses = synth.orbit_poses(100, radius=1.6, elevation_deg=20.0)
    assert len(poses) == 100
    eyes = np.array([p.eye for p in poses]) - C
    assert np.allclose(np.linalg.norm(eyes, axis=1), 1.6)
    assert np.allclose(eyes[:, 2], 1.6 * math.sin(math.radians(20.0)))
    az = np.unwrap(np.arctan2(eyes[:, 1], eyes[:, 0]))
    assert np.allclose(np.diff(az), 2 * math.pi / 100)
    for p in poses:
        _check_pose(p)
        assert (p.width, p.height) == (1024, 1024)


def test_sweep_goes_from_far_to_near():
    poses = synth.sweep_poses(6, far=3.0, near=0.6)
    d = np.array([np.linalg.norm(np.asarray(p.eye) - C) for p in poses])
    assert abs(d[0] - 3.0) < 1e-12 and abs(d[-1] - 0.6) < 1e-12
    assert np.all(np.diff(d) < 0)
    assert np.allclose(np.diff(np.log(d)), np.log(0.6 / 3.0) / 5)
    dirs = (np.array([p.eye for p in poses]) - C) / d[:, None]
    assert np.allclose(dirs, dirs[0])
    for p in poses:
        _check_pose(p)


def test_camera_straight_above_the_centre_gets_a_valid_up():
    p = synth.sweep_poses(2, direction=(0.0, 0.0, 1.0))[0]
    _check_pose(p)


def test_clustered_set_follows_its_recipe():
    """The stand-in for the paper's snapshot: seeded and repeatable, about one
    star per ten particles, positive smoothing lengths and scalars, the
    clustered part within the nested cluster radii, the uniform field last,
    absorption in [0.01, 0.5]."""
    a = synth.soneira_peebles(200_000, seed=5, absorption=True)
    b = synth.soneira_peebles(200_000, seed=5, absorption=True)
    assert a.n == 200_000
    for f in ("x", "y", "z", "h", "intensity", "scalar", "species", "absorption"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    frac = float(np.mean(a.species == 1))
    assert abs(frac - 0.10) < 0.01
    assert np.all(a.h > 0) and np.all(a.scalar > 0) and np.all(a.intensity > 0)
    assert np.all((a.absorption >= 0.01) & (a.absorption <= 0.5))
    # 95% of the particles sit about the leaves: within the sum of the nested
    # cluster radii (0.5 (1 + 1/3 + 1/9 + 1/27)) plus five leaf widths of the
    # cube centre; the uniform field, stored last, fills the cube
    r = np.sqrt((a.x - 0.5) ** 2 + (a.y - 0.5) ** 2 + (a.z - 0.5) ** 2)
    bound = 0.5 * (1 + 1 / 3 + 1 / 9 + 1 / 27) + 5 * 0.5 / 81 / 2
    assert np.mean(r[: int(0.95 * a.n) - 100] <= bound) > 0.999
    field = a.x[-int(0.05 * a.n) + 100:]
    assert field.min() < 0.01 and field.max() > 0.99
    c = synth.soneira_peebles(200_000, seed=6)
    assert not np.array_equal(a.x, c.x)


def test_blobs_follow_their_recipe():
    a = synth.blobs(50_000, seed=3)
    b = synth.blobs(50_000, seed=3)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.h, b.h)
    for v in (a.x, a.y, a.z):
        assert v.min() >= 0.0 and v.max() <= 1.0
    # smoothing length in pixels at the blob camera's depth: [0.5, 8], median 2
    world_per_px = 2.0 * math.tan(math.radians(20.0)) / 128.0
    px = a.h.astype(np.float64) / world_per_px
    assert px.min() >= 0.5 - 1e-4 and px.max() <= 8.0 + 1e-4
    assert abs(np.median(px) - 2.0) < 0.05
    assert np.all(a.species == 0) and np.array_equal(a.intensity, a.scalar)


def test_random_poses_follow_their_recipe():
    poses = synth.random_poses(200, seed=9, dist_range=(0.6, 3.0))
    d = np.array([np.linalg.norm(np.asarray(p.eye) - C) for p in poses])
    assert d.min() >= 0.6 - 1e-9 and d.max() <= 3.0 + 1e-9
    look = np.array([p.lookat for p in poses])
    assert np.all(np.abs(look - C) < 0.3)
    for p in poses:
        fwd = np.asarray(p.lookat) - np.asarray(p.eye)
        assert abs(np.dot(np.asarray(p.up), fwd)) < 1e-9 * np.linalg.norm(fwd)
    assert [p.eye for p in poses] == [p.eye for p in synth.random_poses(200, seed=9)]
