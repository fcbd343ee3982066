"""The seeded scene generator: determinism and the stated recipe."""
import numpy as np

from synth import scenes


def test_seed_fixes_bytes():
    a = scenes.frame_640x480(seed=1)
    b = scenes.frame_640x480(seed=1)
    c = scenes.frame_640x480(seed=2)
    assert np.array_equal(a.depth.view(np.uint32), b.depth.view(np.uint32))
    assert not np.array_equal(a.depth, c.depth)


def test_recipe_ranges():
    s = scenes.frame_640x480(seed=1)
    assert s.depth.dtype == np.float32 and s.depth.shape == (480, 640)
    assert (s.fx, s.fy, s.cx, s.cy) == (525.0, 525.0, 319.5, 239.5)
    clean = s.depth_clean
    assert clean.min() >= 0.5 and clean.max() <= 4.0
    holes = s.depth == 0
    assert 0.015 < holes.mean() < 0.025
    # noise sigma = 0.001 z^2: standardised residual on non-hole pixels
    z = (s.depth[~holes] - clean[~holes]) / (0.001 * clean[~holes] ** 2)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
    # objects in front of the wall by >= 0.3 m
    obj = s.labels > 0
    assert obj.any() and clean[obj].max() <= 3.7


def test_analytic_normals():
    s = scenes.frame_1920x1080(seed=2)
    n = s.normals
    assert np.abs(np.linalg.norm(n, axis=-1) - 1).max() < 1e-12
    r = scenes.pixel_rays(1080, 1920, s.fx, s.fy, s.cx, s.cy)
    assert np.einsum("...k,...k", n, r).max() < 0
    assert len(np.unique(s.labels)) >= 8


def test_batch_mix():
    shapes = scenes.batch_shapes()
    assert len(shapes) == 256
    assert sum(h * w for h, w in shapes) == 159_744_000
    fr = scenes.batch_frames(indices=[0, 64, 160, 255])
    assert [f.depth.shape for f in fr] == [(240, 320), (480, 640), (720, 1280), (1080, 1920)]
    assert [f.seed for f in fr] == [1000, 1064, 1160, 1255]
    assert fr[3].fx == 525.0 * 3
