"""The seeded input generator: determinism, exact max |g|, smoothness, ground truth."""
import numpy as np

from paper_0909_0928_amd import phantom as P


def test_phantom_is_deterministic_and_shaped():
    a = P.make_phantom((24, 20, 12), seed=7, max_u=2.5)
    b = P.make_phantom((24, 20, 12), seed=7, max_u=2.5)
    assert a.static.shape == (12, 20, 24) and a.field_g.shape == (3, 12, 20, 24)
    assert np.array_equal(a.static, b.static) and np.array_equal(a.moving, b.moving)
    c = P.make_phantom((24, 20, 12), seed=8, max_u=2.5)
    assert not np.array_equal(a.moving, c.moving)


def test_field_max_and_lipschitz():
    p = P.make_phantom((32, 28, 16), seed=3, max_u=3.0)
    mag = np.sqrt((p.field_g ** 2).sum(axis=0))
    assert abs(mag.max() - 3.0) < 1e-12
    assert p.lipschitz < P.LIPSCHITZ_LIMIT


def test_intensities_are_ct_like():
    p = P.make_phantom((48, 48, 24), seed=1, max_u=3.0)
    c = tuple(s // 2 for s in p.static.shape)
    assert abs(p.static[0, 0, 0] - P.BACKGROUND_HU) < 1.0   # corner is air
    assert p.lung.sum() > 0 and p.body.sum() > p.lung.sum()
    lung_vals = p.static[p.lung]
    assert np.median(lung_vals) < -500.0


def test_ground_truth_inverts_the_generating_field():
    p = P.make_phantom((32, 32, 16), seed=5, max_u=3.0)
    v, res = p.ground_truth()
    assert res < 1e-10
    # M(x - v*(x)) = S(x) analytically: S(y + g(y)) at y = x - v*
    nz, ny, nx = p.static.shape
    gz, gy, gx = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float), np.arange(nx, dtype=float),
                             indexing="ij")
    y = (gx - v[0], gy - v[1], gz - v[2])
    g = p.g_at(*y)
    back = p.static_at(y[0] + g[0], y[1] + g[1], y[2] + g[2])
    np.testing.assert_allclose(back, p.static, atol=1e-8)
