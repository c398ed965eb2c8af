"""Pins of the oracle's training-side statistics (oracle/training.py)."""
import numpy as np

from oracle import training


def _params(n, D, rng):
    nc = (D + 1) ** 2
    return {"mean": rng.standard_normal((3, n)), "log_scale": rng.standard_normal((3, n)),
            "sh": rng.standard_normal((nc, 3, n))}


def test_update_activity_worked_example():
    """Changes with Pythagorean lengths: d mean = (0.3, 0.4, 0) has length
    0.5, d log scale = (0, 0.6, 0.8) length 1, d SH (degree 0) = (2, 3, 6)
    length 7: activity 2 * 0.5 + 0.1 * 7 + 0.1 * 1 = 1.8."""
    b = {"mean": np.zeros((3, 1)), "log_scale": np.full((3, 1), -4.0), "sh": np.full((1, 3, 1), 0.25)}
    a = {"mean": np.array([[0.3], [0.4], [0.0]]), "log_scale": np.array([[-4.0], [-3.4], [-3.2]]),
         "sh": np.array([[[2.25], [3.25], [6.25]]])}
    out = training.update_activity(b, a, np.zeros(1, np.uint8), 1, np.array([0.5]))
    assert abs(out[0] - (0.5 + 1.8)) < 1e-12


def test_update_activity_only_moved_trainable_gaussians():
    rng = np.random.default_rng(0)
    n, D = 40, 2
    b = _params(n, D, rng)
    a = {k: v.copy() for k, v in b.items()}
    layer = rng.integers(0, 3, n).astype(np.uint8)
    moved = rng.random(n) < 0.5
    for k in a:
        a[k][..., moved] += 0.01
    act0 = rng.random(n)
    out = training.update_activity(b, a, layer, 0b101, act0)
    live = (layer == 0) | (layer == 2)
    # frozen layers and unmoved Gaussians keep their activity exactly
    np.testing.assert_array_equal(out[~(live & moved)], act0[~(live & moved)])
    # a uniform shift c of all k values of a parameter has norm c sqrt(k)
    nc = (D + 1) ** 2
    want = 0.01 * (2 * np.sqrt(3) + 0.1 * np.sqrt(3 * nc) + 0.1 * np.sqrt(3))
    np.testing.assert_allclose(out[live & moved] - act0[live & moved], want, rtol=1e-6)


def test_update_activity_is_sign_and_order_free():
    """The norm of the change does not depend on its direction, so swapping
    before and after, or permuting the Gaussians, changes nothing."""
    rng = np.random.default_rng(1)
    n = 25
    b, a = _params(n, 3, rng), _params(n, 3, rng)
    layer = np.zeros(n, np.uint8)
    x = training.update_activity(b, a, layer, 1, np.zeros(n))
    y = training.update_activity(a, b, layer, 1, np.zeros(n))
    np.testing.assert_allclose(x, y, rtol=1e-14)
    perm = rng.permutation(n)
    z = training.update_activity({k: v[..., perm] for k, v in b.items()}, {k: v[..., perm] for k, v in a.items()},
                                 layer, 1, np.zeros(n))
    np.testing.assert_allclose(z, x[perm], rtol=1e-14)
