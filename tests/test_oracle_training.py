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


# ---------------------------------------------------------------- density control
def test_quat_rotation_special_cases():
    np.testing.assert_allclose(training.quat_rotation([2.0, 0, 0, 0]), np.eye(3), atol=1e-15)
    c = np.cos(np.pi / 4)
    Rz = training.quat_rotation([c, 0, 0, c])  # 90 degrees about z: x -> y, y -> -x
    np.testing.assert_allclose(Rz @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(Rz @ [0, 1, 0], [-1, 0, 0], atol=1e-15)
    R = training.quat_rotation(np.random.default_rng(0).standard_normal(4))
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(R) - 1) < 1e-14


def test_split_child_worked_examples():
    m, s = training.split_child([1.0, 2.0, 3.0], [0.2, 0.1, 0.05], [1, 0, 0, 0], [1.0, 0.0, 0.0], 2)
    np.testing.assert_allclose(m, [1.2, 2.0, 3.0], atol=1e-15)
    np.testing.assert_allclose(s, [0.125, 0.0625, 0.03125], atol=1e-15)
    c = np.cos(np.pi / 4)
    m, _ = training.split_child([0.0, 0.0, 0.0], [0.2, 0.1, 0.05], [c, 0, 0, c], [1.0, 0.0, -2.0], 2)
    np.testing.assert_allclose(m, [0.0, 0.2, -0.1], atol=1e-15)


def test_split_children_sample_the_parent():
    """With z ~ N(0, I) the children's positions have the parent's covariance
    R diag(s^2) R^T."""
    rng = np.random.default_rng(3)
    q = rng.standard_normal(4)
    s = np.array([0.3, 0.1, 0.02])
    R = training.quat_rotation(q)
    pts = np.array([training.split_child([0, 0, 0], s, q, z, 2)[0] for z in rng.standard_normal((40000, 3))])
    cov = np.cov(pts.T)
    want = R @ np.diag(s ** 2) @ R.T
    assert np.abs(cov - want).max() < 0.03 * s[0] ** 2


def test_densify_plan_worked_example():
    # Gaussians: seen twice with mean 3e-4 (clone: small), seen once at 2e-4
    # exactly (reaches the threshold; split: large), below the threshold,
    # never seen, frozen layer
    grad_sum = np.array([6e-4, 2e-4, 1e-4, 0.0, 9.0])
    count = np.array([2.0, 1.0, 1.0, 0.0, 1.0])
    scale = np.array([[0.005, 0.5, 0.005, 0.005, 0.005]] * 3)
    layer = np.array([1, 1, 1, 1, 0], np.uint8)
    plan = training.densify_plan(grad_sum, count, scale, layer, 0b10, 2e-4, 0.01, 1.0, 1)
    assert plan == ["clone", "split", None, None, None]
    # with 4 views per step every mean counts 4 times: the third now clones
    plan = training.densify_plan(grad_sum, count, scale, layer, 0b10, 2e-4, 0.01, 1.0, 4)
    assert plan == ["clone", "split", "clone", None, None]
