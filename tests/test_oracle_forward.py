"""Pins of the CPU oracle's forward pass against closed forms, library
routines, brute force and invariants (no GPU)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2410_16978_amd import scenes
from tests.helpers import axis_camera, make_scene, small_layered_scene, to64

KAPPA = 0.3
QMAX = 11.09375


def rec_fields(r, i):
    u, v, ca, cb, cc, op, depth, cr, cg, cbl = r["rec"][i]
    return dict(u=u, v=v, conic=np.array([[ca, cb], [cb, cc]]), op=op, depth=depth, rgb=np.array([cr, cg, cbl]))


# ---------------------------------------------------------------- projection
@pytest.mark.parametrize("sigma,z0,f", [(0.02, 3.0, 110.0), (0.05, 2.0, 300.0), (0.004, 5.0, 1662.77)])
def test_isotropic_footprint_closed_form(orc, sigma, z0, f):
    """Isotropic Gaussian on the optical axis: Sigma' = ((f sigma / z0)^2 + kappa) I
    for any rotation, centre at the principal point."""
    q = Rotation.random(random_state=1).as_quat()  # x, y, z, w
    sc = make_scene([[0, 0, z0]], [[sigma] * 3], quats=[[q[3], q[0], q[1], q[2]]], opacity=0.7)
    cam = axis_camera(f=f)
    r = orc.render(to64(sc), [cam], [scenes.view_state()], dtype=np.float64)
    sigma, f, z0 = (float(np.float32(x)) for x in (sigma, f, z0))  # inputs are float32
    s2 = (f * sigma / z0) ** 2 + KAPPA
    got = rec_fields(r, 0)
    np.testing.assert_allclose(got["conic"], np.eye(2) / s2, rtol=1e-12, atol=1e-15)
    assert got["u"] == pytest.approx(cam["cx"], abs=1e-12) and got["v"] == pytest.approx(cam["cy"], abs=1e-12)
    assert got["depth"] == pytest.approx(z0, abs=1e-15)


def test_isotropic_footprint_pixels(orc):
    """Pixels with alpha >= 1/255 form the disk d^2 <= 2 s'^2 ln(255 o)."""
    sigma, z0, f, o = 0.05, 3.0, 110.0, 0.7
    sc = make_scene([[0, 0, z0]], [[sigma] * 3], opacity=o)
    cam = axis_camera(f=f, cx=64.25, cy=63.8)
    r = orc.render(to64(sc), [cam], [scenes.view_state()], dtype=np.float64)
    sigma, o = float(np.float32(sigma)), float(np.float32(o))
    s2 = (f * sigma / z0) ** 2 + KAPPA
    R2 = 2 * s2 * math.log(255 * o)
    ys, xs = np.mgrid[0:128, 0:128]
    d2 = (xs + 0.5 - cam["cx"]) ** 2 + (ys + 0.5 - cam["cy"]) ** 2
    assert np.min(np.abs(d2 - R2)) > 1e-6  # no pixel centre on the boundary
    inside = d2 <= R2
    assert inside.sum() > 20
    np.testing.assert_array_equal(r["alpha"][0] > 0, inside)
    # where drawn, alpha = o exp(-d^2 / (2 s'^2))
    np.testing.assert_allclose(r["alpha"][0][inside], (o * np.exp(-d2 / (2 * s2)))[inside], rtol=1e-12)


def test_anisotropic_on_axis(orc):
    """Rotation about the optical axis: Sigma' = (f/z0)^2 R diag(s1^2, s2^2) R^T + kappa I."""
    th, s1, s2, s3, z0, f = 0.7, 0.03, 0.011, 0.02, 2.5, 200.0
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    sc = make_scene([[0, 0, z0]], [[s1, s2, s3]], quats=[q])
    cam = axis_camera(f=f)
    r = orc.render(to64(sc), [cam], [scenes.view_state()], dtype=np.float64)
    s1, s2, z0 = (float(np.float32(x)) for x in (s1, s2, z0))
    th = 2 * math.atan2(float(np.float32(math.sin(th / 2))), float(np.float32(math.cos(th / 2))))
    Rt = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    S2 = (f / z0) ** 2 * Rt @ np.diag([s1 ** 2, s2 ** 2]) @ Rt.T + KAPPA * np.eye(2)
    np.testing.assert_allclose(rec_fields(r, 0)["conic"], np.linalg.inv(S2), rtol=1e-11)


def test_projection_matches_numerical_jacobian(orc):
    """Off-axis Gaussians: Sigma' equals J_fd W Sigma W^T J_fd^T + kappa I with
    J_fd the central difference of the pinhole map and Sigma from scipy's
    rotation of the (w,x,y,z) quaternion."""
    rng = np.random.default_rng(5)
    cam = scenes.orbit_camera([0.4, -0.3, -1.0], 160, 120)
    W = cam["R"].astype(np.float64)
    t = cam["t"].astype(np.float64)
    n = 12
    means = rng.uniform(-0.4, 0.4, (n, 3))
    scales = np.exp(rng.normal(-3.5, 0.4, (n, 3)))
    quats = rng.standard_normal((n, 4))
    sc = make_scene(means, scales, quats=quats, opacity=0.9)
    s64 = to64(sc)
    r = orc.render(s64, [cam], [scenes.view_state()], dtype=np.float64)
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]

    def proj(p):
        return np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])

    checked = 0
    for i in range(n):
        if r["n_tiles"][i] == 0:
            continue
        m = s64["mean"][:, i]
        tc = W @ m + t
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            J[:, k] = (proj(tc + e) - proj(tc - e)) / 2e-6
        qw, qx, qy, qz = s64["quat"][:, i]
        Rq = Rotation.from_quat([qx, qy, qz, qw]).as_matrix()
        M = Rq @ np.diag(s64["scale"][:, i])
        Sig = M @ M.T
        S2 = J @ W @ Sig @ W.T @ J.T + KAPPA * np.eye(2)
        np.testing.assert_allclose(rec_fields(r, i)["conic"], np.linalg.inv(S2), rtol=2e-6)
        np.testing.assert_allclose([r["rec"][i][0], r["rec"][i][1]], proj(tc), rtol=1e-12)
        assert r["rec"][i][6] == pytest.approx(tc[2], rel=1e-14)
        checked += 1
    assert checked >= 8


def test_guard_band_clamps_jacobian(orc):
    """Far off-screen centres use the Jacobian at the guard-band edge: the 2D
    covariance of an isotropic Gaussian no longer grows with the off-axis slope
    beyond the guard."""
    cam = axis_camera(f=100.0, cx=64.0, cy=64.0)
    lim = 1.3 * 64 / 100.0
    z = 2.0
    sig = 0.2  # big enough to still touch the image from outside
    xs = [lim * z * 1.2, lim * z * 1.5]
    sc = make_scene([[x, 0, z] for x in xs], [[sig] * 3], opacity=0.9)
    r = orc.render(to64(sc), [cam], [scenes.view_state()], dtype=np.float64)
    sig = float(np.float32(sig))
    lim = float(np.float32(1.3)) * 64 / 100.0
    for i in range(2):
        if r["n_tiles"][i] == 0:
            continue
        # J at the clamped slope: J00 = f/z, J02 = -f*lim/z
        J = np.array([[100 / z, 0, -100 * lim / z], [0, 100 / z, 0]])
        S2 = J @ (sig ** 2 * np.eye(3)) @ J.T + KAPPA * np.eye(2)
        np.testing.assert_allclose(rec_fields(r, i)["conic"], np.linalg.inv(S2), rtol=1e-12)


# ---------------------------------------------------------------- colour
def _real_sh_reference(l, m, d):
    """Real SH from scipy's complex SH (Condon-Shortley phase included)."""
    from scipy.special import sph_harm_y
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m < 0:
        return math.sqrt(2) * Y.imag
    if m > 0:
        return math.sqrt(2) * Y.real
    return Y.real


def test_sh_basis_matches_scipy(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        got = orc.sh_basis(d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert got[l * l + l + m] == pytest.approx(_real_sh_reference(l, m, d), abs=1e-13)


def test_sh_orthonormal_by_quadrature(orc):
    n = 20000
    k = np.arange(n) + 0.5
    z = 1 - 2 * k / n
    phi = math.pi * (1 + 5 ** 0.5) * k
    rr = np.sqrt(1 - z * z)
    dirs = np.stack([rr * np.cos(phi), rr * np.sin(phi), z], 1)
    Y = np.stack([orc.sh_basis(d) for d in dirs])
    gram = Y.T @ Y * (4 * math.pi / n)
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-3)


def test_sh0_colour_recovers_dc(orc):
    w = scenes.plain_forward_4k()
    r = orc.render(w.scene, w.cams, w.views)
    valid = r["n_tiles"] > 0
    rgb_in = w.scene["sh"][0] * np.float32(0.28209479177387814) + np.float32(0.5)
    np.testing.assert_allclose(r["rec"][valid][:, 7:10], rgb_in.T[valid], atol=2e-7)


def test_sh3_zero_high_bands_equals_sh0(orc):
    w = scenes.plain_forward_4k()
    s3 = dict(w.scene)
    sh = np.zeros((16, 3, w.scene["sh"].shape[2]), np.float32)
    sh[0] = w.scene["sh"][0]
    s3["sh"], s3["sh_degree"] = sh, 3
    a = orc.render(w.scene, w.cams, w.views)
    b = orc.render(s3, w.cams, w.views)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])


def test_view_dependent_colour_direction(orc):
    """Degree-1 colour: rgb = 0.5 + Y00 dc + sum_m c_m Y_1m(dir), with dir from
    the eye centre to the Gaussian."""
    cam = scenes.orbit_camera([0.5, 0.2, -1.0], 64, 64)
    sh = np.zeros((4, 3, 1))
    sh[1, 0], sh[2, 1], sh[3, 2] = 0.3, -0.2, 0.25
    sc = make_scene([[0.1, -0.05, 0.2]], [[0.05] * 3], sh=sh)
    s64 = to64(sc)
    r = orc.render(s64, [cam], [scenes.view_state()], dtype=np.float64)
    c = scenes.camera_center(cam)
    d = s64["mean"][:, 0] - c
    d /= np.linalg.norm(d)
    exp = [0.5 + 0.3 * _real_sh_reference(1, -1, d), 0.5 - 0.2 * _real_sh_reference(1, 0, d),
           0.5 + 0.25 * _real_sh_reference(1, 1, d)]
    np.testing.assert_allclose(r["rec"][0][7:10], exp, atol=1e-12)


def test_negative_colour_clamped(orc):
    sc = make_scene([[0, 0, 3]], [[0.05] * 3], rgb=[[-0.4, 0.3, 0.9]])
    r = orc.render(sc, [axis_camera()], [scenes.view_state()])
    assert r["clamp"][0] == 1
    assert r["rec"][0][7] == 0.0


# ---------------------------------------------------------------- blending
def _stack(orc, opac, rgbs, dtype=np.float32):
    n = len(opac)
    means = [[0.0, 0.0, 2.0 + 0.1 * k] for k in range(n)]
    sc = make_scene(means, [[0.05] * 3], opacity=opac, rgb=rgbs)
    cam = axis_camera()  # pixel (64, 64) has its centre on the axis
    vs = scenes.view_state(bg=(0.1, 0.2, 0.3))
    r = orc.render(to64(sc) if dtype == np.float64 else sc, [cam], [vs], dtype=dtype)
    return r, vs


def test_transmittance_is_product(orc):
    rng = np.random.default_rng(2)
    o = rng.uniform(0.1, 0.6, 6)
    c = rng.uniform(0, 1, (6, 3))
    r, vs = _stack(orc, o, c, np.float64)
    a = np.minimum(0.99, o.astype(np.float32).astype(np.float64))  # inputs are float32
    T = np.cumprod(np.concatenate([[1.0], 1 - a]))
    C = (r["rec"][:, 7:10] * (a * T[:-1])[:, None]).sum(0)
    assert r["final_T"][0, 64, 64] == pytest.approx(T[-1], rel=1e-14)
    np.testing.assert_allclose(r["rgb"][0, :, 64, 64], C + T[-1] * vs["bg"], rtol=1e-13)
    assert r["n_contrib"][0, 64, 64] == 6


def test_stop_rule_stacked_example(orc):
    """20 stacked splats with alpha = 0.5: 0.5^13 >= 1e-4 > 0.5^14, so exactly
    13 are blended and the 14th is not."""
    r, vs = _stack(orc, [0.5] * 20, [[0.9, 0.4, 0.2]] * 20)
    assert r["n_contrib"][0, 64, 64] == 13
    assert r["final_T"][0, 64, 64] == np.float32(2.0 ** -13)
    c = r["rec"][0, 7:10].astype(np.float64)
    np.testing.assert_allclose(r["rgb"][0, :, 64, 64], c * (1 - 2.0 ** -13) + 2.0 ** -13 * vs["bg"], rtol=1e-6)


def test_alpha_clamp(orc):
    r, _ = _stack(orc, [0.999], [[0.5, 0.5, 0.5]])
    assert r["alpha"][0, 64, 64] == pytest.approx(0.99, abs=1e-7)


def test_cutoff_culls_transparent_gaussians(orc):
    sc = make_scene([[0, 0, 3]], [[0.1] * 3], opacity=0.9 / 255)
    vs = scenes.view_state(bg=(0.25, 0.5, 0.75))
    r = orc.render(sc, [axis_camera()], [vs])
    assert r["n_tiles"][0] == 0 and r["counts"]["K"] == 0
    assert np.all(r["alpha"] == 0)
    np.testing.assert_array_equal(r["rgb"][0], np.broadcast_to(vs["bg"][:, None, None], (3, 128, 128)))


def test_empty_scene_is_background(orc):
    sc = make_scene(np.zeros((0, 3)), np.zeros((0, 3)))
    vs = scenes.view_state(bg=(0.3, 0.1, 0.9))
    r = orc.render(sc, [axis_camera(40, 24)], [vs])
    assert r["rgb"].shape == (1, 3, 24, 40)
    np.testing.assert_array_equal(r["rgb"][0], np.broadcast_to(vs["bg"][:, None, None], (3, 24, 40)))
    assert np.all(r["alpha"] == 0) and r["counts"]["K"] == 0


def test_near_plane_cull(orc):
    sc = make_scene([[0, 0, 0.19], [0, 0, 0.21]], [[0.01] * 3])
    r = orc.render(sc, [axis_camera()], [scenes.view_state()])
    assert r["n_tiles"][0] == 0 and r["n_tiles"][1] > 0


# ---------------------------------------------------------------- tiles and sort
@pytest.fixture(scope="module")
def layered(orc):
    sc = small_layered_scene(seed=4)
    cam = scenes.orbit_camera([0.2, 0.5, -1.0], 100, 70)  # ragged tiles on both axes
    scenes.enforce_distinct_depths(sc, [cam])
    vs = scenes.view_state(0b111, clips=[([0.3, -0.2, 0.9], 0.05, 0b100)], bg=(0.1, 0.1, 0.2))
    return sc, cam, vs


def test_tile_path_equals_brute_force(orc, layered):
    sc, cam, vs = layered
    a = orc.render(sc, [cam], [vs])
    b = orc.render(sc, [cam], [vs], brute_force=True)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    np.testing.assert_array_equal(a["final_T"], b["final_T"])
    np.testing.assert_array_equal(a["n_contrib"], b["n_contrib"])


def test_tile_size_independence(orc, layered):
    sc, cam, vs = layered
    a = orc.render(sc, [cam], [vs], tile=16)
    for t in (8, 32):
        b = orc.render(sc, [cam], [vs], tile=t)
        np.testing.assert_array_equal(a["rgb"], b["rgb"])


def test_keys_sorted_stably(orc, layered):
    sc, cam, vs = layered
    r = orc.render(sc, [cam], [vs], pairs=True)
    order = np.argsort(r["keys_emit"], kind="stable")
    np.testing.assert_array_equal(r["keys"], r["keys_emit"][order])
    np.testing.assert_array_equal(r["vals"], r["vals_emit"][order])
    assert int(r["n_tiles"].sum()) == r["counts"]["K"] == len(r["keys"])
    # key = tile << 32 | bits(depth)
    depth_bits = r["rec"][:, 6].astype(np.float32).view(np.uint32)
    np.testing.assert_array_equal(r["keys"] & 0xFFFFFFFF, depth_bits[r["vals"]])
    # ranges partition [0, K) in tile order
    rg = r["ranges"]
    nonempty = rg[:, 1] > rg[:, 0]
    tiles = (r["keys"] >> 32).astype(np.int64)
    for t in np.nonzero(nonempty)[0]:
        assert np.all(tiles[rg[t, 0]:rg[t, 1]] == t)
    assert (rg[:, 1] - rg[:, 0]).sum() == len(r["keys"])


def test_tile_lists_by_box_overlap(orc, layered):
    """A Gaussian is listed in exactly the tiles its pixel box overlaps."""
    sc, cam, vs = layered
    r = orc.render(sc, [cam], [vs], pairs=True)
    tx = (cam["width"] + 15) // 16
    ty = (cam["height"] + 15) // 16
    rec = r["rec"].astype(np.float64)
    for i in np.nonzero(r["n_tiles"])[0][:60]:
        u, v, ca, cb, cc = rec[i, :5]
        S = np.linalg.inv(np.array([[ca, cb], [cb, cc]]))
        hx, hy = math.sqrt(QMAX * S[0, 0]), math.sqrt(QMAX * S[1, 1])
        want = {(x, y) for y in range(ty) for x in range(tx)
                if (x * 16 <= u + hx and u - hx < (x + 1) * 16 and y * 16 <= v + hy and v - hy < (y + 1) * 16)}
        got = {(int(k >> 32) % tx, int(k >> 32) // tx) for k, val in zip(r["keys_emit"], r["vals_emit"]) if val == i}
        assert got == want


# ---------------------------------------------------------------- layers, cuts, views
def test_layer_mask_equals_deleting_layers(orc, layered):
    sc, cam, _ = layered
    for mask in (0b001, 0b101, 0b110):
        keep = np.nonzero((mask >> sc["layer"].astype(np.int64)) & 1)[0]
        a = orc.render(sc, [cam], [scenes.view_state(mask)])
        b = orc.render(scenes.subset(sc, keep), [cam], [scenes.view_state(0xFFFFFFFF)])
        np.testing.assert_array_equal(a["rgb"], b["rgb"])


def test_clip_equals_deleting_clipped(orc, layered):
    sc, cam, _ = layered
    n, d, bits = np.array([0.6, 0.0, -0.8], np.float32), np.float32(0.1), 0b011
    s = (sc["mean"].astype(np.float32).T @ n).astype(np.float64) + d
    # evaluate the plane test independently in float64; keep the cases far from 0
    applies = ((bits >> sc["layer"].astype(np.int64)) & 1).astype(bool)
    assert np.min(np.abs(s[applies])) > 1e-5
    keep = np.nonzero(~(applies & (s < 0)))[0]
    a = orc.render(sc, [cam], [scenes.view_state(clips=[(n, d, bits)])])
    b = orc.render(scenes.subset(sc, keep), [cam], [scenes.view_state()])
    np.testing.assert_array_equal(a["rgb"], b["rgb"])


def test_quaternion_sign_invariance(orc, layered):
    sc, cam, vs = layered
    s2 = dict(sc)
    s2["quat"] = -sc["quat"]
    np.testing.assert_array_equal(orc.render(sc, [cam], [vs])["rgb"], orc.render(s2, [cam], [vs])["rgb"])


def test_permutation_invariance(orc, layered):
    sc, cam, vs = layered
    perm = np.random.default_rng(1).permutation(sc["mean"].shape[1])
    a = orc.render(sc, [cam], [vs])
    b = orc.render(scenes.subset(sc, perm), [cam], [vs])
    np.testing.assert_array_equal(a["rgb"], b["rgb"])


def test_stereo_views_equal_mono(orc, layered):
    sc, _, vs = layered
    eyes = scenes.stereo_cameras([0.1, 0.3, -1.0], 64, 48)
    both = orc.render(sc, eyes, [vs, vs])
    for e in range(2):
        mono = orc.render(sc, [eyes[e]], [vs])
        np.testing.assert_array_equal(both["rgb"][e], mono["rgb"][0])


def test_multi_model_batch_equals_single(orc, layered):
    sc, cam, vs = layered
    other = scenes.uniform_cube_scene(300, 3, seed=9)
    cam2 = scenes.orbit_camera([1, 0, 0], 40, 56)
    both = orc.render([sc, other], [cam, cam2], [vs, scenes.view_state()])
    a = orc.render(sc, [cam], [vs])
    b = orc.render(other, [cam2], [scenes.view_state()])
    np.testing.assert_array_equal(both["rgb"][0], a["rgb"][0])
    np.testing.assert_array_equal(both["rgb"][1], b["rgb"][0])


def test_double_and_float_agree(orc, layered):
    sc, cam, vs = layered
    a = orc.render(sc, [cam], [vs])
    b = orc.render(to64(sc), [cam], [vs], dtype=np.float64)
    ok = a["margin"] >= 1
    np.testing.assert_allclose(a["rgb"][:, :, ok[0]], b["rgb"][:, :, ok[0]], atol=2e-5)


# ---------------------------------------------------------------- shared depth order (stereo)
def _stereo_case(toe_in_deg, seed=2, W=96, H=80):
    sc = small_layered_scene(seed=seed, n_per_layer=250, log_scale_mu=-3.4)
    left, right, centre = scenes.stereo_rig([0.2, 0.3, -1.0], W, H, ipd=0.3, distance=1.6, toe_in_deg=toe_in_deg)
    vs = scenes.view_state(0b111, bg=(0.1, 0.2, 0.3))
    return sc, [left, right], [vs, vs], centre


def test_sort_camera_equal_to_the_view_is_the_default(orc):
    """Sorting each view by the depth in its own camera is the default order."""
    sc, cams, vss, _ = _stereo_case(4.0)
    a = orc.render(sc, cams, vss, pairs=True)
    b = orc.render(sc, cams, vss, pairs=True, sort_cams=cams)
    for k in ("rgb", "alpha", "keys", "vals", "ranges", "last"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_shared_order_sorts_every_tile_by_the_centre_depth(orc):
    """Converging eyes sorted by the centre camera's depth: every tile holds
    the same pairs as with per-eye sorting, ordered by (centre depth bits,
    Gaussian index); the brute-force blend in the same order agrees bit for
    bit; the images differ from per-eye sorting, but only slightly (pairs of
    nearly equal depth swap)."""
    sc, cams, vss, centre = _stereo_case(6.0)
    n = sc["mean"].shape[1]
    own = orc.render(sc, cams, vss, pairs=True)
    sh = orc.render(sc, cams, vss, pairs=True, sort_cams=[centre, centre])
    bf = orc.render(sc, cams, vss, brute_force=True, sort_cams=[centre, centre])
    # centre depth of every Gaussian, float32 in the oracle's operation order
    R = centre["R"].astype(np.float32).reshape(9)
    m = sc["mean"].astype(np.float32)
    zc = ((R[6] * m[0] + R[7] * m[1]) + R[8] * m[2]) + np.float32(centre["t"][2])
    kc = zc.astype(np.float32).view(np.uint32)
    np.testing.assert_array_equal(sh["ranges"], own["ranges"])
    for t0, t1 in sh["ranges"]:
        v_sh, v_own = sh["vals"][t0:t1], own["vals"][t0:t1]
        assert sorted(v_sh.tolist()) == sorted(v_own.tolist())
        g = v_sh % n
        order = np.lexsort((g, kc[g]))
        np.testing.assert_array_equal(order, np.arange(len(g)))
        np.testing.assert_array_equal(sh["keys"][t0:t1] & 0xFFFFFFFF, kc[g])
    np.testing.assert_array_equal(bf["rgb"], sh["rgb"])
    d = np.abs(sh["rgb"] - own["rgb"])
    assert 0 < d.max() and d.mean() < 1e-3
    assert not np.array_equal(sh["keys"], own["keys"])


def test_parallel_eyes_share_the_per_eye_order(orc):
    """Parallel eyes: the centre camera's depth rows equal the eyes', so
    the shared order is each eye's own and the images are identical."""
    sc, cams, vss, centre = _stereo_case(0.0)
    own = orc.render(sc, cams, vss, pairs=True)
    sh = orc.render(sc, cams, vss, pairs=True, sort_cams=[centre, centre])
    for k in ("rgb", "alpha", "keys", "vals", "last"):
        np.testing.assert_array_equal(sh[k], own[k], err_msg=k)


# ---------------------------------------------------------------- per-layer opacity (fading)
def _premultiplied(sc, factors):
    """The scene with each Gaussian's opacity multiplied by its layer's factor
    (in float32 for a float32 scene, one rounding like the render's)."""
    out = dict(sc)
    f = np.asarray(factors, np.float32)[sc["layer"].astype(np.int64)]
    out["opacity"] = (sc["opacity"] * f.astype(sc["opacity"].dtype)).astype(sc["opacity"].dtype)
    return out


def test_layer_fade_of_ones_is_no_fading(orc, layered):
    sc, cam, vs = layered
    a = orc.render(sc, [cam], [vs], pairs=True)
    b = orc.render(sc, [cam], [scenes.view_state(vs["layer_mask"], vs["clips"], vs["bg"], layer_opacity=[1.0] * 32)],
                   pairs=True)
    for k in ("rgb", "alpha", "final_T", "rec", "keys", "vals"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_layer_fade_equals_premultiplied_opacity(orc, layered, dtype):
    """Fading layer l by f draws the scene whose layer-l opacities are o f."""
    sc, cam, vs = layered
    fac = [0.35, 1.0, 0.6]
    s = to64(sc) if dtype == np.float64 else sc
    vf = scenes.view_state(vs["layer_mask"], vs["clips"], vs["bg"], layer_opacity=fac)
    a = orc.render(s, [cam], [vf], dtype=dtype, pairs=True)
    b = orc.render(_premultiplied(s, fac), [cam], [vs], dtype=dtype, pairs=True)
    for k in ("rgb", "alpha", "final_T", "rec", "keys", "vals"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    # and the fading changed the image
    assert np.abs(a["rgb"] - orc.render(s, [cam], [vs], dtype=dtype)["rgb"]).max() > 1e-3


def test_layer_fade_to_zero_hides_the_layer(orc, layered):
    """A factor of 0 takes every opacity below the 1/255 cut: the layer is
    gone, exactly as if its mask bit were clear."""
    sc, cam, vs = layered
    vf = scenes.view_state(0b111, vs["clips"], vs["bg"], layer_opacity=[1.0, 0.0, 1.0])
    a = orc.render(sc, [cam], [vf])
    b = orc.render(sc, [cam], [scenes.view_state(0b101, vs["clips"], vs["bg"])])
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    np.testing.assert_array_equal(a["alpha"], b["alpha"])


def test_layer_fade_monotone_in_the_factor(orc):
    """One splat over a black background: its peak alpha is o f, clamped at
    0.99, and zero below the 1/255 cut."""
    sc = make_scene([[0.0, 0.0, 3.0]], [[0.05, 0.05, 0.05]], opacity=[0.8], rgb=[[1.0, 1.0, 1.0]])
    cam = axis_camera(33, 33, f=80.0, cx=16.5, cy=16.5)
    for f in (1.0, 0.5, 0.1, 0.004):
        r = orc.render(to64(sc), [cam], [scenes.view_state(layer_opacity=[f])], dtype=np.float64)
        peak = r["alpha"][0].max()
        of = float(np.float32(0.8)) * float(np.float32(f))  # the float32 inputs, multiplied in float64
        want = of if of >= 1 / 255 else 0.0
        assert abs(peak - want) < 1e-9 * max(want, 1.0), (f, peak)
