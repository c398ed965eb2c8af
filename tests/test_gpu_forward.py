"""GPU parity of the forward pass (HIP kernels through the C ABI) against the
CPU oracle: records, tile boxes, emitted and sorted keys and tile ranges
bit-exact; images within 1e-4 max-abs."""
import numpy as np
import pytest

from paper_2410_16978_amd import scenes
from tests.gpu_helpers import compare_forward, gpu_forward
from tests.helpers import axis_camera, make_scene, small_layered_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_16978_amd import rasterizer
    rasterizer.lib()


def test_plain_forward_4k(orc):
    w = scenes.plain_forward_4k()
    st = compare_forward(w.scene, w.cams, w.views, orc, label="4k")
    print("plain 4k:", st)


def test_layered_sh3_mask_clip_ragged(orc):
    sc = small_layered_scene(seed=4, n_per_layer=400)
    cam = scenes.orbit_camera([0.2, 0.5, -1.0], 100, 70)
    scenes.enforce_distinct_depths(sc, [cam])
    vs = scenes.view_state(0b101, clips=[([0.3, -0.2, 0.9], 0.05, 0b100), ([1, 0, 0], 0.2, 0b001)],
                           bg=(0.1, 0.2, 0.3))
    print("layered:", compare_forward(sc, [cam], [vs], orc, label="layered"))


def test_stereo_two_views(orc):
    sc = small_layered_scene(seed=5, n_per_layer=500, n_layers=5)
    eyes = scenes.stereo_cameras([0.1, 0.3, -1.0], 96, 112)
    scenes.enforce_distinct_depths(sc, eyes)
    vs = scenes.view_state(0b11011, clips=[([0.0, 1.0, 0.2], 0.1, 0b00011)])
    print("stereo:", compare_forward(sc, eyes, [vs, vs], orc, label="stereo"))


def test_many_views_sh1(orc):
    sc = scenes.shell_scene(300, 3, 1, seed=8, log_scale_mu=-3.5, log_scale_sigma=0.4, opacity="normal")
    cams = [scenes.orbit_camera(d, 64, 48) for d in ([1, 0, 0], [0, 1, 0.1], [0, 0, -1], [-1, 0.2, 0.1],
                                                      [0.3, -1, 0.2])]
    scenes.enforce_distinct_depths(sc, cams)
    vss = [scenes.view_state(0b111, bg=(0.5, 0.5, 0.5))] * 5
    print("5 views:", compare_forward(sc, cams, vss, orc, label="5 views"))


def test_sh2_large_splats_many_tiles(orc):
    rng = np.random.default_rng(3)
    n = 60
    sh = rng.normal(0, 0.2, (9, 3, n))
    sh[0] += 0.5
    sc = make_scene(rng.uniform(-0.6, 0.6, (n, 3)), np.exp(rng.normal(-1.8, 0.3, (n, 3))),
                    quats=rng.standard_normal((n, 4)), opacity=rng.uniform(0.05, 0.95, n), sh=sh)
    cam = scenes.orbit_camera([0.0, 0.2, -1.0], 150, 130)
    scenes.enforce_distinct_depths(sc, [cam])
    print("large splats:", compare_forward(sc, [cam], [scenes.view_state()], orc, label="large"))


def test_crowded_tiles_and_depth_ties(orc):
    """40k small splats over 9 tiles of a 128x96 image: per-tile segments of
    about 1k to 22k pairs, so both the in-LDS and the chunked per-tile depth
    sort run; a third of the splats share one of 9 exact depths, so equal
    keys must keep emission order."""
    rng = np.random.default_rng(11)
    n = 40000
    z = rng.uniform(1.5, 6.0, n)
    tied = rng.random(n) < 0.33
    z[tied] = 1.5 + 0.5 * rng.integers(0, 9, tied.sum())
    xy = rng.uniform(-0.12, 0.12, (n, 2)) * z[:, None]
    means = np.column_stack([xy, z])
    sc = make_scene(means, np.exp(rng.normal(-5.5, 0.3, (n, 3))), quats=rng.standard_normal((n, 4)),
                    opacity=rng.uniform(0.01, 0.3, n), rgb=rng.uniform(0, 1, (n, 3)))
    cam = axis_camera(128, 96, f=110.0, cx=70.0, cy=52.0)
    st = compare_forward(sc, [cam], [scenes.view_state()], orc, label="crowded")
    print("crowded tiles:", st)
    assert st["K"] > 3 * 8192


def test_tile_grouping_at_the_4096_tile_boundary(orc):
    """A view of exactly 4096 tiles (1024 x 1024: the one-pass 12-bit tile
    grouping) and one of 4160 tiles (1040 x 1024: the 8-bit tile passes)
    both give the oracle's sorted keys, tile ranges and images."""
    sc = small_layered_scene(seed=5, n_per_layer=1500, n_layers=2, sh_degree=1, log_scale_mu=-3.0)
    for W, H in ((1024, 1024), (1040, 1024)):
        cam = scenes.orbit_camera([0.1, 0.3, -1.0], W, H)
        scenes.enforce_distinct_depths(sc, [cam])
        st = compare_forward(sc, [cam], [scenes.view_state()], orc, label=f"{W}x{H}")
        print(f"{W}x{H}:", st)
        assert st["K"] > 1000


def test_raw_parameters_match_activated():
    """A model given as log-scales and logits (raw = 1) renders bit-for-bit
    like the same model given the activated values gsr_activate returns, and
    those match exp / logistic of float64 within float32 rounding."""
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=9, n_per_layer=300)
    cam = scenes.orbit_camera([0.3, -0.2, -1.0], 90, 70)
    raw = rz.to_device(sc)
    raw["scale"] = torch.tensor(sc["log_scale"], device="cuda").contiguous()
    raw["opacity"] = torch.tensor(sc["opacity_logit"], device="cuda").contiguous()
    raw["raw"] = True
    s_act, o_act = rz.activate(raw)
    np.testing.assert_allclose(s_act.cpu().numpy(), np.exp(sc["log_scale"].astype(np.float64)), rtol=4e-7)
    np.testing.assert_allclose(o_act.cpu().numpy(), 1 / (1 + np.exp(-sc["opacity_logit"].astype(np.float64))),
                               rtol=4e-7)
    act = dict(raw, scale=s_act, opacity=o_act, raw=False)
    vs = [scenes.view_state(0b111, bg=(0.1, 0.2, 0.3))]
    rgb_r, a_r, st_r = rz.rasterize_forward(raw, [cam], vs)
    rgb_a, a_a, st_a = rz.rasterize_forward(act, [cam], vs)
    assert st_r.n_pairs == st_a.n_pairs > 0
    np.testing.assert_array_equal(rgb_r.cpu().numpy(), rgb_a.cpu().numpy())
    np.testing.assert_array_equal(a_r.cpu().numpy(), a_a.cpu().numpy())


def test_tiny_and_odd_images(orc):
    sc = scenes.uniform_cube_scene(500, 0, seed=2, log_scale_mu=-2.5)
    for W, H in ((1, 1), (17, 5), (33, 64)):
        cam = scenes.front_camera(W, H)
        compare_forward(sc, [cam], [scenes.view_state(bg=(0.2, 0.4, 0.6))], orc, label=f"{W}x{H}")


def test_empty_and_fully_culled(orc):
    cam = scenes.front_camera(40, 24)
    vs = scenes.view_state(bg=(0.3, 0.1, 0.9))
    empty = make_scene(np.zeros((0, 3)), np.zeros((0, 3)))
    _, (rgb, alpha, st, dbg) = gpu_forward(empty, [cam], [vs])
    np.testing.assert_array_equal(rgb.cpu().numpy()[0], np.broadcast_to(vs["bg"][:, None, None], (3, 24, 40)))
    assert np.all(alpha.cpu().numpy() == 0)
    # every Gaussian on a hidden layer
    sc = scenes.uniform_cube_scene(300, 0, seed=1)
    _, (rgb, alpha, st, dbg) = gpu_forward(sc, [cam], [scenes.view_state(0b10, bg=(0.3, 0.1, 0.9))])
    assert st.n_pairs == 0
    np.testing.assert_array_equal(rgb.cpu().numpy()[0], np.broadcast_to(vs["bg"][:, None, None], (3, 24, 40)))
    compare_forward(sc, [cam], [scenes.view_state(0b10)], orc, label="culled")


def test_stop_rule_on_gpu():
    """20 stacked splats with alpha 0.5: exactly 13 blended (T = 2^-13)."""
    means = [[0.0, 0.0, 2.0 + 0.1 * k] for k in range(20)]
    sc = make_scene(means, [[0.05] * 3], opacity=[0.5] * 20, rgb=[[0.9, 0.4, 0.2]] * 20)
    cam = scenes.make_camera(np.eye(3), [0, 0, 0], 128, 128, fx=110, fy=110, cx=64.5, cy=64.5)
    _, (rgb, alpha, st, dbg) = gpu_forward(sc, [cam], [scenes.view_state()])
    T = st.final_T.cpu().numpy().reshape(128, 128)
    assert st.last.cpu().numpy().reshape(128, 128)[64, 64] > 0
    assert T[64, 64] == np.float32(2.0 ** -13)


def test_capacity_regrow_and_overflow_flag(orc):
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    w = scenes.plain_forward_4k()
    model = rz.to_device(w.scene)
    rgb, alpha, st = rz.rasterize_forward(model, w.cams, w.views, capacity=100)  # regrows to the exact need
    ref = orc.render(w.scene, w.cams, w.views)
    assert st.n_pairs == ref["counts"]["K"] and st.capacity >= st.n_pairs
    small = rz.make_state(4096, 1, 128, 128, 100, "cuda")
    rz.rasterize_forward(model, w.cams, w.views, state=small, sync=False)
    torch.cuda.synchronize()
    with pytest.raises(rz.GsrError) as e:
        rz.forward_check(small)
    assert e.value.status == rz.GSR_ENOSPACE


def test_overflow_and_error_words_are_sticky_until_checked():
    """An overflow in one non-synchronising call is still reported after a
    later call that fits (the flags are not reset per call); the check clears
    them.  An error word set on the state (here from the host, standing in
    for a kernel's bounded wait giving up) makes the next synchronising
    forward fail with GSR_EDEVICE, and the check reports and clears it."""
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    w = scenes.plain_forward_4k()
    model = rz.to_device(w.scene)
    small = rz.make_state(4096, 1, 128, 128, 100, "cuda")
    rz.rasterize_forward(model, w.cams, w.views, state=small, sync=False)  # overflows
    empty = [scenes.view_state(0)]  # every layer hidden: no pairs
    rz.rasterize_forward(model, w.cams, empty, state=small, sync=False)
    torch.cuda.synchronize()
    with pytest.raises(rz.GsrError) as e:
        rz.forward_check(small)
    assert e.value.status == rz.GSR_ENOSPACE
    assert rz.forward_check(small) == 0  # reported once
    st = rz.make_state(4096, 1, 128, 128, 100_000, "cuda")
    st.counters[2] = 16
    with pytest.raises(rz.GsrError) as e:
        rz.rasterize_forward(model, w.cams, w.views, state=st)
    assert e.value.status == rz.GSR_EDEVICE
    with pytest.raises(rz.GsrError) as e:
        rz.forward_check(st)
    assert e.value.status == rz.GSR_EDEVICE
    rgb, alpha, st = rz.rasterize_forward(model, w.cams, w.views, state=st)
    assert rz.forward_check(st) == st.n_pairs > 0


def test_invalid_arguments_rejected():
    from paper_2410_16978_amd import rasterizer as rz
    w = scenes.plain_forward_4k()
    model = rz.to_device(w.scene)
    bad = dict(w.cams[0])
    bad["width"] = 0
    with pytest.raises(rz.GsrError) as e:
        rz.rasterize_forward(model, [bad], w.views)
    assert e.value.status == rz.GSR_EINVAL
    vs = scenes.view_state()
    vs["clips"] = [([0, 0, 1], 0.0, 1)] * 8
    rz.rasterize_forward(model, w.cams, [vs])  # 8 planes are allowed
    model2 = dict(model)
    model2["sh_degree"] = 4
    with pytest.raises(ValueError):
        rz.rasterize_forward(model2, w.cams, w.views)


def test_layer_fading(orc):
    """Per-layer opacity factors (fading between layers), one of them small
    enough to push part of its layer below the 1/255 cut."""
    sc = small_layered_scene(seed=12, n_per_layer=500, n_layers=4)
    cams = [scenes.orbit_camera([0.2, 0.4, -1.0], 90, 66), scenes.orbit_camera([-0.3, 0.1, -1.0], 90, 66)]
    scenes.enforce_distinct_depths(sc, cams)
    vss = [scenes.view_state(0b1111, clips=[([0.3, -0.2, 0.9], 0.05, 0b0100)], bg=(0.1, 0.2, 0.3),
                             layer_opacity=[1.0, 0.3, 0.012, 0.75]),
           scenes.view_state(0b1011, layer_opacity=[0.0, 0.5, 1.0, 1.0])]
    print("fading:", compare_forward(sc, cams, vss, orc, label="fading"))


def test_mip_filters(orc):
    """Mip-Splatting's 2D filter (per view) and 3D filter (per Gaussian
    variances from the cameras): records bit-exact, images within the bar;
    also from compressed attributes."""
    from paper_2410_16978_amd import compress, mip
    from paper_2410_16978_amd import rasterizer as rz
    from oracle import compressed as oc
    sc = small_layered_scene(seed=14, n_per_layer=400)
    cams = scenes.stereo_cameras([0.2, 0.4, -1.0], 96, 72)
    scenes.enforce_distinct_depths(sc, cams)
    sc["filter_3d"] = mip.filter_3d_variance(sc["mean"], cams) * 50.0  # widened to matter at this size
    vs = scenes.view_state(0b111, bg=(0.1, 0.2, 0.3), mip_2d_var=0.1)
    print("mip:", compare_forward(sc, cams, [vs, vs], orc, label="mip"))
    comp = compress.compress(sc, "packed")
    comp["filter_3d"] = sc["filter_3d"]
    dec = oc.decode(comp)
    dec["filter_3d"] = sc["filter_3d"]
    print("mip packed:", compare_forward(dec, cams, [vs, vs], orc, label="mip packed",
                                         device_model=rz.to_device_compressed(comp)))


def test_mip_filters_are_forward_only():
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=15, n_per_layer=50)
    cam = scenes.orbit_camera([0.2, 0.4, -1.0], 32, 32)
    model = rz.to_device(sc)
    vs = scenes.view_state(mip_2d_var=0.1)
    rgb, alpha, st = rz.rasterize_forward(model, [cam], [vs])
    with pytest.raises(rz.GsrError):
        rz.rasterize_backward(model, [cam], [vs], st, torch.zeros_like(rgb), torch.zeros_like(alpha))


def test_dense_tiles(orc):
    """Tiles of more than 1024 pairs (up to about 2900 here, a dozen batches
    of 256) on two views: the same bar as every other tile."""
    sc = scenes.shell_scene(1000, 3, 1, seed=41, log_scale_mu=-2.8, log_scale_sigma=0.4, opacity="normal")
    cams = [scenes.orbit_camera([0.2, 0.3, -1.0], 48, 40), scenes.orbit_camera([-0.1, 0.35, -1.0], 48, 40)]
    scenes.enforce_distinct_depths(sc, cams)
    ref = orc.render(sc, cams[:1], [scenes.view_state()], pairs=True)
    counts = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    assert (counts >= 1024).sum() >= 2
    print("dense:", compare_forward(sc, cams, [scenes.view_state(bg=(0.2, 0.1, 0.3))] * 2, orc, label="dense"))


def test_batch_boundaries_and_early_stop(orc):
    """One 16 x 16 tile holding exactly N pairs for N around the 256-pair
    batches (255 to 769).  Faint splats keep pixels live through the last,
    partial batch (each batch's records load during the one before);
    opaque, wide splats stop every pixel in the first batch while the second
    batch's records are already loading, so the block leaves at the next
    batch's test.  Records, pairs and images against the oracle."""
    cam = axis_camera(16, 16, f=20.0, cx=8.0, cy=8.0)
    vs = scenes.view_state()
    for n in (255, 256, 257, 511, 512, 513, 769):
        for label, op_lo, op_hi, log_s in (("faint", 0.005, 0.02, -3.5), ("opaque", 0.95, 0.99, -0.5)):
            rng = np.random.default_rng(n)
            z = rng.uniform(2.0, 4.0, n)
            xy = rng.uniform(-0.1, 0.1, (n, 2)) * z[:, None]
            sc = make_scene(np.column_stack([xy, z]), np.exp(rng.normal(log_s, 0.2, (n, 3))),
                            quats=rng.standard_normal((n, 4)), opacity=rng.uniform(op_lo, op_hi, n),
                            rgb=rng.uniform(0, 1, (n, 3)))
            scenes.enforce_distinct_depths(sc, [cam])
            if label == "opaque":
                ref = orc.render(sc, [cam], [vs], pairs=True)
                assert int(ref["last"].max()) <= 256  # every pixel stops in the first batch
            st = compare_forward(sc, [cam], [vs], orc, label=f"{label} {n}")
            assert st["K"] == n
