"""GPU parity of the backward pass against the oracle's exact gradient of the
same float32 forward (the bar of tests/gpu_helpers.assert_grad_close), GPU
central differences, frozen layers, max contribution and activity, and the
autograd wrapper's chain rule.  Every gradient comparison first checks the
forward (images and last blended index) against the oracle."""
import numpy as np
import pytest

from paper_2410_16978_amd import scenes
from tests.gpu_helpers import assert_grad_close, checked_exempt, grad_refs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(seed=3, n_per_layer=300, n_layers=3, D=3, W=72, H=56, n_views=1):
    sc = scenes.shell_scene(n_per_layer, n_layers, D, seed=seed, log_scale_mu=-3.2, log_scale_sigma=0.4,
                            opacity="normal")
    cams = [scenes.orbit_camera([0.3 + 0.5 * v, 0.2, -1.0], W, H) for v in range(n_views)]
    scenes.enforce_distinct_depths(sc, cams)
    vss = [scenes.view_state((1 << n_layers) - 1, clips=[([0.2, 0.1, 1.0], 0.3, 0b1)], bg=(0.2, 0.3, 0.1))] * n_views
    rng = np.random.default_rng(seed)
    Gr = rng.standard_normal((n_views, 3, H, W)).astype(np.float32)
    Ga = rng.standard_normal((n_views, H, W)).astype(np.float32)
    return sc, cams, vss, Gr, Ga


def _gpu_grads(sc, cams, vss, Gr, Ga, trainable=0xFFFFFFFF):
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    model = rz.to_device(sc)
    rgb, alpha, st = rz.rasterize_forward(model, cams, vss)
    n = sc["mean"].shape[1]
    mc = torch.zeros(n, device="cuda")
    act = torch.zeros(n, device="cuda")
    g = rz.rasterize_backward(model, cams, vss, st, torch.as_tensor(Gr).cuda(), torch.as_tensor(Ga).cuda(),
                              trainable=trainable, max_contrib=mc, activity=act)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in g.items()}
    out["max_contrib"] = mc.cpu().numpy()
    out["activity"] = act.cpu().numpy()
    out["last"] = st.last.cpu().numpy().view(np.uint32)
    out["final_T"] = st.final_T.cpu().numpy()
    out["rgb"] = rgb.cpu().numpy()
    out["alpha"] = alpha.cpu().numpy()
    return out


def _refs(orc, sc, cams, vss, Gr, Ga, got, trainable=0xFFFFFFFF, label=""):
    """Exact reference gradient, its float32 sensitivity, and the flip
    exemption (after checking the GPU forward against the oracle)."""
    ref, sens, g32 = grad_refs(orc, sc, cams, vss, Gr, Ga, trainable=trainable)
    ex = checked_exempt(orc, sc, cams, vss, got["rgb"], got["alpha"], got["last"], got["final_T"], label)
    return ref, sens, g32, ex


@pytest.mark.parametrize("D,n_views", [(3, 1), (0, 1), (1, 2), (2, 3)])
def test_gradients_match_oracle(orc, D, n_views):
    sc, cams, vss, Gr, Ga = _case(seed=3 + D, D=D, n_views=n_views)
    got = _gpu_grads(sc, cams, vss, Gr, Ga)
    ref, sens, g32, ex = _refs(orc, sc, cams, vss, Gr, Ga, got, label=f"D{D} views{n_views}")
    for k in ("mean", "scale", "quat", "opacity", "sh", "activity"):
        assert_grad_close(got[k], ref[k], sens[k], k, ex, g32[k])
    np.testing.assert_allclose(got["max_contrib"][~ex], ref["max_contrib"][~ex], rtol=1e-4, atol=1e-7)


def test_backward_is_bitwise_reproducible():
    sc, cams, vss, Gr, Ga = _case(seed=14, D=3, n_views=2)
    a = _gpu_grads(sc, cams, vss, Gr, Ga)
    b = _gpu_grads(sc, cams, vss, Gr, Ga)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_frozen_layers_exactly_zero(orc):
    sc, cams, vss, Gr, Ga = _case(seed=9)
    got = _gpu_grads(sc, cams, vss, Gr, Ga, trainable=0b100)
    frozen = sc["layer"] != 2
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        assert np.all(got[k][..., frozen] == 0)
    assert np.all(got["activity"][frozen] == 0)
    ref, sens, g32, ex = _refs(orc, sc, cams, vss, Gr, Ga, got, 0b100, label="frozen")
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        assert_grad_close(got[k], ref[k], sens[k], k, ex, g32[k])


def test_gradient_central_differences_on_gpu():
    """Central differences of the GPU forward itself on a window-limited loss
    (float32 forward, so the tolerance is 2e-2)."""
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc, cams, vss, Gr, Ga = _case(seed=21, n_per_layer=60, n_layers=2, D=2)
    n = sc["mean"].shape[1]
    model = rz.to_device(sc)
    rgb, alpha, st = rz.rasterize_forward(model, cams, vss)
    rng = np.random.default_rng(1)
    mc = torch.zeros(n, device="cuda")
    g_full = rz.rasterize_backward(model, cams, vss, st, torch.as_tensor(Gr).cuda(), torch.as_tensor(Ga).cuda(),
                                   max_contrib=mc)
    cand = np.nonzero(mc.cpu().numpy() > 0.1)[0]
    checked = 0
    for i in rng.permutation(cand)[:12]:
        for key, comp in (("mean", int(rng.integers(0, 3))), ("opacity", None), ("sh", 0)):
            t = model[key]
            idx = (comp, int(i)) if key == "mean" else ((int(i),) if key == "opacity" else (0, 0, int(i)))
            g_an = float(g_full[key][idx])
            th = float(t[idx])
            h = 2e-3 if key == "mean" else 1e-2

            def loss(val):
                t[idx] = val
                r, a, _ = rz.rasterize_forward(model, cams, vss)
                t[idx] = th
                return float((r.double() * torch.as_tensor(Gr).cuda().double()).sum()
                             + (a.double() * torch.as_tensor(Ga).cuda().double()).sum())

            fd = (loss(th + h) - loss(th - h)) / (2 * h)
            fd2 = (loss(th + h / 2) - loss(th - h / 2)) / h
            if abs(fd - fd2) > 2e-2 * max(abs(fd), 1e-2):
                continue
            assert abs(g_an - fd) <= 2e-2 * max(abs(fd), 1e-2), (key, idx, g_an, fd)
            checked += 1
    assert checked >= 12


def test_autograd_function_chain_rule(orc):
    """render_params: the kernels apply exp / logistic to the raw parameters
    and chain their gradients."""
    import torch
    from paper_2410_16978_amd import autograd as ag
    from paper_2410_16978_amd import rasterizer as rz
    sc, cams, vss, Gr, Ga = _case(seed=12, D=1)
    dev = "cuda"
    params = {k: torch.tensor(sc[k], device=dev, requires_grad=True)
              for k in ("mean", "log_scale", "quat", "opacity_logit", "sh")}
    layer = torch.tensor(sc["layer"], device=dev)
    rctx = ag.RenderContext()
    rgb, alpha = ag.render_params(params, layer, 1, cams, vss, rctx)
    loss = (rgb * torch.tensor(Gr, device=dev)).sum() + (alpha * torch.tensor(Ga, device=dev)).sum()
    loss.backward()
    torch.cuda.synchronize()
    # the oracle takes the activations exactly as the kernels computed them
    act = dict(sc)
    sc_t, op_t = rz.activate({"mean": params["mean"].detach(), "scale": params["log_scale"].detach(),
                              "quat": params["quat"].detach(), "opacity": params["opacity_logit"].detach(),
                              "sh": params["sh"].detach(), "layer": layer, "sh_degree": sc["sh_degree"],
                              "raw": True})
    act["scale"] = sc_t.cpu().numpy()
    act["opacity"] = op_t.cpu().numpy()
    got = {"rgb": rgb.detach().cpu().numpy(), "alpha": alpha.detach().cpu().numpy(),
           "last": rctx.state.last.cpu().numpy().view(np.uint32), "final_T": rctx.state.final_T.cpu().numpy()}
    ref, sens, g32, ex = _refs(orc, act, cams, vss, Gr, Ga, got, label="autograd")
    o = act["opacity"].astype(np.float64)
    s_ = act["scale"].astype(np.float64)
    assert_grad_close(params["mean"].grad.cpu().numpy(), ref["mean"], sens["mean"], "mean", ex, g32["mean"])
    assert_grad_close(params["log_scale"].grad.cpu().numpy(), ref["scale"] * s_, sens["scale"] * s_, "log_scale", ex,
                      g32["scale"] * s_)
    assert_grad_close(params["opacity_logit"].grad.cpu().numpy(), ref["opacity"] * o * (1 - o),
                      sens["opacity"] * o * (1 - o), "logit", ex, g32["opacity"] * o * (1 - o))
    assert_grad_close(params["sh"].grad.cpu().numpy(), ref["sh"], sens["sh"], "sh", ex, g32["sh"])


def test_backward_of_an_overwritten_forward_raises():
    """Two forwards on one RenderContext share its buffers: the first graph's
    backward must refuse (its records and checkpoints are the second's)."""
    import torch
    from paper_2410_16978_amd import autograd as ag
    sc, cams, vss, Gr, Ga = _case(seed=15, D=1)
    params = {k: torch.tensor(sc[k], device="cuda", requires_grad=True)
              for k in ("mean", "log_scale", "quat", "opacity_logit", "sh")}
    layer = torch.tensor(sc["layer"], device="cuda")
    rctx = ag.RenderContext()
    rgb1, _ = ag.render_params(params, layer, 1, cams, vss, rctx)
    rgb2, _ = ag.render_params(params, layer, 1, cams, vss, rctx)
    with pytest.raises(RuntimeError, match="overwritten"):
        rgb1.sum().backward()
    rgb2.sum().backward()  # the latest forward's backward is fine
    torch.cuda.synchronize()
    assert torch.isfinite(params["mean"].grad).all()


def test_gradients_with_layer_fading(orc):
    sc, cams, _, Gr, Ga = _case(seed=21, D=2, n_views=2)
    vss = [scenes.view_state(0b111, clips=[([0.2, 0.1, 1.0], 0.3, 0b1)], bg=(0.2, 0.3, 0.1),
                             layer_opacity=[0.4, 1.0, 0.7]),
           scenes.view_state(0b111, bg=(0.2, 0.3, 0.1), layer_opacity=[1.0, 0.25, 0.9])]
    got = _gpu_grads(sc, cams, vss, Gr, Ga)
    ref, sens, g32, ex = _refs(orc, sc, cams, vss, Gr, Ga, got, label="fading")
    for k in ("mean", "scale", "quat", "opacity", "sh", "activity"):
        assert_grad_close(got[k], ref[k], sens[k], k, ex, g32[k])
    np.testing.assert_allclose(got["max_contrib"][~ex], ref["max_contrib"][~ex], rtol=1e-4, atol=1e-7)


def test_density_control_statistic_matches_oracle(orc):
    """The backward's density-control accumulators (gsr_grads.densify_*):
    counts exact (visibility is decided by the bit-exact records), sums of
    the centre's NDC gradient lengths under the gradient bar; accumulation
    over two calls doubles them; frozen layers untouched."""
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc, cams, vss, Gr, Ga = _case(seed=23, D=1, n_views=2)
    model = rz.to_device(sc)
    rgb, alpha, st = rz.rasterize_forward(model, cams, vss)
    n = sc["mean"].shape[1]
    dg = torch.zeros(n, device="cuda")
    dc = torch.zeros(n, device="cuda")
    for _ in range(2):
        rz.rasterize_backward(model, cams, vss, st, torch.as_tensor(Gr).cuda(), torch.as_tensor(Ga).cuda(),
                              trainable=0b110, densify=(dg, dc))
    torch.cuda.synchronize()
    got_g, got_c = dg.cpu().numpy() / 2, dc.cpu().numpy() / 2
    ref, sens, g32 = grad_refs(orc, sc, cams, vss, Gr, Ga, trainable=0b110)
    frozen = sc["layer"] == 0
    assert np.all(dg.cpu().numpy()[frozen] == 0) and np.all(dc.cpu().numpy()[frozen] == 0)
    np.testing.assert_array_equal(got_c, ref["densify_count"])
    assert got_c.max() == 2 and (got_c > 0).sum() > 100
    last = st.last.cpu().numpy().view(np.uint32)
    ex = checked_exempt(orc, sc, cams, vss, rgb.cpu().numpy(), alpha.cpu().numpy(), last, st.final_T.cpu().numpy(),
                        "densify")
    assert_grad_close(got_g, ref["densify_grad"], sens["densify_grad"], "densify_grad", ex, g32["densify_grad"])


def test_gradients_of_large_splats_with_long_pair_lists(orc):
    """Splats covering dozens of tiles (up to 72 pairs per record, each
    record's pair partials summed over a long list): gradients match and stay
    bitwise reproducible."""
    sc = scenes.shell_scene(120, 3, 2, seed=33, log_scale_mu=-2.3, log_scale_sigma=0.5, opacity="normal")
    cams = [scenes.orbit_camera([0.3, 0.2, -1.0], 256, 192), scenes.orbit_camera([-0.4, 0.3, -1.0], 256, 192)]
    scenes.enforce_distinct_depths(sc, cams)
    vss = [scenes.view_state(0b111, bg=(0.2, 0.3, 0.1))] * 2
    rng = np.random.default_rng(33)
    Gr = rng.standard_normal((2, 3, 192, 256)).astype(np.float32)
    Ga = rng.standard_normal((2, 192, 256)).astype(np.float32)
    nt = orc.render(sc, cams, vss)["n_tiles"]
    assert (nt >= 18).sum() > 50 and nt.max() > 64  # many split records, some past a full wave
    got = _gpu_grads(sc, cams, vss, Gr, Ga)
    again = _gpu_grads(sc, cams, vss, Gr, Ga)
    for k in ("mean", "scale", "quat", "opacity", "sh", "max_contrib"):
        np.testing.assert_array_equal(got[k], again[k])
    ref, sens, g32 = grad_refs(orc, sc, cams, vss, Gr, Ga)
    # a large splat's 1/255 boundary crosses many pixels, so more records than
    # in the other scenes have a decision within rounding of its threshold in
    # the oracle itself (8 of 360): the exemption's cap is 3 % here.  Other
    # seeds of this recipe: 31 leaves one SH entry at 1.08 x the plain bar
    # (inside the sensitivity bar; the float32 oracle has none there), 32 has
    # one pixel decided the other way whose tile list exempts 155 Gaussians
    ex = checked_exempt(orc, sc, cams, vss, got["rgb"], got["alpha"], got["last"], got["final_T"], "large splats",
                        cap=0.03)
    for k in ("mean", "scale", "quat", "opacity", "sh", "activity"):
        assert_grad_close(got[k], ref[k], sens[k], k, ex, g32[k])
    np.testing.assert_allclose(got["max_contrib"][~ex], ref["max_contrib"][~ex], rtol=1e-4, atol=1e-7)


def test_gradients_through_dense_tiles(orc):
    """Tiles of up to about 2900 pairs (a dozen batches, most of them past
    the pixels' stops): gradients within the bar, bitwise reproducible."""
    sc = scenes.shell_scene(1000, 3, 1, seed=41, log_scale_mu=-2.8, log_scale_sigma=0.4, opacity="normal")
    cams = [scenes.orbit_camera([0.2, 0.3, -1.0], 48, 40), scenes.orbit_camera([-0.1, 0.35, -1.0], 48, 40)]
    scenes.enforce_distinct_depths(sc, cams)
    vss = [scenes.view_state(bg=(0.2, 0.1, 0.3))] * 2
    rng = np.random.default_rng(41)
    Gr = rng.standard_normal((2, 3, 40, 48)).astype(np.float32)
    Ga = rng.standard_normal((2, 40, 48)).astype(np.float32)
    got = _gpu_grads(sc, cams, vss, Gr, Ga)
    again = _gpu_grads(sc, cams, vss, Gr, Ga)
    for k in ("mean", "scale", "quat", "opacity", "sh", "max_contrib"):
        np.testing.assert_array_equal(got[k], again[k])
    ref, sens, g32, ex = _refs(orc, sc, cams, vss, Gr, Ga, got, label="dense tiles")
    for k in ("mean", "scale", "quat", "opacity", "sh", "activity"):
        assert_grad_close(got[k], ref[k], sens[k], k, ex, g32[k])
    np.testing.assert_allclose(got["max_contrib"][~ex], ref["max_contrib"][~ex], rtol=1e-4, atol=1e-7)


def test_gradients_at_batch_boundaries(orc):
    """One 16 x 16 tile of exactly N pairs around the 256-pair batches:
    faint splats (every batch has live pixels, the last one partial) and
    opaque wide ones (every pixel stops in the first batch, the later
    batches have no work).  Gradients within the bar."""
    from tests.helpers import axis_camera, make_scene
    cam = axis_camera(16, 16, f=20.0, cx=8.0, cy=8.0)
    vss = [scenes.view_state(bg=(0.2, 0.1, 0.3))]
    for n in (256, 257, 513):
        for label, op_lo, op_hi, log_s in (("faint", 0.005, 0.02, -3.5), ("opaque", 0.95, 0.99, -0.5)):
            rng = np.random.default_rng(100 + n)
            z = rng.uniform(2.0, 4.0, n)
            xy = rng.uniform(-0.1, 0.1, (n, 2)) * z[:, None]
            sc = make_scene(np.column_stack([xy, z]), np.exp(rng.normal(log_s, 0.2, (n, 3))),
                            quats=rng.standard_normal((n, 4)), opacity=rng.uniform(op_lo, op_hi, n),
                            rgb=rng.uniform(0, 1, (n, 3)))
            scenes.enforce_distinct_depths(sc, [cam])
            Gr = rng.standard_normal((1, 3, 16, 16)).astype(np.float32)
            Ga = rng.standard_normal((1, 16, 16)).astype(np.float32)
            got = _gpu_grads(sc, [cam], vss, Gr, Ga)
            ref, sens, g32, ex = _refs(orc, sc, [cam], vss, Gr, Ga, got, label=f"{label} {n}")
            for k in ("mean", "scale", "quat", "opacity", "sh", "activity"):
                assert_grad_close(got[k], ref[k], sens[k], k, ex, g32[k])
