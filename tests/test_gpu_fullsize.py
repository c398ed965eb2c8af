"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times.

* 200k-Gaussian training step (4 shells, SH3, 800x800): records, keys, sorted
  pairs and ranges bit-exact, images within 1e-4; the backward through the
  autograd wrapper with a pre-sized state and no host synchronisation,
  against the oracle's exact gradient of the same float32 forward on every
  Gaussian; the float64 oracle and the GPU gradient against central
  differences on 32 sampled parameters (4 each of mean, log-scale,
  quaternion, opacity logit, SH bands 0-3).
* 1M-Gaussian layered stereo frame (5 shells, two 1832x1920 eyes, random
  layer mask and clip planes): bit-exact pairs, images within 1e-4.
* Serving: three requests (512^2, 1024^2, stereo 1832x1920) on the 500k and
  2M resident models in one render_batch launch, each image against the
  oracle.
"""
import numpy as np
import pytest

from paper_2410_16978_amd import scenes
from tests.gpu_helpers import SENS_K, assert_grad_close, assert_images, checked_exempt, compare_forward, grad_refs

pytestmark = pytest.mark.gpu

# threshold-near pixels (oracle decision margin < 1), measured on these
# scenes (the oracle's margins are deterministic): the image bar holds on
# every other pixel, and no more pixels than these may be flagged
C2_FLAGGED = 183
STEREO_1M_FLAGGED = 2033


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_16978_amd import rasterizer
    rasterizer.lib()


@pytest.fixture(scope="module")
def c2():
    return scenes.training_step_200k(seed=0)


def test_training_step_200k_forward(c2, orc):
    st = compare_forward(c2.scene, c2.cams, c2.views, orc, label="200k", max_flagged=C2_FLAGGED)
    print("200k forward:", st, flush=True)


def _raw_to_scene64(raw, layer, D):
    """Activated float64 scene from raw parameters (exp of log-scales,
    logistic function of logits)."""
    return {"mean": raw["mean"], "scale": np.exp(raw["log_scale"]), "quat": raw["quat"],
            "opacity": 1.0 / (1.0 + np.exp(-raw["opacity_logit"])), "sh": raw["sh"], "layer": layer,
            "sh_degree": D}


KEYS = ("mean", "log_scale", "quat", "opacity_logit", "sh")
SRC = {"mean": "mean", "log_scale": "scale", "quat": "quat", "opacity_logit": "opacity", "sh": "sh"}


@pytest.fixture(scope="module")
def c2_grads(c2, orc):
    """GPU gradients of L = sum(rgb * Gr) + sum(alpha * Ga) with respect to the
    raw parameters, through the autograd wrapper with the pair buffers sized
    once and no host synchronisation (as the benchmark runs it), and the
    oracle's exact gradient with its float32 sensitivity, chained to the raw
    parameters."""
    import torch
    from paper_2410_16978_amd import autograd as ag
    from paper_2410_16978_amd import rasterizer as rz
    sc, cams, vss = c2.scene, c2.cams, c2.views
    n, D = sc["mean"].shape[1], sc["sh_degree"]
    W, H = cams[0]["width"], cams[0]["height"]
    rng = np.random.default_rng(5)
    Gr = rng.standard_normal((1, 3, H, W)).astype(np.float32)
    Ga = rng.standard_normal((1, H, W)).astype(np.float32)
    params = {k: torch.tensor(sc[k], device="cuda", requires_grad=True) for k in KEYS}
    layer = torch.tensor(sc["layer"], device="cuda")
    Gr_t, Ga_t = torch.tensor(Gr, device="cuda"), torch.tensor(Ga, device="cuda")
    rctx = ag.RenderContext(sync=True, track_activity=True)
    with torch.no_grad():
        ag.render_params(params, layer, D, cams, vss, rctx)
    torch.cuda.synchronize()
    rctx.state = rz.make_state(n, 1, W, H, int(rctx.state.n_pairs * 1.25) + 4096)
    rctx.sync = False
    rgb, alpha = ag.render_params(params, layer, D, cams, vss, rctx)
    ((rgb * Gr_t).sum() + (alpha * Ga_t).sum()).backward()
    torch.cuda.synchronize()
    rz.forward_check(rctx.state)
    got = {k: params[k].grad.cpu().numpy() for k in KEYS}
    # the oracle takes the activations exactly as the kernels computed them
    act = dict(sc)
    sc_t, op_t = rz.activate({"mean": params["mean"].detach(), "scale": params["log_scale"].detach(),
                              "quat": params["quat"].detach(), "opacity": params["opacity_logit"].detach(),
                              "sh": params["sh"].detach(), "layer": layer, "sh_degree": sc["sh_degree"],
                              "raw": True})
    act["scale"] = sc_t.cpu().numpy()
    act["opacity"] = op_t.cpu().numpy()
    ref, sens, g32 = grad_refs(orc, act, cams, vss, Gr, Ga)
    o = act["opacity"].astype(np.float64)
    chain = {"mean": 1.0, "log_scale": act["scale"].astype(np.float64), "quat": 1.0,
             "opacity_logit": o * (1 - o), "sh": 1.0}
    st = rctx.state
    ex = checked_exempt(orc, act, cams, vss, rgb.detach(), alpha.detach(), st.last.cpu().numpy().view(np.uint32),
                        st.final_T.cpu().numpy(), "200k step", max_flagged=C2_FLAGGED)
    return {"Gr": Gr, "Ga": Ga, "got": got, "max_contrib": rctx.max_contrib.cpu().numpy(), "exempt": ex,
            "ref": {k: ref[SRC[k]] * chain[k] for k in KEYS},
            "sens": {k: sens[SRC[k]] * chain[k] for k in KEYS},
            "ref32": {k: g32[SRC[k]] * chain[k] for k in KEYS},
            "ref_max_contrib": ref["max_contrib"]}


def test_training_step_200k_backward(c2, c2_grads):
    """Every Gaussian's gradient within the bar, except those on pixels where
    a threshold decision went the other way (see flip_exempt, at most 1 % of
    the Gaussians)."""
    g = c2_grads
    ex = g["exempt"]
    for k in KEYS:
        assert_grad_close(g["got"][k], g["ref"][k], g["sens"][k], k, ex, g["ref32"][k])
    np.testing.assert_allclose(g["max_contrib"][~ex], g["ref_max_contrib"][~ex], rtol=1e-4, atol=1e-7)


def test_training_step_200k_central_differences(c2, c2_grads, orc):
    """Central differences of the float64 oracle render on 32 parameters (4 of
    each of mean, log-scale, quaternion, opacity logit and SH bands 0-3) of
    Gaussians with max alpha*T > 0.05: step 1e-6 max(1, |theta|); a parameter
    whose h and h/2 estimates disagree (a pixel decision flips inside the
    step) is replaced by the next candidate.  The float64 oracle gradient
    must agree to 1e-3; the GPU gradient to 1e-3 plus its bar against the
    exact gradient of its float32 forward."""
    sc, cams, vss = c2.scene, c2.cams, c2.views
    D = sc["sh_degree"]
    g = c2_grads
    raw64 = {k: sc[k].astype(np.float64) for k in KEYS}
    G64, GA64 = g["Gr"].astype(np.float64), g["Ga"].astype(np.float64)

    def loss(r):
        out = orc.render(_raw_to_scene64(r, sc["layer"], D), cams, vss, pairs=False, dtype=np.float64)
        return float((out["rgb"] * G64).sum() + (out["alpha"] * GA64).sum())

    rng = np.random.default_rng(6)
    cand = rng.permutation(np.nonzero(g["max_contrib"] > 0.05)[0])
    groups = [("mean", lambda i, c: (c % 3, i)), ("log_scale", lambda i, c: (c % 3, i)),
              ("quat", lambda i, c: (c % 4, i)), ("opacity_logit", lambda i, c: (i,))]
    groups += [("sh", (lambda b: lambda i, c: (b * b + c % (2 * b + 1), c % 3, i))(b)) for b in range(4)]
    checked = 0
    for gi, (k, index) in enumerate(groups):
        rms = float(np.sqrt(np.mean(g["ref"][k] ** 2)))
        done = 0
        for j, i in enumerate(cand[gi * 40:(gi + 1) * 40]):
            idx = index(int(i), j)
            th = raw64[k][idx]
            h = 1e-6 * max(1.0, abs(th))

            def fd(step):
                raw64[k][idx] = th + step
                lp = loss(raw64)
                raw64[k][idx] = th - step
                lm = loss(raw64)
                raw64[k][idx] = th
                return (lp - lm) / (2 * step)

            f1, f2 = fd(h), fd(h / 2)
            if abs(f1 - f2) > 2e-4 * max(abs(f1), abs(f2), 1e-3 * rms):
                continue
            fdv = (4 * f2 - f1) / 3
            scale = max(abs(fdv), 1e-3 * rms)
            an = float(g["ref"][k][idx])
            assert abs(an - fdv) <= 1e-3 * scale, (k, idx, "oracle", an, fdv)
            gpu = float(g["got"][k][idx])
            # the GPU within its bar of the exact gradient of its float32
            # forward, which is within 1e-3 of the differences (above)
            tol = 1e-3 * scale + 1e-3 * max(abs(an), 1e-3 * rms) + SENS_K * float(g["sens"][k][idx])
            assert abs(gpu - fdv) <= tol, (k, idx, "gpu", gpu, fdv)
            done += 1
            checked += 1
            if done == 4:
                break
        assert done == 4, f"{k}: only {done} parameters with a smooth loss"
    assert checked == 32


def test_layered_stereo_1m(orc):
    w = scenes.layered_stereo()
    st = compare_forward(w.scene, w.cams, w.views, orc, label="stereo 1M", max_flagged=STEREO_1M_FLAGGED)
    print("stereo 1M:", st, flush=True)


def test_serving_requests_full_models(orc):
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    models_np = scenes.serving_models()
    models = [rz.to_device(m) for m in models_np]
    rng = np.random.default_rng(11)
    reqs = []
    for m, (Wd, Ht, eyes) in ((0, (512, 512, 1)), (1, (1024, 1024, 1)), (0, (1832, 1920, 2))):
        d = scenes.random_direction(rng)
        cams = scenes.stereo_cameras(d, Wd, Ht) if eyes == 2 else [scenes.orbit_camera(d, Wd, Ht)]
        reqs.append({"model": m, "cams": cams, "view": scenes.random_view_state(rng, 5, bg=(0.1, 0.2, 0.3))})
    outs, status, _ = rz.render_batch(models, reqs, 16_000_000)
    torch.cuda.synchronize()
    assert [int(s) for s in status] == [0, 0, 0]
    for q, r in enumerate(reqs):
        ref = orc.render(models_np[r["model"]], r["cams"], [r["view"]] * len(r["cams"]), pairs=False)
        rgb = torch.stack(outs[q][0]).cpu().numpy()
        alpha = torch.stack(outs[q][1]).cpu().numpy()
        st = assert_images(rgb, alpha, ref, label=f"request {q}")
        print(f"request {q}:", st, flush=True)
