"""Comparison helpers of the GPU parity tests (HIP path through the C ABI vs
the CPU oracle)."""
import numpy as np
import torch

IMAGE_TOL = 1e-4  # max-abs on images, FP32
GRAD_RTOL = 1e-3  # relative error of gradients


def gpu_forward(scene, cams, views, debug=True, capacity=None, model=None):
    """model (optional): a device model to render instead of scene's."""
    from paper_2410_16978_amd import rasterizer as rz
    if model is None:
        model = rz.to_device(scene)
    res = rz.rasterize_forward(model, cams, views, debug=debug, capacity=capacity)
    torch.cuda.synchronize()
    return model, res


def oracle_rect_to_box(rect, depth, tile_off, tiles_x):
    x0, y0, x1, y1 = (rect[:, k].astype(np.int64) for k in range(4))
    base = tile_off + y0 * tiles_x + x0
    wh = (x1 - x0) | ((y1 - y0) << 16)
    return np.stack([base, wh, depth.astype(np.float32).view(np.uint32).astype(np.int64),
                     np.full_like(base, tiles_x)], 1).astype(np.uint32)


def compare_forward(scene, cams, views, orc, check_pairs=True, label="", max_flagged=None, device_model=None):
    """Run both paths and assert the parity bar; returns a stats dict.  With
    a shared depth order (views[0]["sort_cam"]) the oracle sorts every view
    by the depth in that camera and the emission order differs by design
    (the GPU emits each view's pairs in the sorted Gaussian order), so the
    emitted keys are compared as multisets.  device_model (optional): the
    device model the GPU renders (a compressed one, whose decoded scene is
    `scene`)."""
    model, (rgb, alpha, st, dbg) = gpu_forward(scene, cams, views, model=device_model)
    sort_cam = views[0].get("sort_cam")
    ref = orc.render(scene, cams, views, pairs=check_pairs, n_threads=0,
                     sort_cams=None if sort_cam is None else [sort_cam] * len(cams))
    V = len(cams)
    n = scene["mean"].shape[1]
    R = n * V
    # per-record tile counts: bit-exact
    n_tiles = dbg["n_tiles"].cpu().numpy().view(np.uint32)[:R]
    np.testing.assert_array_equal(n_tiles, ref["n_tiles"], err_msg=f"{label} n_tiles")
    valid = ref["n_tiles"] > 0
    # records of surviving Gaussians: bit-exact
    rec = st.records.view(-1, 12).cpu().numpy()[:R]
    got = rec[valid][:, [0, 1, 2, 3, 4, 5, 9, 6, 7, 8]]  # u v a b c o depth r g b
    want = ref["rec"][valid]
    diff = got.view(np.int32).astype(np.int64) - want.astype(np.float32).view(np.int32).astype(np.int64)
    if np.any(diff):
        names = "u v conic_a conic_b conic_c opacity depth r g b".split()
        for c in range(10):
            bad = np.nonzero(diff[:, c])[0]
            if len(bad):
                print(f"{label} record field {names[c]}: {len(bad)} differ, max ulps {np.abs(diff[:, c]).max()}, "
                      f"e.g. gpu {got[bad[0], c]!r} oracle {want[bad[0], c]!r}")
    np.testing.assert_array_equal(got.view(np.uint32), want.astype(np.float32).view(np.uint32),
                                  err_msg=f"{label} records")
    np.testing.assert_array_equal(rec[valid][:, 10].view(np.uint32), ref["clamp"][valid], err_msg=f"{label} clamp")
    # tile boxes: bit-exact
    W, H = cams[0]["width"], cams[0]["height"]
    tiles_x = (W + 15) // 16
    tpv = tiles_x * ((H + 15) // 16)
    tb = dbg["tile_box"].cpu().numpy().view(np.uint32)[:R]
    view_of = np.repeat(np.arange(V), n)
    want_tb = oracle_rect_to_box(ref["rect"], ref["rec"][:, 6], view_of * tpv, tiles_x)
    np.testing.assert_array_equal(tb[valid], want_tb[valid], err_msg=f"{label} tile boxes")
    K = ref["counts"]["K"]
    assert st.n_pairs == K, f"{label} pair count {st.n_pairs} vs {K}"
    if check_pairs:
        ke = dbg["keys_emit"].cpu().numpy().view(np.uint64)[:K]
        ve = dbg["vals_emit"].cpu().numpy().view(np.uint32)[:K]
        if sort_cam is None:
            np.testing.assert_array_equal(ke, ref["keys_emit"], err_msg=f"{label} emitted keys")
            np.testing.assert_array_equal(ve, ref["vals_emit"], err_msg=f"{label} emitted values")
        else:
            order_g, order_o = np.lexsort((ve, ke)), np.lexsort((ref["vals_emit"], ref["keys_emit"]))
            np.testing.assert_array_equal(ke[order_g], ref["keys_emit"][order_o], err_msg=f"{label} emitted keys")
            np.testing.assert_array_equal(ve[order_g], ref["vals_emit"][order_o], err_msg=f"{label} emitted values")
        ks = dbg["keys_sorted"].cpu().numpy().view(np.uint64)[:K]
        np.testing.assert_array_equal(ks, ref["keys"], err_msg=f"{label} sorted keys")
        sel = int(st.sort_sel.item())
        vs_ = st.pair_vals.cpu().numpy().view(np.uint32)[sel * st.capacity: sel * st.capacity + K]
        np.testing.assert_array_equal(vs_, ref["vals"], err_msg=f"{label} sorted values")
        rg = st.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)[:len(ref["ranges"])]
        np.testing.assert_array_equal(rg, ref["ranges"], err_msg=f"{label} tile ranges")
    last = st.last.cpu().numpy().view(np.uint32).reshape(V, H, W)
    stats = assert_images(rgb, alpha, ref, label, last=last, max_flagged=max_flagged)
    stats["K"] = K
    return stats


def assert_images(rgb, alpha, ref, label="", last=None, max_flagged=None):
    """Images within IMAGE_TOL max-abs on every pixel whose oracle decision
    margin is >= 1 (no threshold within the rounding tolerance); at most
    max_flagged pixels may be flagged (default max(2, 1e-3 * pixels); the
    full-size tests pass the count measured for their scene, the oracle's
    margins being deterministic).  `last` (optional) must equal the oracle's
    last blended index on the unflagged pixels."""
    flag = ref["margin"] < 1.0
    g_rgb = rgb.cpu().numpy() if hasattr(rgb, "cpu") else np.asarray(rgb)
    g_alpha = alpha.cpu().numpy() if hasattr(alpha, "cpu") else np.asarray(alpha)
    ok = ~flag
    err_rgb = np.abs(g_rgb - ref["rgb"]).max(axis=1)
    err_a = np.abs(g_alpha - ref["alpha"])
    max_err = max(float(err_rgb[ok].max(initial=0)), float(err_a[ok].max(initial=0)))
    assert max_err <= IMAGE_TOL, f"{label} image max-abs {max_err}"
    if last is not None:
        mism_last = int(((last != ref["last"]) & ok).sum())
        assert mism_last == 0, f"{label} last index differs on {mism_last} pixels"
    n_flag = int(flag.sum())
    cap = max(2, 1e-3 * flag.size) if max_flagged is None else max_flagged
    assert n_flag <= cap, f"{label} too many threshold-near pixels {n_flag} (cap {cap})"
    return {"max_err": max_err, "flagged": n_flag, "pixels": int(flag.size),
            "max_err_all": max(float(err_rgb.max()), float(err_a.max()))}


SENS_K = 4.0  # multiple of an entry's float32 sensitivity allowed beyond the plain bar
EXTRA_FLOOR_FRACTION = 1e-5  # plain-bar misses allowed beyond the float32 oracle's own count
U32 = 2.0 ** -24  # unit roundoff of float32


def grad_refs(orc, scene, cams, views, Gr, Ga, trainable=0xFFFFFFFF):
    """Reference gradient, per-entry float32 sensitivity and the float32
    oracle's gradient.

    ref: the float32 forward's gradient evaluated in float64 (oracle dtype
    "exact": the same records, pair lists and per-pixel decisions as the
    GPU's float32 forward; the chain rule differentiates the projection at
    the parameters in float64).
    sens: the larger of (a) how far the same float64 arithmetic lands when
    fed with the float32 forward's own per-pixel offsets, G, alpha and
    transmittances ("exact_fwd_values") and (b) 2^-24 times the entry's
    condition (oracle "cond": the depth-weighted magnitude sum of its
    per-pixel terms; float32 per-pixel arithmetic errs by a small multiple of
    it).  Both are large only where an entry is a near-cancellation of
    per-pixel terms.
    g32: the float32 oracle (its count of plain-bar misses is the yardstick
    of what a float32 evaluation achieves).  Also returns the exact
    max_contrib and activity."""
    ex = orc.backward(scene, cams, views, Gr, Ga, trainable=trainable, dtype="exact", cond=True)
    fv = orc.backward(scene, cams, views, Gr, Ga, trainable=trainable, dtype="exact_fwd_values")
    g32 = orc.backward(scene, cams, views, Gr, Ga, trainable=trainable, dtype=np.float32)
    keys = ("mean", "scale", "quat", "opacity", "sh")
    sens = {k: np.maximum(np.abs(ex[k] - fv[k]), U32 * ex["cond"][k]) for k in keys}
    # activity = 2 |g_mean| + 0.1 |g_sh| + 0.1 |g_log s|: its sensitivity from
    # the parts' (triangle inequality), plus the float32 forward values' own
    n = ex["opacity"].shape[-1]
    s = np.asarray(scene["scale"], np.float64)
    sens["activity"] = np.maximum(
        np.abs(ex["activity"] - fv["activity"]),
        2.0 * np.linalg.norm(sens["mean"].reshape(-1, n), axis=0)
        + 0.1 * np.linalg.norm(sens["sh"].reshape(-1, n), axis=0)
        + 0.1 * np.linalg.norm((sens["scale"] * s).reshape(-1, n), axis=0))
    # density-control statistic: a sum of norms of the centre's 2D gradient;
    # its sensitivity from the float32 forward values
    sens["densify_grad"] = np.abs(ex["densify_grad"] - fv["densify_grad"])
    ref = {k: ex[k] for k in keys + ("activity", "max_contrib", "densify_grad", "densify_count")}
    return ref, sens, {k: g32[k].astype(np.float64) for k in keys + ("activity", "densify_grad")}


def assert_grad_close(got, ref, sens, name, exempt=None, ref32=None):
    """Gradient parity bar, per entry against the exact reference (grad_refs):

        |got - ref| <= 1e-3 * max(|ref|, 1e-3 * RMS(ref)) + SENS_K * sens.

    The first term is the plain relative bar; the second admits entries that
    float32 arithmetic cannot pin to it (near-cancellations: the float32
    oracle misses the plain bar on about 1e-4 of the entries of the
    200k-Gaussian step).  The entries that miss the plain bar are counted,
    printed and limited to the float32 oracle's own count (ref32, same
    entries) plus EXTRA_FLOOR_FRACTION of the entries (without ref32: that
    fraction alone).  `exempt` (bool [n], last axis) excludes Gaussians on
    pixels where a threshold decision went the other way (flip_exempt).
    Returns the number of plain-bar misses."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    sens = np.asarray(sens, np.float64)
    keep = np.arange(got.shape[-1])
    if exempt is not None:
        got, ref, sens = got[..., ~exempt], ref[..., ~exempt], sens[..., ~exempt]
        keep = keep[~exempt]
        ref32 = None if ref32 is None else np.asarray(ref32, np.float64)[..., ~exempt]
    rms = float(np.sqrt(np.mean(ref ** 2))) if ref.size else 0.0
    plain = GRAD_RTOL * np.maximum(np.abs(ref), 1e-3 * rms)
    err = np.abs(got - ref)
    tol = plain + SENS_K * sens
    bad = err > tol
    misses = int((err > plain).sum())
    misses32 = int((np.abs(np.asarray(ref32) - ref) > plain).sum()) if ref32 is not None else 0
    if bad.any():
        for w in np.argsort(-(err - tol).ravel())[:5]:
            ix = np.unravel_index(w, err.shape)
            print(f"{name}[{', '.join(str(int(v)) for v in ix[:-1] + (keep[ix[-1]],))}]: got {float(got[ix])!r} "
                  f"ref {float(ref[ix])!r} plain {float(plain[ix])!r} sens {float(sens[ix])!r}")
    worst = float(np.max(err / np.maximum(plain, 1e-300))) if err.size else 0.0
    print(f"{name}: {err.size} entries, worst err / plain bar {worst:.3f}, {misses} beyond the plain bar "
          f"(float32 oracle: {misses32 if ref32 is not None else '-'})", flush=True)
    assert not bad.any(), (f"{name}: {int(bad.sum())}/{bad.size} outside the bar; worst err/tol "
                           f"{float(np.max(err / tol))}")
    cap = misses32 + EXTRA_FLOOR_FRACTION * err.size
    assert misses <= cap, f"{name}: {misses} of {err.size} entries beyond the plain bar (cap {cap:.1f})"
    return misses


def checked_exempt(orc, scene, cams, views, rgb, alpha, last, final_T, label="", cap=0.01, max_flagged=None):
    """Forward parity first (images and last index on the unflagged pixels,
    see assert_images), then the flip exemption, capped at max(2, cap * n)
    Gaussians."""
    ref_fwd = orc.render(scene, cams, views, pairs=True)
    assert_images(rgb, alpha, ref_fwd, label, last=np.asarray(last).reshape(ref_fwd["last"].shape),
                  max_flagged=max_flagged)
    n = scene["mean"].shape[1]
    ex = flip_exempt(ref_fwd, n, last, final_T)
    print(f"{label} exempt Gaussians: {int(ex.sum())} of {n}", flush=True)
    assert ex.sum() <= max(2, cap * n), f"{label} {int(ex.sum())} exempt Gaussians"
    return ex


def flip_exempt(ref_fwd, n, last_gpu=None, T_gpu=None):
    """Gaussians whose gradient may legitimately differ because a threshold
    decision (sign of q, alpha vs 1/255, T vs 1e-4) lies within the rounding
    tolerance: the records with such a decision (the oracle's near_rec), and
    every pair evaluated up to the last blended one on a pixel where the GPU
    did decide otherwise — its last blended pair differs from the oracle's, or
    its final transmittance differs by more than 1e-3 relative (a flipped
    pair changes T by at least 1/255, rounding by far less).  Needs the
    oracle forward with pairs=True.  Returns a bool mask [n]."""
    ex = np.zeros(n, bool)
    ex[np.nonzero(ref_fwd["near_rec"])[0] % n] = True
    if last_gpu is None:
        return ex
    lo_o = ref_fwd["last"].astype(np.int64)
    lo_g = np.asarray(last_gpu).astype(np.int64).reshape(lo_o.shape)
    flipped = lo_o != lo_g
    if T_gpu is not None:
        To = ref_fwd["final_T"].astype(np.float64)
        Tg = np.asarray(T_gpu, np.float64).reshape(To.shape)
        flipped |= np.abs(Tg - To) > 1e-3 * To
    V, H, W = lo_o.shape
    tx = (W + 15) // 16
    tpv = tx * ((H + 15) // 16)
    ranges = ref_fwd["ranges"].astype(np.int64)
    vals = ref_fwd["vals"].astype(np.int64)
    for v, y, x in zip(*np.nonzero(flipped)):
        t = v * tpv + (y // 16) * tx + x // 16
        s0, e0 = ranges[t]
        stop = min(max(int(lo_o[v, y, x]), int(lo_g[v, y, x])) + 1, e0)
        ex[vals[s0:stop] % n] = True
    return ex
