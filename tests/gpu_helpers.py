"""Comparison helpers of the GPU parity tests (HIP path through the C ABI vs
the CPU oracle)."""
import numpy as np
import torch

IMAGE_TOL = 1e-4  # max-abs on images, FP32


def gpu_forward(scene, cams, views, debug=True, capacity=None):
    from paper_2410_16978_amd import rasterizer as rz
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


def compare_forward(scene, cams, views, orc, check_pairs=True, label=""):
    """Run both paths and assert the parity bar; returns a stats dict."""
    model, (rgb, alpha, st, dbg) = gpu_forward(scene, cams, views)
    ref = orc.render(scene, cams, views, pairs=check_pairs, n_threads=0)
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
        np.testing.assert_array_equal(ke, ref["keys_emit"], err_msg=f"{label} emitted keys")
        np.testing.assert_array_equal(ve, ref["vals_emit"], err_msg=f"{label} emitted values")
        ks = dbg["keys_sorted"].cpu().numpy().view(np.uint64)[:K]
        np.testing.assert_array_equal(ks, ref["keys"], err_msg=f"{label} sorted keys")
        sel = int(st.sort_sel.item())
        vs_ = st.pair_vals.cpu().numpy().view(np.uint32)[sel * st.capacity: sel * st.capacity + K]
        np.testing.assert_array_equal(vs_, ref["vals"], err_msg=f"{label} sorted values")
        rg = st.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)[:len(ref["ranges"])]
        np.testing.assert_array_equal(rg, ref["ranges"], err_msg=f"{label} tile ranges")
    # images: max-abs <= 1e-4 away from threshold-near pixels
    flag = ref["margin"] < 1.0
    g_rgb = rgb.cpu().numpy()
    g_alpha = alpha.cpu().numpy()
    ok = ~flag
    err_rgb = np.abs(g_rgb - ref["rgb"]).max(axis=1)
    err_a = np.abs(g_alpha - ref["alpha"])
    max_err = max(float(err_rgb[ok].max(initial=0)), float(err_a[ok].max(initial=0)))
    assert max_err <= IMAGE_TOL, f"{label} image max-abs {max_err}"
    last = st.last.cpu().numpy().view(np.uint32).reshape(V, H, W)
    mism_last = int(((last != ref["last"]) & ok).sum())
    assert mism_last == 0, f"{label} last index differs on {mism_last} pixels"
    n_flag = int(flag.sum())
    assert n_flag <= max(2, 1e-3 * flag.size), f"{label} too many threshold-near pixels {n_flag}"
    return {"max_err": max_err, "flagged": n_flag, "K": K, "pixels": int(flag.size),
            "max_err_all": max(float(err_rgb.max()), float(err_a.max()))}
