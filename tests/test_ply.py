"""Layered PLY assets (paper_2410_16978_amd/ply.py): the layer is a
per-Gaussian property of one PLY file (Sec. 3.2).  Round trip bit-exact,
the header's property list, the channel-major order of the higher SH
coefficients against a file assembled by hand, a missing layer property,
and a render of the read scene equal to the original's."""
import numpy as np
import pytest

from paper_2410_16978_amd import ply, scenes


@pytest.fixture
def scene():
    return scenes.shell_scene(300, 3, 2, seed=7)


def test_round_trip_is_bit_exact(tmp_path, scene):
    p = tmp_path / "m.ply"
    ply.write_ply(p, scene)
    back = ply.read_ply(p)
    assert back["sh_degree"] == scene["sh_degree"]
    for k in ("mean", "log_scale", "quat", "opacity_logit", "sh", "layer", "scale", "opacity"):
        np.testing.assert_array_equal(back[k], scene[k], err_msg=k)


def test_header_lists_the_properties(tmp_path, scene):
    p = tmp_path / "m.ply"
    ply.write_ply(p, scene)
    head = p.read_bytes().split(b"end_header\n")[0].decode().splitlines()
    assert head[:3] == ["ply", "format binary_little_endian 1.0", f"element vertex {scene['mean'].shape[1]}"]
    props = [ln.split()[-1] for ln in head if ln.startswith("property")]
    M = 8  # degree 2: 9 coefficients, 8 above the DC term
    assert props[:9] == ["x", "y", "z", "nx", "ny", "nz", "f_dc_0", "f_dc_1", "f_dc_2"]
    assert props[9:9 + 3 * M] == [f"f_rest_{i}" for i in range(3 * M)]
    assert props[9 + 3 * M:] == ["opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3",
                                 "layer"]
    assert head[3 + 9 + 3 * M + 8] == "property uchar layer"


def _hand_written(path, n, D, with_layer, rng):
    """A PLY assembled without ply.py: shuffled property order, a comment,
    an extra property; returns the values written."""
    M = (D + 1) ** 2 - 1
    names = ["x", "y", "z", "f_dc_0", "f_dc_1", "f_dc_2"] + [f"f_rest_{i}" for i in range(3 * M)]
    names += ["opacity", "scale_0", "scale_1", "scale_2", "rot_0", "rot_1", "rot_2", "rot_3", "extra"]
    order = rng.permutation(len(names))
    names = [names[i] for i in order]
    cols = {nm: rng.standard_normal(n).astype(np.float32) for nm in names}
    fields = [(nm, "<f4") for nm in names]
    if with_layer:
        cols["layer"] = rng.integers(0, 5, n).astype(np.uint8)
        fields.append(("layer", "u1"))
    arr = np.zeros(n, np.dtype(fields))
    for nm in cols:
        arr[nm] = cols[nm]
    head = ["ply", "format binary_little_endian 1.0", "comment hand-written", f"element vertex {n}"]
    head += [f"property float {nm}" for nm in names] + (["property uchar layer"] if with_layer else [])
    head += ["end_header"]
    with open(path, "wb") as f:
        f.write(("\n".join(head) + "\n").encode())
        f.write(arr.tobytes())
    return cols


@pytest.mark.parametrize("with_layer", [True, False])
def test_reads_a_hand_written_file(tmp_path, with_layer):
    rng = np.random.default_rng(3)
    n, D = 17, 3
    p = tmp_path / "h.ply"
    cols = _hand_written(p, n, D, with_layer, rng)
    sc = ply.read_ply(p)
    assert sc["sh_degree"] == 3
    np.testing.assert_array_equal(sc["mean"][1], cols["y"])
    # higher coefficients are channel-major: f_rest_{ch*15 + k-1} is coefficient k of channel ch
    for ch in range(3):
        np.testing.assert_array_equal(sc["sh"][0, ch], cols[f"f_dc_{ch}"])
        for k in (1, 7, 15):
            np.testing.assert_array_equal(sc["sh"][k, ch], cols[f"f_rest_{ch * 15 + k - 1}"])
    np.testing.assert_array_equal(sc["quat"][0], cols["rot_0"])
    np.testing.assert_array_equal(sc["log_scale"][2], cols["scale_2"])
    np.testing.assert_array_equal(sc["opacity_logit"], cols["opacity"])
    np.testing.assert_allclose(sc["opacity"], 1 / (1 + np.exp(-cols["opacity"].astype(np.float64))), rtol=1e-6)
    np.testing.assert_array_equal(sc["layer"], cols["layer"] if with_layer else np.zeros(n, np.uint8))


def test_rejects_other_formats(tmp_path):
    p = tmp_path / "a.ply"
    p.write_bytes(b"ply\nformat ascii 1.0\nelement vertex 0\nend_header\n")
    with pytest.raises(ValueError, match="binary_little_endian"):
        ply.read_ply(p)


def test_render_of_the_read_scene_equals_the_original(tmp_path, orc, scene):
    p = tmp_path / "m.ply"
    ply.write_ply(p, scene)
    back = ply.read_ply(p)
    cam = scenes.orbit_camera([0.3, 0.2, -1.0], 64, 48)
    vs = scenes.view_state(0b101)
    a = orc.render(scene, [cam], [vs], pairs=False)
    b = orc.render(back, [cam], [vs], pairs=False)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
