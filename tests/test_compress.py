"""Compressed attribute sets (Sec. 4.3 compression levels): the oracle's
decoding pinned to the IEEE half format and worked examples, and the
importer (compress.py) pinned to the definitions of its codes and of
K-means (CPU only)."""
import numpy as np
import pytest

from oracle import compressed as oc
from paper_2410_16978_amd import compress, scenes


def test_half_decoding_known_patterns():
    bits = np.array([0x3C00, 0xC000, 0x0001, 0x03FF, 0x7BFF, 0x8000, 0x3555, 0x7C00, 0x0400], np.uint16)
    v = oc.half_to_float(bits)
    assert v[0] == 1.0 and v[1] == -2.0
    assert v[2] == 2.0 ** -24 and v[3] == 1023 * 2.0 ** -24  # subnormals
    assert v[4] == 65504.0 and np.signbit(v[5]) and v[5] == 0
    assert v[6] == 0.333251953125 and np.isinf(v[7]) and v[8] == 2.0 ** -14


def test_packed_word_worked_example():
    """Codes r = 5, g = 1000, b = 1023 in one word: bits 0-10, 11-21, 22-31."""
    w = np.uint32(5 | (1000 << 11) | (1023 << 22))
    comp = {"format": "half_packed", "sh_degree": 1, "n": 1, "layer": np.zeros(1, np.uint8),
            "mean": np.zeros((3, 1), np.uint16), "scale": np.zeros((3, 1), np.uint16),
            "quat": np.zeros((4, 1), np.uint16), "opacity": np.zeros(1, np.uint16),
            "sh_dc": np.full((3, 1), 0x3C00, np.uint16), "sh_packed": np.full((3, 1), w, np.uint32),
            "sh_lo": np.array([-1.0, 0.5, 0.0], np.float32), "sh_step": np.array([2 ** -10, 2 ** -9, 0.25], np.float32)}
    sh = oc.decode(comp)["sh"]
    np.testing.assert_array_equal(sh[0, :, 0], [1.0, 1.0, 1.0])
    # every product and sum here is exact in float32
    np.testing.assert_array_equal(sh[1:, 0, 0], [-1 + 5 / 1024] * 3)
    np.testing.assert_array_equal(sh[1:, 1, 0], [0.5 + 1000 / 512] * 3)
    np.testing.assert_array_equal(sh[1:, 2, 0], [255.75] * 3)


def test_codebook_lookup_worked_example():
    """Two Gaussians, degree 1 (M = 3), entries of 16 halves holding [k][ch]
    in their first 9: Gaussian 0 takes entry 1, Gaussian 1 entry 0."""
    vals = np.arange(2 * 3 * 3, dtype=np.float32).reshape(2, 3, 3)
    cb = np.full((2, 16), 7777.0, np.float32)  # padding: never read
    cb[:, :9] = vals.reshape(2, 9)
    comp = {"format": "half_codebook", "sh_degree": 1, "n": 2, "layer": np.zeros(2, np.uint8),
            "mean": np.zeros((3, 2), np.uint16), "scale": np.zeros((3, 2), np.uint16),
            "quat": np.zeros((4, 2), np.uint16), "opacity": np.zeros(2, np.uint16),
            "sh_dc": np.zeros((3, 2), np.uint16), "sh_index": np.array([1, 0], np.uint16),
            "codebook": cb.astype(np.float16).view(np.uint16), "codebook_size": 2}
    sh = oc.decode(comp)["sh"]
    assert sh[2, 1, 0] == 9 + 1 * 3 + 1  # entry 1, k = 2 (row 1 of the entry), green
    assert sh[3, 2, 1] == 0 + 2 * 3 + 2  # entry 0, k = 3, blue
    np.testing.assert_array_equal(sh[1:, :, 0], vals[1])


@pytest.fixture(scope="module")
def shells():
    return scenes.shell_scene(600, 3, 3, seed=2, log_scale_mu=-3.5, opacity="normal")


def test_pack_codes_are_the_nearest_codes(shells):
    words, lo, step = compress.pack_sh(shells["sh"][1:])
    rest = shells["sh"][1:]
    for ch, (shift, bits) in enumerate(((0, 11), (11, 11), (22, 10))):
        assert lo[ch] == rest[:, ch].min()
        assert step[ch] == np.float32((float(rest[:, ch].max()) - float(lo[ch])) / ((1 << bits) - 1))
        got = (words >> np.uint32(shift)) & np.uint32((1 << bits) - 1)
        np.testing.assert_array_equal(got, oc.pack_codes(rest[:, ch], lo[ch], step[ch], bits))


def test_compressed_values_within_their_quantisation(shells):
    comp = compress.compress(shells, "packed")
    dec = oc.decode(comp)
    for k in ("mean", "scale", "quat", "opacity"):
        x = np.asarray(shells[k], np.float64)
        assert np.all(np.abs(dec[k] - x) <= 2.0 ** -11 * np.abs(x) + 2.0 ** -25), k
    rest = shells["sh"][1:].astype(np.float64)
    err = np.abs(dec["sh"][1:] - rest)
    bound = comp["sh_step"].astype(np.float64)[None, :, None] * 0.5 * (1 + 1e-5) + 1e-6
    assert np.all(err <= bound)
    np.testing.assert_array_equal(dec["layer"], shells["layer"])
    assert compress.nbytes_per_gaussian(comp) == 6 + 6 + 8 + 2 + 6 + 1 + 15 * 4


def test_kmeans_reaches_a_lloyd_fixed_point():
    """On blobs, after enough iterations every centre is the mean of the
    rows assigned to it: the update step changes nothing."""
    rng = np.random.default_rng(0)
    centres = rng.normal(0, 10, (8, 45))
    lab = rng.integers(0, 8, 4000)
    x = (centres[lab] + rng.normal(0, 0.1, (4000, 45))).astype(np.float32)
    c, idx = compress.kmeans(x, 8, iters=30, sample=4000, seed=1)
    for j in np.unique(idx):
        np.testing.assert_allclose(c[j], x[idx == j].astype(np.float64).mean(0), atol=1e-4)


def test_kmeans_assigns_each_row_its_nearest_centre():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1500, 45)).astype(np.float32)
    c, idx = compress.kmeans(x, 40, iters=3, sample=800, seed=2)
    dmin, d = oc.nearest(x, c)
    got = d[np.arange(len(x)), idx]
    assert np.all(got <= dmin + 1e-4 * (1 + dmin))


def test_codebook_layout_with_one_entry_per_gaussian(shells):
    """As many entries as Gaussians, every Gaussian its own centre: decoding
    gives back each Gaussian's coefficients to half precision (checks the
    [index][k][ch] layout against the [k][ch][n] planes)."""
    sub = scenes.subset(shells, np.arange(300))
    comp = compress.compress(sub, "codebook", codebook_size=300, iters=0, sample=300)
    dec = oc.decode(comp)
    want = sub["sh"][1:].astype(np.float16).astype(np.float32)
    np.testing.assert_array_equal(dec["sh"][1:], want)


def test_codebook_stride():
    assert [compress.codebook_stride(D) for D in range(4)] == [0, 16, 24, 48]
