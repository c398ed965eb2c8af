"""GPU parity of rendering from compressed attributes (16-bit parameters
with packed or codebook SH, Sec. 4.3): the projection decodes exactly, so
records, pairs and ranges are bit-exact against the oracle's render of the
decoded float32 scene, images within the image bar."""
import numpy as np
import pytest

from oracle import compressed as oc
from paper_2410_16978_amd import compress, scenes
from tests.gpu_helpers import compare_forward
from tests.helpers import small_layered_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_16978_amd import rasterizer
    rasterizer.lib()


@pytest.mark.parametrize("mode,D", [("packed", 3), ("codebook", 3), ("packed", 1), ("codebook", 2), ("packed", 0),
                                    ("codebook", 0)])
def test_compressed_forward_matches_oracle_of_decoded(orc, mode, D):
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=7 + D, n_per_layer=400, sh_degree=D)
    cams = scenes.stereo_cameras([0.2, 0.4, -1.0], 90, 70)
    comp = compress.compress(sc, mode, codebook_size=257, iters=3)
    dec = oc.decode(comp)  # half centres may share depths: both sides order ties by index
    vs = scenes.view_state(0b111, clips=[([0.3, -0.2, 0.9], 0.05, 0b100)], bg=(0.1, 0.2, 0.3))
    st = compare_forward(dec, cams, [vs, vs], orc, label=f"{mode} D{D}", device_model=rz.to_device_compressed(comp))
    print(mode, D, st)


def test_compressed_batch_equals_single_renders():
    """A batch mixing a float model and both compressed forms renders each
    request as it renders alone."""
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=3, n_per_layer=300)
    models = [rz.to_device(sc), rz.to_device_compressed(compress.compress(sc, "packed")),
              rz.to_device_compressed(compress.compress(sc, "codebook", codebook_size=64, iters=2))]
    cams = [scenes.orbit_camera([0.1 * k, 0.3, -1.0], 64, 48) for k in range(3)]
    vs = scenes.view_state()
    reqs = [{"model": m, "cams": [cams[m]], "view": vs} for m in range(3)]
    out, status, _ = rz.render_batch(models, reqs, 2_000_000)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, 0, 0]
    for m in range(3):
        rgb, alpha, _ = rz.rasterize_forward(models[m], [cams[m]], [vs])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[m][0][0].cpu().numpy(), rgb[0].cpu().numpy())
        np.testing.assert_array_equal(out[m][1][0].cpu().numpy(), alpha[0].cpu().numpy())


def test_codebook_index_out_of_range_is_reported(orc):
    """An index at or above codebook_size reads entry 0 and the forward
    reports a device error."""
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=5, n_per_layer=200, sh_degree=2)
    comp = compress.compress(sc, "codebook", codebook_size=16, iters=1)
    comp["sh_index"][7] = 16
    model = rz.to_device_compressed(comp)
    cam = scenes.orbit_camera([0.2, 0.4, -1.0], 64, 48)
    rgb, _, st = rz.rasterize_forward(model, [cam], [scenes.view_state()], sync=False)
    torch.cuda.synchronize()
    with pytest.raises(RuntimeError):
        rz.forward_check(st)
    comp["sh_index"][7] = 0
    rgb0, _, _ = rz.rasterize_forward(rz.to_device_compressed(comp), [cam], [scenes.view_state()])
    np.testing.assert_array_equal(rgb.cpu().numpy(), rgb0.cpu().numpy())


def test_backward_rejects_a_compressed_model():
    import torch
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=6, n_per_layer=50)
    model = rz.to_device_compressed(compress.compress(sc, "packed"))
    cam = scenes.orbit_camera([0.2, 0.4, -1.0], 32, 32)
    rgb, alpha, st = rz.rasterize_forward(model, [cam], [scenes.view_state()])
    with pytest.raises(Exception):
        rz.rasterize_backward(model, [cam], [scenes.view_state()], st, torch.zeros_like(rgb), torch.zeros_like(alpha))


def test_half_subnormals_and_signed_zeros_decode_exactly(orc):
    """Codebook entries and DC coefficients holding half subnormals, signed
    zeros and the halves next to +-1: the records (colours) stay bit-exact.
    (Colours are kept of order one: the image bar is absolute.)"""
    from paper_2410_16978_amd import rasterizer as rz
    sc = small_layered_scene(seed=11, n_per_layer=200, sh_degree=3)
    comp = compress.compress(sc, "codebook", codebook_size=32, iters=1)
    rng = np.random.default_rng(0)
    cb = comp["codebook"]
    special = np.array([0x0001, 0x8001, 0x03FF, 0x83FF, 0x0000, 0x8000, 0x0200, 0x3BFF, 0xBBFF], np.uint16)
    mask = rng.random(cb[:, :45].shape) < 0.5
    cb[:, :45][mask] = rng.choice(special, int(mask.sum()))
    comp["sh_dc"][:, ::5] = rng.choice(special[:7], comp["sh_dc"][:, ::5].shape)
    dec = oc.decode(comp)
    cams = [scenes.orbit_camera([0.1, 0.3, -1.0], 80, 64)]
    st = compare_forward(dec, cams, [scenes.view_state()], orc, label="half specials",
                         device_model=rz.to_device_compressed(comp))
    print(st)
