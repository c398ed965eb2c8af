"""GPU test of the continuous-batching server: requests that arrive while
others render are admitted into batched launches on two streams, and every
request's image equals rendering it alone."""
import numpy as np
import pytest

from paper_2410_16978_amd import scenes

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_16978_amd import rasterizer as rz
    from paper_2410_16978_amd.serve import GpuExecutor, Scheduler, requests_from_trace
    models = [rz.to_device(scenes.shell_scene(2000, 5, 3, seed=1, palette=True)),
              rz.to_device(scenes.shell_scene(4000, 5, 3, seed=2, palette=True))]
    trace = scenes.poisson_trace(3000, 0.02, seed=4, resolutions=((96, 96, 1), (160, 128, 1), (120, 136, 2)))
    reqs = requests_from_trace(trace)
    assert len(reqs) >= 30
    ex = GpuExecutor(models, slots=2)
    ex.calibrate(reqs)
    stats = Scheduler(ex, budget_bytes=1 << 30, max_batch=16).run(reqs)
    torch.cuda.synchronize()
    assert all(r.status == 0 for r in reqs)
    assert stats.launches < len(reqs)  # requests were batched
    for r in reqs:
        outs, st, _ = rz.render_batch(models, [{"model": r.model, "cams": r.cams, "view": r.view}], 400_000)
        torch.cuda.synchronize()
        assert int(st[0]) == 0
        for e in range(len(r.cams)):
            np.testing.assert_array_equal(r.result[0][e].cpu().numpy(), outs[0][0][e].cpu().numpy())
            np.testing.assert_array_equal(r.result[1][e].cpu().numpy(), outs[0][1][e].cpu().numpy())
    print("served:", stats.summary())
