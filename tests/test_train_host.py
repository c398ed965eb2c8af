"""Host-side tests of the inactive-pruning rule (Sec. 3.2.2): the threshold
schedule, the window average, the comparison, frozen layers and the
max-contribution criterion (CPU tensors, no GPU)."""
import json
import os

import pytest
import torch

from paper_2410_16978_amd.train import PruneConfig, PruneState

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pruning_constants.json")


def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def test_defaults_are_the_papers():
    g = gold()
    c = PruneConfig()
    assert c.interval == g["densification_rate_dR"]
    assert c.threshold == g["initial_threshold_T0"]
    assert c.decay == g["decay_per_pruning_step"]


def test_threshold_schedule_closed_form():
    g = gold()
    ps = PruneState(PruneConfig(use_max_contrib=False))
    layer = torch.zeros(4, dtype=torch.uint8)
    for k in range(40):
        want = g["initial_threshold_T0"] * g["decay_per_pruning_step"] ** k
        assert ps.T == pytest.approx(want, rel=1e-12)
        assert ps.schedule(k) == pytest.approx(want, rel=1e-12)
        ps.steps_in_window = 100
        ps.decide(torch.ones(4), torch.ones(4), layer, 0xFFFFFFFF)


def test_window_average_and_comparison():
    """The gradient measure: the window's average against T."""
    ps = PruneState(PruneConfig(interval=100, threshold=0.015, use_max_contrib=False, measure="gradient"))
    ps.steps_in_window = 100
    # sums over a 100-step window: averages 0.0149, 0.015 (equal: pruned), 0.0151
    act = torch.tensor([1.49, 1.5, 1.51], dtype=torch.float64)
    keep, counts = ps.decide(act, torch.ones(3), torch.zeros(3, dtype=torch.uint8), 0xFFFFFFFF)
    assert keep.tolist() == [False, False, True]
    assert counts["activity"] == 2 and counts["pruned"] == 2
    assert ps.T == pytest.approx(0.015 * 0.975)
    assert ps.steps_in_window == 0


def test_frozen_layers_never_pruned():
    ps = PruneState(PruneConfig(use_max_contrib=True))
    ps.steps_in_window = 100
    layer = torch.tensor([0, 0, 1, 1, 2], dtype=torch.uint8)
    keep, counts = ps.decide(torch.zeros(5), torch.zeros(5), layer, 0b100)  # only layer 2 trains
    assert keep.tolist() == [True, True, True, True, False]


def test_max_contrib_criterion_counted_separately():
    ps = PruneState(PruneConfig(threshold=0.0, use_max_contrib=True))
    ps.steps_in_window = 100
    act = torch.tensor([1.0, 1.0, 0.0])
    mc = torch.tensor([0.5, 1.0 / 255.0 * 0.5, 0.0])
    keep, counts = ps.decide(act, mc, torch.zeros(3, dtype=torch.uint8), 1)
    assert keep.tolist() == [True, False, False]
    assert counts["max_contrib"] == 2 and counts["activity"] == 1 and counts["both"] == 1


def test_both_measures_compare_the_window_average():
    """AvgSample, the window's mean activity, against T for either reading."""
    for measure in ("update", "gradient"):
        ps = PruneState(PruneConfig(interval=100, threshold=0.015, use_max_contrib=False, measure=measure))
        ps.steps_in_window = 100
        act = torch.tensor([1.49, 1.5, 1.51, 0.0], dtype=torch.float64)
        keep, counts = ps.decide(act, torch.ones(4), torch.zeros(4, dtype=torch.uint8), 0xFFFFFFFF)
        assert keep.tolist() == [False, False, True, False]
        assert counts["activity"] == 3
        assert counts["avg_quantiles"][-1] == pytest.approx(0.0151)


def test_unknown_measure_rejected():
    ps = PruneState(PruneConfig(measure="hessian"))
    with pytest.raises(ValueError):
        ps.decide(torch.ones(2), torch.ones(2), torch.zeros(2, dtype=torch.uint8), 1)


# ---------------------------------------------------------------- density control
def test_densify_masks_match_the_oracle_plan():
    import numpy as np
    from oracle import training
    from paper_2410_16978_amd.train import DensifyConfig, densify_masks
    rng = np.random.default_rng(5)
    n = 500
    cnt = rng.integers(0, 4, n).astype(np.float32)
    gs = (rng.random(n) * 6e-4 * cnt).astype(np.float32)
    ls = rng.normal(-4.6, 0.8, (3, n)).astype(np.float32)
    layer = rng.integers(0, 3, n).astype(np.uint8)
    for cfg, V in ((DensifyConfig(), 1), (DensifyConfig.hq(), 8)):
        clone, split = densify_masks(torch.tensor(gs), torch.tensor(cnt), torch.tensor(ls), torch.tensor(layer),
                                     0b110, cfg, 1.3, V)
        plan = training.densify_plan(gs, cnt, np.exp(ls.astype(np.float64)), layer, 0b110, cfg.grad_threshold,
                                     cfg.percent_dense, 1.3, V)
        # float32 and float64 can disagree only at the exact threshold; none is closer than 1e-6 relative here
        assert clone.tolist() == [p == "clone" for p in plan]
        assert split.tolist() == [p == "split" for p in plan]
        assert clone.any() and split.any()


def test_hq_settings_are_the_papers():
    from paper_2410_16978_amd.train import DensifyConfig
    g = gold()
    h = DensifyConfig.hq()
    assert h.grad_threshold == g["hq_densify_grad_threshold"]
    assert h.percent_dense == g["hq_percent_dense"]


def test_split_children_match_the_oracle():
    import numpy as np
    from oracle import training
    from paper_2410_16978_amd.train import split_children
    rng = np.random.default_rng(6)
    m = 37
    mean = rng.standard_normal((3, m))
    ls = rng.normal(-3, 0.5, (3, m))
    q = rng.standard_normal((4, m))
    z = rng.standard_normal((2, 3, m))
    cm, cl = split_children(torch.tensor(mean), torch.tensor(ls), torch.tensor(q), torch.tensor(z), 2)
    for k in range(2):
        for i in range(m):
            wm, ws = training.split_child(mean[:, i], np.exp(ls[:, i]), q[:, i], z[k, :, i], 2)
            np.testing.assert_allclose(cm[:, k * m + i].numpy(), wm, rtol=1e-12, atol=1e-14)
            np.testing.assert_allclose(np.exp(cl[:, k * m + i].numpy()), ws, rtol=1e-12)


def test_camera_extent():
    import numpy as np
    from paper_2410_16978_amd import scenes
    from paper_2410_16978_amd.train import camera_extent
    cams = [scenes.orbit_camera(d, 32, 32) for d in ([1, 0, 0], [-1, 0, 0], [0, 1, 0])]
    cs = np.array([-np.asarray(c["R"], np.float64).reshape(3, 3).T @ np.asarray(c["t"], np.float64) for c in cams])
    want = 1.1 * np.linalg.norm(cs - cs.mean(0), axis=1).max()
    assert camera_extent(cams) == pytest.approx(want, rel=1e-12)
    assert camera_extent(cams[:1]) == 1.0
