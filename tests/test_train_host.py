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


def test_update_measure_compares_the_window_sum():
    """The update measure: the window's accumulated activity against T."""
    ps = PruneState(PruneConfig(interval=100, threshold=0.015, use_max_contrib=False))
    assert ps.cfg.measure == "update"
    ps.steps_in_window = 100
    act = torch.tensor([0.0149, 0.015, 0.0151, 0.0], dtype=torch.float64)
    keep, counts = ps.decide(act, torch.ones(4), torch.zeros(4, dtype=torch.uint8), 0xFFFFFFFF)
    assert keep.tolist() == [False, False, True, False]
    assert counts["activity"] == 3
    assert ps.T == pytest.approx(0.015 * 0.975)


def test_unknown_measure_rejected():
    ps = PruneState(PruneConfig(measure="hessian"))
    with pytest.raises(ValueError):
        ps.decide(torch.ones(2), torch.ones(2), torch.zeros(2, dtype=torch.uint8), 1)
