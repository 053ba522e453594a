"""Host-side checks of the multilayer-perceptron wrapper (no GPU calls)."""
import pytest
import torch

import paper_1912_04379_amd as mg


def test_step_flops_counted_by_hand():
    # batch 2, widths 3 -> 4 -> 5: forward 2*2*(3*4 + 4*5) = 128; the input
    # gradient of layer 2 only, 2*2*4*5 = 80; weight gradients 128.
    assert mg.mlp_step_flops(2, [3, 4, 5]) == 336


def test_rejects_widths_that_do_not_chain():
    with pytest.raises(ValueError):
        mg.MLP([torch.zeros(3, 4), torch.zeros(5, 2)])


def test_rejects_non_contiguous_or_non_float32_weights():
    with pytest.raises(ValueError):
        mg.MLP([torch.zeros(4, 3).t()])
    with pytest.raises(ValueError):
        mg.MLP([torch.zeros(3, 4, dtype=torch.float64)])
    with pytest.raises(ValueError):
        mg.MLP([])
