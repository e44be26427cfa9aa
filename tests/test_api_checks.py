"""Argument checks of the torch binding: a short output or payload, or a
tensor of the wrong width or device, is refused before any kernel runs
(the kernels would otherwise read or write past the buffer)."""
import pytest
import torch

from paper_1608_08648_amd import api

CPU = torch.device("cpu")


def test_buffer_too_short_is_refused():
    with pytest.raises(ValueError, match="holds 3 elements, 5 needed"):
        api._check_buf("out", torch.empty(3, dtype=torch.int32), 5, 4, CPU)


def test_buffer_of_wrong_width_is_refused():
    with pytest.raises(ValueError, match="8-byte elements, 4 needed"):
        api._check_buf("vals_out", torch.empty(5, dtype=torch.int64), 5, 4, CPU)


def test_buffer_on_another_device_is_refused():
    with pytest.raises(ValueError, match="is on"):
        api._check_buf("keys_out", torch.empty(5, dtype=torch.int32), 5, 4, torch.device("meta"))


def test_buffer_of_the_right_shape_passes():
    api._check_buf("out", torch.empty(5, dtype=torch.int32), 5, 4, CPU)
    api._check_buf("out", None, 5, 4, CPU)


def test_host_tensors_are_refused():
    with pytest.raises(ValueError, match="on the GPU"):
        api.sort_keys(torch.arange(10, dtype=torch.int32))


@pytest.mark.gpu
def test_short_outputs_are_refused_on_the_gpu():
    k = torch.arange(100, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        api.sort_keys(k, out=torch.empty(99, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        api.sort_pairs(k, torch.arange(99, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        api.sort_pairs(k, iota="int64", vals_out=torch.empty(100, dtype=torch.int32, device="cuda"))
    off = torch.tensor([0, 50, 101], dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        api.segmented_sort(k, off, total=101, max_len=51)
    with pytest.raises(ValueError):
        api.segmented_sort(k, off[:2], total=50, max_len=50, keys_out=torch.empty(40, dtype=torch.int32,
                                                                                    device="cuda"))
