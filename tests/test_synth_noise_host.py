"""Host-side checks of the device noise generator for regenerated data sets
(synth/noise.hip, synth/gpu_noise.py): the library loads and exports its
entry point, rejects invalid sizes before touching the GPU, and the Python
wrapper rejects tensors of the wrong kind.  The noise itself is checked on
the GPU (tests/test_gpu_stream.py)."""
import ctypes

import pytest
import torch

from synth import gpu_noise


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(gpu_noise.LIB):
        gpu_noise.build()
    return gpu_noise.lib()


def test_invalid_sizes_are_rejected_on_the_host(lib):
    f = lib.synth_add_disk_noise
    assert f(None, None, 70000, 64, 100, 1.0, 1, None) == -1        # more images than one launch holds
    assert f(None, None, -1, 64, 100, 1.0, 1, None) == -1
    assert f(None, None, 4, 0, 100, 1.0, 1, None) == -1             # no image side
    assert f(None, None, 4, 8192, 100, 1.0, 1, None) == -1
    assert f(None, None, 4, 64, 100, -1.0, 1, None) == -1           # negative variance
    assert f(None, None, 4, 64, 100, float("nan"), 1, None) == -1
    assert f(None, None, 0, 64, 100, 1.0, 1, None) == 0             # empty batch: nothing to do


def test_wrapper_checks_its_tensors():
    x = torch.zeros((2, 8, 8), dtype=torch.complex64)
    idx = torch.zeros(2, dtype=torch.int64)
    with pytest.raises(ValueError):
        gpu_noise.add_disk_noise(x, idx, 16, 1.0, 1)                 # host tensor
    with pytest.raises(ValueError):
        gpu_noise.add_disk_noise(torch.zeros((2, 8, 4), dtype=torch.complex64), idx, 16, 1.0, 1)


def test_noise_key():
    k = gpu_noise.noise_seed(5320, 3)
    assert k == (5320 << 8) | 3 and 0 <= k < 2 ** 64
    assert gpu_noise.noise_seed(5320, 3) != gpu_noise.noise_seed(5321, 3)
