"""The seeded input generators (no TT-UTV arithmetic): the PyTorch build of
the Gaussian-TT recipe used for multi-GB tensors equals the NumPy one."""
import numpy as np
import pytest

import ttgen


@pytest.mark.parametrize("dims,ranks", [([3, 4, 5, 2], [2, 3, 2]), ([4, 3, 5, 2, 3], [2, 3, 4, 2]), ([5, 6], [3])])
def test_device_generator_matches_host_generator(dims, ranks):
    a, _ = ttgen.gaussian_tt_tensor(dims, ranks, 0.0, 11)
    b = ttgen.gaussian_tt_tensor_device(dims, ranks, 0.0, 11, dtype="float64", device="cpu").numpy()
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


def test_device_generator_noise_level():
    a, _ = ttgen.gaussian_tt_tensor([4, 3, 5, 2], [2, 3, 2], 0.0, 11)
    b = ttgen.gaussian_tt_tensor_device([4, 3, 5, 2], [2, 3, 2], 1e-3, 11, dtype="float64", device="cpu").numpy()
    assert np.linalg.norm(a - b) / np.linalg.norm(a) == pytest.approx(1e-3, rel=1e-9)
