"""Pin of the oracle adjoint gradients: central finite differences of the
direct solve (h = 1e-6)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint


@pytest.mark.parametrize("base", [W.TINY.replace(nc=3, nm=6), W.ADJOINT.replace(nc=3, nm=6, n_th=1e-15)])
def test_adjoint_matches_central_differences(base):
    vals, g = adjoint.gradients(base)
    fd = adjoint.finite_differences(base, h=1e-6)
    scale = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max(axis=1, keepdims=True))
    assert np.max(np.abs(g - fd) / scale) <= 1e-5
