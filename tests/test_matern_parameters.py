"""Host logic: the Matern parameters of the wavelet form (Prop. 3.2: s = nu + d/2; Cor. 4.3: the
depth puts the unweighted scale at the correlation scale rho / sqrt(2 nu))."""
import math

import pytest

from paper_2507_02401_amd import matern_depth, matern_parameters, matern_to_s


def test_matern_depth_values():
    # Prop. 3.2's own case rho = sqrt(2 nu): the unweighted scale is the unit length, so a unit box
    # with n samples per side needs the full depth log2(n)
    for nu in (0.5, 1.0, 2.5):
        assert matern_depth(nu, math.sqrt(2 * nu), 1 / 1024) == 10
    assert matern_depth(0.5, 1.0, 1 / 512) == 9
    assert matern_depth(1.5, math.sqrt(3) / 8, 1 / 1024) == 7
    assert matern_depth(1.5, math.sqrt(3), 1.0) == 0


def test_matern_depth_shifts_one_level_per_octave_of_rho():
    for k in range(4):
        assert matern_depth(0.75, math.sqrt(1.5) * 0.3 * 2 ** (3 + k), 0.3) == 3 + k


def test_matern_depth_rejects_non_dyadic_scales():
    with pytest.raises(ValueError):
        matern_depth(0.5, 1.0, 1 / 500)
    with pytest.raises(ValueError):
        matern_depth(0.5, 0.25, 1.0)  # coarser than the grid spacing: negative depth
    with pytest.raises(ValueError):
        matern_depth(0.0, 1.0, 0.1)


def test_matern_parameters():
    assert matern_parameters(0.5, 1.0, 2, 1 / 512) == (1.5, 9)
    assert matern_parameters(1.0, math.sqrt(2), 3, 1 / 64) == (matern_to_s(1.0, 3), 6)
