"""The parity gates of the GPU tests (``oracle.compare``) on planted errors."""
import numpy as np
import pytest

from oracle.compare import check_fields, point_rel, rel_l2


def _fields(n=32768, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(3, n)), rng.normal(size=(3, n))


def test_one_wrong_point_passes_l2_but_fails_the_point_bound():
    """A single point off by 3e-4 of the component's largest value is
    diluted below 1e-5 in relative L2 over 32768 points."""
    E, B = _fields()
    Eg = E.copy()
    Eg[1, 12345] += 3e-4 * np.abs(E[1]).max()
    e, _ = rel_l2(Eg, E)
    assert max(e) < 1e-5
    assert point_rel(Eg, E)[1] == pytest.approx(3e-4, rel=1e-9)
    with pytest.raises(AssertionError):
        check_fields(Eg, B, E, B, 1e-5)


def test_uniform_small_error_passes_both():
    E, B = _fields()
    rng = np.random.default_rng(1)
    Eg = E * (1 + 1e-7 * rng.normal(size=E.shape))
    Bg = B * (1 + 1e-7 * rng.normal(size=B.shape))
    l2, pt = check_fields(Eg, Bg, E, B, 1e-5)
    assert l2 < 1e-6 and pt < 1e-5


def test_vanishing_component_is_normalised_by_the_field():
    E, B = _fields()
    E[2] = 0.0
    Eg = E.copy()
    Eg[2] = 1e-9
    assert point_rel(Eg, E)[2] == pytest.approx(1e-9 / np.abs(E).max())
    check_fields(Eg, B, E, B, 1e-5)


def test_non_finite_results_fail():
    E, B = _fields(64)
    Eg = E.copy()
    Eg[0, 3] = np.nan
    with pytest.raises(AssertionError):
        check_fields(Eg, B, E, B, 1e-5)
