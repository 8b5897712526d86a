"""Pins for oracle/chebyshev.py against library routines (scipy.fft, numpy.polynomial)."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
import scipy.fft

from oracle import chebyshev as cheb

NS = [4, 8, 16, 64, 96]


@pytest.mark.parametrize("N", NS)
def test_forward_matches_scipy_dct1(N):
    rng = np.random.default_rng(N)
    f = rng.standard_normal(N + 1)
    a = cheb.forward_matrix(N) @ f
    ref = scipy.fft.dct(f, type=1) / (N * cheb.cbar(N))
    assert np.allclose(a, ref, rtol=0, atol=1e-14 * np.abs(f).max() * 4)


@pytest.mark.parametrize("N", NS)
def test_inverse_is_chebval_at_nodes(N):
    rng = np.random.default_rng(N + 1)
    a = rng.standard_normal(N + 1)
    y = cheb.nodes(N)
    assert np.allclose(cheb.inverse_matrix(N) @ a, npc.chebval(y, a), atol=1e-13)
    assert np.allclose(cheb.forward_matrix(N) @ npc.chebval(y, a), a, atol=1e-13)


@pytest.mark.parametrize("N", NS)
def test_nodes_order(N):
    y = cheb.nodes(N)
    assert y[0] == 1.0 and abs(y[N] + 1.0) < 1e-15
    assert np.all(np.diff(y) < 0)


@pytest.mark.parametrize("N", NS)
def test_derivatives_match_chebder(N):
    rng = np.random.default_rng(N + 2)
    a = rng.standard_normal(N + 1)
    d1 = np.zeros(N + 1)
    d1[:N] = npc.chebder(a)
    d2 = np.zeros(N + 1)
    d2[:N - 1] = npc.chebder(a, 2)
    scale = N ** 4
    assert np.allclose(cheb.derivative_matrix(N) @ a, d1, atol=1e-14 * N * N)
    assert np.allclose(cheb.second_derivative_matrix(N) @ a, d2, atol=1e-14 * scale)


@pytest.mark.parametrize("N", NS)
def test_boundary_rows_and_integral(N):
    rng = np.random.default_rng(N + 3)
    a = rng.standard_normal(N + 1)
    for side in (+1, -1):
        assert np.isclose(cheb.value_row(N, side) @ a, npc.chebval(side, a), atol=1e-12)
        assert np.isclose(cheb.slope_row(N, side) @ a, npc.chebval(side, npc.chebder(a)),
                          rtol=1e-12, atol=1e-12)
    ia = npc.chebint(a, lbnd=-1)
    assert np.isclose(cheb.integral_weights(N) @ a, npc.chebval(1.0, ia), atol=1e-12)


def test_evaluate_matches_chebval():
    rng = np.random.default_rng(7)
    a = rng.standard_normal(33)
    y = np.linspace(-1, 1, 17)
    assert np.allclose([cheb.evaluate(a, t) for t in y], npc.chebval(y, a), atol=1e-13)
