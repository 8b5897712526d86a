"""Pins for oracle/tau.py: the tau method reproduces every polynomial of degree <= N
exactly, so manufactured polynomial solutions (right-hand sides built with
numpy.polynomial.chebyshev, not with the oracle's own matrices) must come back."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle.tau import tau_solve


def manufactured(N, lam, rng, cplx=False):
    X = rng.standard_normal(N + 1) / (1.0 + np.arange(N + 1)) ** 2
    if cplx:
        X = X + 1j * rng.standard_normal(N + 1) / (1.0 + np.arange(N + 1)) ** 2
    d2 = np.zeros(N + 1, dtype=X.dtype)
    d2[:N - 1] = npc.chebder(X, 2)
    f = d2 - lam * X
    return X, f


@pytest.mark.parametrize("N", [8, 16, 64, 96])
@pytest.mark.parametrize("lam", [0.0, 1.0, 37.5, 2.43e6, 9.72e6])
def test_dirichlet_manufactured(N, lam):
    rng = np.random.default_rng(N)
    X, f = manufactured(N, lam, rng, cplx=True)
    gt, gb = npc.chebval(1.0, X), npc.chebval(-1.0, X)
    sol = tau_solve(N, lam, f, gt, gb)
    # round-off of the D^2 rows grows like N^2 relative to the data
    assert np.abs(sol - X).max() < 5e-17 * N * N * max(1.0, np.abs(X).max())


@pytest.mark.parametrize("N", [16, 64])
def test_neumann_manufactured(N):
    rng = np.random.default_rng(11)
    lam = 5.0
    X, f = manufactured(N, lam, rng)
    d = npc.chebder(X)
    sol = tau_solve(N, lam, f, npc.chebval(1.0, d), npc.chebval(-1.0, d), bc=("neumann", "neumann"))
    assert np.abs(sol - X).max() < 1e-12


def test_batched_matches_single():
    rng = np.random.default_rng(3)
    N = 32
    lams = np.array([1.0, 10.0, 1e5])
    Xs, fs = zip(*[manufactured(N, l, rng) for l in lams])
    fs = np.array(fs)
    sol = tau_solve(N, lams, fs, [npc.chebval(1, x) for x in Xs], [npc.chebval(-1, x) for x in Xs])
    for k in range(3):
        assert np.abs(sol[k] - Xs[k]).max() < 1e-12
