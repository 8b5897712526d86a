"""Small configurations and analytic states shared by the oracle and GPU tests.

Everything here is input construction; the method's arithmetic lives in
oracle/ (CPU) and in the library (GPU)."""
import numpy as np
from scipy.optimize import brentq

from oracle import channel as ch


def minimal_channel(**kw):
    """Minimal channel of §3.1 with the closed-channel reading: 2.67 x 2 x 0.8,
    16 x 65 x 16 modes, Re_tau = 180, dt+ = 0.05, sensing at y+ = 15."""
    base = dict(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05,
                obs_y_plus=15.0)
    base.update(kw)
    return ch.Config(**base)


def larger_channel(**kw):
    """Larger channel of §3.1: 2 pi x 2 x pi, 64 x 65 x 64 modes, Re_tau = 180."""
    base = dict(nx=64, ny=65, nz=64, lx=2 * np.pi, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                obs_y_plus=15.0, ic_profile=ch.IC_REICHARDT)
    base.update(kw)
    return ch.Config(**base)


def tiny(**kw):
    base = dict(nx=8, ny=33, nz=8, lx=2.0, lz=1.0, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0)
    base.update(kw)
    return ch.Config(**base)


def rk_amplification(dt, sigma):
    """Exact one-step factor of the three RK3/CN stages for a linear mode
    du/dt = sigma u (explicit part zero)."""
    G = 1.0
    for a, b in zip(ch.RK_ALPHA, ch.RK_BETA):
        G *= (1.0 + a * dt * sigma) / (1.0 - b * dt * sigma)
    return G


def stokes_p(k, parity):
    """Wall-normal wavenumber p of the gravest unsteady-Stokes mode of a
    channel: k tanh k = -p tan p (even v) or k coth k = p cot p (odd v)."""
    if parity == "even":
        f = lambda p: k * np.tanh(k) + p * np.tan(p)
        return brentq(f, np.pi / 2 + 1e-9, np.pi - 1e-9)
    f = lambda p: k / np.tanh(k) - p / np.tan(p)
    return brentq(f, np.pi + 1e-9, 1.5 * np.pi - 1e-9)


def stokes_profile(k, p, parity, y):
    if parity == "even":
        return np.cos(p * y) - np.cos(p) / np.cosh(k) * np.cosh(k * y)
    return np.sin(p * y) - np.sin(p) / np.sinh(k) * np.sinh(k * y)


def cheb_colloc(N):
    """Collocation differentiation matrix on the Gauss--Lobatto nodes
    (Trefethen, Spectral Methods in MATLAB, cheb.m)."""
    x = np.cos(np.pi * np.arange(N + 1) / N)
    c = np.hstack([2.0, np.ones(N - 1), 2.0]) * (-1.0) ** np.arange(N + 1)
    X = np.tile(x, (N + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(N + 1))
    D = D - np.diag(D.sum(axis=1))
    return D, x


def orr_sommerfeld_mode(N, re, alpha):
    """Least-stable Orr--Sommerfeld eigenpair for plane Poiseuille flow
    U = 1 - y^2, by collocation with clamped conditions imposed through
    phi = (1 - y^2) g (Trefethen, Spectral Methods in MATLAB, p40).
    Returns (lambda, phi at all N+1 nodes) for time dependence exp(lambda t)."""
    import scipy.linalg
    D, x = cheb_colloc(N)
    D2 = D @ D
    D3 = D2 @ D
    D4 = D3 @ D
    S = np.diag(np.hstack([0.0, 1.0 / (1.0 - x[1:N] ** 2), 0.0]))
    D4c = ((np.diag(1.0 - x ** 2) @ D4 - 8.0 * np.diag(x) @ D3 - 12.0 * D2) @ S)[1:N, 1:N]
    D2c = D2[1:N, 1:N]
    I = np.eye(N - 1)
    a2 = alpha * alpha
    U = 1.0 - x[1:N] ** 2
    A = (D4c - 2 * a2 * D2c + a2 * a2 * I) / re - 1j * alpha * np.diag(U) @ (D2c - a2 * I) - 2j * alpha * I
    B = D2c - a2 * I
    lam, vec = scipy.linalg.eig(A, B)
    k = np.argmax(lam.real)
    phi = np.zeros(N + 1, dtype=complex)
    phi[1:N] = vec[:, k]
    phi /= phi[np.argmax(np.abs(phi))]
    return lam[k], phi
