"""Chebyshev--Gauss--Lobatto tools along the wall-normal direction (oracle).

TEST INFRASTRUCTURE: see ``oracle/__init__.py``.

The paper (§3.1) discretises y with Chebyshev polynomials; N_y = N + 1 is the
number of Chebyshev modes.  A field is f(y) = sum_{n=0}^{N} a_n T_n(y) on
y in [-1, 1] (closed channel of half-height h = 1), collocated at the
Gauss--Lobatto nodes y_j = cos(pi j / N), j = 0..N.  Node j = 0 is the top
wall y = +1 and node j = N the bottom (actuated) wall y = -1.

Everything here is a plain matrix written from its textbook definition
(Gottlieb & Orszag 1977; Canuto, Hussaini, Quarteroni & Zang), and each is
pinned by ``tests/test_oracle_chebyshev.py`` against ``scipy.fft.dct`` and
``numpy.polynomial.chebyshev``.
"""
import numpy as np


def nodes(N):
    """Gauss--Lobatto nodes y_j = cos(pi j / N), j = 0..N (top wall first)."""
    j = np.arange(N + 1)
    return np.cos(np.pi * j / N)


def cbar(N):
    """Weights c-bar_j: 2 at both end points, 1 elsewhere."""
    c = np.ones(N + 1)
    c[0] = 2.0
    c[N] = 2.0
    return c


def forward_matrix(N):
    """DCT-I: a = C f, a_n = 2/(N cb_n) sum_j f_j cos(pi n j/N) / cb_j."""
    j = np.arange(N + 1)
    cb = cbar(N)
    cosm = np.cos(np.pi * np.outer(j, j) / N)
    return (2.0 / N) * cosm / np.outer(cb, cb)


def inverse_matrix(N):
    """Inverse DCT-I: f = B a, f_j = sum_n a_n cos(pi n j / N) = sum_n a_n T_n(y_j)."""
    j = np.arange(N + 1)
    return np.cos(np.pi * np.outer(j, j) / N)


def derivative_matrix(N):
    """First derivative on coefficients.

    b_n = (2 / c_n) sum_{p > n, p + n odd} p a_p, with c_0 = 2 and c_n = 1
    otherwise (b_N = 0).
    """
    D = np.zeros((N + 1, N + 1))
    for n in range(N + 1):
        cn = 2.0 if n == 0 else 1.0
        for p in range(n + 1, N + 1, 2):
            D[n, p] = 2.0 * p / cn
    return D


def second_derivative_matrix(N):
    """Second derivative on coefficients.

    b_n = (1 / c_n) sum_{p >= n + 2, p + n even} p (p^2 - n^2) a_p
    (b_{N-1} = b_N = 0).
    """
    D2 = np.zeros((N + 1, N + 1))
    for n in range(N + 1):
        cn = 2.0 if n == 0 else 1.0
        for p in range(n + 2, N + 1, 2):
            D2[n, p] = p * (p * p - n * n) / cn
    return D2


def value_row(N, side):
    """Row r with r @ a = f(side), side = +1 or -1: T_n(+-1) = (+-1)^n."""
    n = np.arange(N + 1)
    return np.where(n % 2 == 0, 1.0, float(side))


def slope_row(N, side):
    """Row r with r @ a = f'(side): T_n'(+-1) = (+-1)^(n+1) n^2."""
    n = np.arange(N + 1)
    sgn = np.where(n % 2 == 1, 1.0, float(side))
    return sgn * n * n


def integral_weights(N):
    """Row r with r @ a = integral_{-1}^{1} f dy: int T_n = 2/(1-n^2), n even; 0, n odd."""
    n = np.arange(N + 1)
    w = np.zeros(N + 1)
    even = n % 2 == 0
    w[even] = 2.0 / (1.0 - n[even] ** 2)
    return w


def evaluate(a, y):
    """sum_n a_n T_n(y) at arbitrary y in [-1, 1] (T_n(y) = cos(n arccos y)).

    ``a`` has the coefficient index last; the result has shape a.shape[:-1]."""
    n = np.arange(a.shape[-1])
    t = np.cos(n * np.arccos(np.clip(y, -1.0, 1.0)))
    return a @ t
