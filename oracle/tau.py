"""Dense Chebyshev-tau solves (oracle).

TEST INFRASTRUCTURE: see ``oracle/__init__.py``.

The implicit (Crank--Nicolson) part of each Runge--Kutta stage (§3.1) leaves,
for every wavenumber pair, one-dimensional Helmholtz problems
(D^2 - lam) X = f on y in [-1, 1] with two boundary conditions.  The tau
method (Gottlieb & Orszag 1977) keeps the equations for the Chebyshev
coefficients n = 0 .. N-2 and replaces the last two by the boundary rows.
Written here as the plain dense (N+1) x (N+1) matrix and solved by LAPACK
(``numpy.linalg.solve``).  Pinned in ``tests/test_oracle_tau.py`` by
polynomial manufactured solutions, which the tau method reproduces exactly.
"""
import numpy as np

from . import chebyshev as cheb


def tau_matrix(N, lam, bc=("dirichlet", "dirichlet")):
    """(N+1)x(N+1) tau matrix for (D^2 - lam); rows N-1, N are the conditions
    at y = +1 and y = -1 ("dirichlet" -> value row, "neumann" -> slope row).
    ``lam`` may be an array; the result then has shape lam.shape + (N+1, N+1)."""
    lam = np.asarray(lam, dtype=float)
    D2 = cheb.second_derivative_matrix(N)
    I = np.eye(N + 1)
    A = np.broadcast_to(D2, lam.shape + (N + 1, N + 1)).copy()
    A -= lam[..., None, None] * I
    rows = []
    for side, kind in zip((+1, -1), bc):
        rows.append(cheb.value_row(N, side) if kind == "dirichlet" else cheb.slope_row(N, side))
    A[..., N - 1, :] = rows[0]
    A[..., N, :] = rows[1]
    return A


def tau_solve(N, lam, f, g_top, g_bot, bc=("dirichlet", "dirichlet")):
    """Solve (D^2 - lam) X = f (rows 0..N-2) with X or X' = g_top at y=+1, g_bot at y=-1.

    ``f`` has the coefficient axis last; ``lam``, ``g_top``, ``g_bot``
    broadcast against f.shape[:-1].  Complex data are solved as two real
    right-hand sides (real and imaginary parts) of the same real system."""
    f = np.asarray(f)
    batch = f.shape[:-1]
    lam = np.broadcast_to(np.asarray(lam, dtype=float), batch)
    g_top = np.broadcast_to(np.asarray(g_top), batch)
    g_bot = np.broadcast_to(np.asarray(g_bot), batch)
    A = tau_matrix(N, lam, bc)
    is_c = np.iscomplexobj(f) or np.iscomplexobj(g_top) or np.iscomplexobj(g_bot)
    rhs = np.zeros(batch + (N + 1,), dtype=complex if is_c else float)
    rhs[..., : N - 1] = f[..., : N - 1]
    rhs[..., N - 1] = g_top
    rhs[..., N] = g_bot
    if is_c:
        b = np.stack([rhs.real, rhs.imag], axis=-1)
        x = np.linalg.solve(A, b)
        return x[..., 0] + 1j * x[..., 1]
    return np.linalg.solve(A, rhs[..., None])[..., 0]
