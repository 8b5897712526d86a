"""A second numerical route through the oracle's algorithm (test infrastructure).

The same discrete method with every numerical kernel computed another way:
* tau systems by an LU factorisation (scipy.linalg.lu_factor / lu_solve) with the real and
  imaginary right-hand sides solved separately, instead of numpy.linalg.solve on complex data;
* the Chebyshev transform matrices built from scipy.fft.dct (forward) and from the cosines of
  the reduced angle (inverse), instead of the oracle's explicit products;
* the padded (x, z) transforms as explicit DFT matrices whose angles are reduced modulo the
  length before scaling (accurate to an ulp), instead of numpy.fft.

Differences between this route and the oracle on the same inputs are the algorithm's own
round-off floor: the stiff tau systems (lam ~ 1e6) and the derivative weights (up to N^4) make
some element-wise comparisons sensitive well above machine precision."""
import contextlib

import numpy as np
import scipy.fft
import scipy.linalg

from oracle import channel as ch
from oracle import fourier as fr
from oracle import tau as tau_mod


def lu_tau_solve(N, lam, f, g_top, g_bot, bc=("dirichlet", "dirichlet")):
    f = np.asarray(f)
    batch = f.shape[:-1]
    lam = np.broadcast_to(np.asarray(lam, dtype=float), batch)
    A = tau_mod.tau_matrix(N, lam, bc)
    rhs = np.zeros(batch + (N + 1,), dtype=complex)
    rhs[..., : N - 1] = f[..., : N - 1]
    rhs[..., N - 1] = np.broadcast_to(g_top, batch)
    rhs[..., N] = np.broadcast_to(g_bot, batch)
    out = np.empty(batch + (N + 1,), dtype=complex)
    for idx in np.ndindex(*batch):
        lu = scipy.linalg.lu_factor(A[idx])
        out[idx] = scipy.linalg.lu_solve(lu, rhs[idx].real) + 1j * scipy.linalg.lu_solve(lu, rhs[idx].imag)
    return out if np.iscomplexobj(f) or np.iscomplexobj(g_top) or np.iscomplexobj(g_bot) else out.real


def _signed_rows(nz):
    h = nz // 2
    return np.r_[np.arange(h), np.arange(h + 1, nz)], np.r_[np.arange(h), np.arange(h + 1, nz) - nz]


def dft_to_padded(fh, mx, mz):
    nz, nkx = fh.shape[-2], fh.shape[-1]
    rows, qs = _signed_rows(nz)
    Ez = np.exp(2j * np.pi * (np.outer(np.arange(mz), qs) % mz) / mz)
    ps = np.arange(nkx)
    Ex = np.exp(2j * np.pi * (np.outer(ps, np.arange(mx)) % mx) / mx)
    t = np.einsum("zq,...qp->...zp", Ez, fh[..., rows, :])
    t[..., 0] = t[..., 0].real
    return np.real(np.einsum("...zp,px->...zx", t * np.where(ps == 0, 1.0, 2.0), Ex))


def dft_from_padded(f, nx, nz):
    mz, mx = f.shape[-2], f.shape[-1]
    rows, qs = _signed_rows(nz)
    Ez = np.exp(-2j * np.pi * (np.outer(qs, np.arange(mz)) % mz) / mz)
    Ex = np.exp(-2j * np.pi * (np.outer(np.arange(mx), np.arange(nx // 2)) % mx) / mx)
    g = np.einsum("qz,...zp->...qp", Ez, np.einsum("...zx,xp->...zp", f, Ex)) / (mx * mz)
    out = np.zeros(f.shape[:-2] + (nz, nx // 2), dtype=complex)
    out[..., rows, :] = g
    return fr.hermitian_fix_qp(out)


def second_route_matrices(S):
    """Replace the Setup's Chebyshev transform matrices by the second route's."""
    N = S.N
    C2 = scipy.fft.dct(np.eye(N + 1), type=1, axis=0) / N
    C2[0] *= 0.5
    C2[N] *= 0.5
    S.C = C2
    S.B = np.cos(np.pi * (np.outer(np.arange(N + 1), np.arange(N + 1)) % (2 * N)) / N)
    return S


@contextlib.contextmanager
def second_route():
    """Within the block the oracle's tau solves and padded transforms take the second route;
    Setups made inside should pass through second_route_matrices."""
    saved = (ch.tau_solve, fr.to_padded_physical, fr.from_padded_physical)
    ch.tau_solve = lu_tau_solve
    fr.to_padded_physical, fr.from_padded_physical = dft_to_padded, dft_from_padded
    try:
        yield
    finally:
        ch.tau_solve, fr.to_padded_physical, fr.from_padded_physical = saved
