"""Fourier transforms in the wall-parallel directions (oracle).

TEST INFRASTRUCTURE: see ``oracle/__init__.py``.

Convention (§3.1: N_x, N_z Fourier modes): on the physical grid
x_i = i L_x / N_x, z_k = k L_z / N_z a real field is

    f(x, z) = sum_{p, q} fh[q, p] exp(i (alpha_p x + beta_q z)),

alpha_p = 2 pi p / L_x, beta_q = 2 pi q / L_z.  Spectral arrays hold
p = 0 .. N_x/2 - 1 (the other half follows from f being real) and q stored
at index q mod N_z, shape (N_z, N_x/2), index order [q, p].  The Nyquist
modes p = N_x/2 and q = N_z/2 are never stored or kept (always zero).

Non-linear products are formed on the 3/2-padded grid M_x = 3 N_x / 2,
M_z = 3 N_z / 2 (the paper is silent on dealiasing; the 3/2 rule in x and z
is the reading used throughout).  ``numpy.fft`` is the transform; pinned by
``tests/test_oracle_fourier.py`` against direct convolution sums.
"""
import numpy as np


def wavenumbers(nx, nz, lx, lz):
    """alpha (N_x/2,), beta (N_z,) with beta at index q mod N_z and 0 at Nyquist."""
    p = np.arange(nx // 2)
    alpha = 2.0 * np.pi * p / lx
    q = np.arange(nz)
    qs = np.where(q < nz // 2, q, q - nz).astype(float)
    qs[nz // 2] = 0.0
    beta = 2.0 * np.pi * qs / lz
    return alpha, beta


def signed_q(nz):
    q = np.arange(nz)
    return np.where(q < nz // 2, q, q - nz)


def hermitian_fix_qp(fh):
    """Make the p = 0 column Hermitian, for arrays shaped (..., N_z, N_x/2).

    fh[-q, 0] := conj(fh[q, 0]) for 0 < q < N_z/2 (the q > 0 half is the one
    kept), Im fh[0, 0] := 0, and the Nyquist row q = N_z/2 is zeroed.  A real
    field has this symmetry exactly; applying it after every forward transform
    and every solve removes the round-off that would otherwise break it."""
    nz = fh.shape[-2]
    out = fh.copy()
    for q in range(1, nz // 2):
        out[..., nz - q, 0] = np.conj(out[..., q, 0])
    out[..., 0, 0] = out[..., 0, 0].real
    out[..., nz // 2, :] = 0.0
    return out


def hermitian_fix_qpy(fh):
    """Hermitian fix for arrays shaped (N_z, N_x/2, N_y) (y axis last)."""
    return np.moveaxis(hermitian_fix_qp(np.moveaxis(fh, -1, 0)), 0, -1)


def to_padded_physical(fh, mx, mz):
    """Spectral (..., N_z, N_x/2) -> real values on the padded (..., M_z, M_x) grid."""
    nz, nkx = fh.shape[-2], fh.shape[-1]
    big = np.zeros(fh.shape[:-2] + (mz, mx // 2 + 1), dtype=complex)
    h = nz // 2
    big[..., :h, :nkx] = fh[..., :h, :]
    big[..., mz - h + 1:, :nkx] = fh[..., h + 1:, :]
    return np.fft.irfft2(big, s=(mz, mx), axes=(-2, -1)) * (mx * mz)


def from_padded_physical(f, nx, nz):
    """Real values on the padded (..., M_z, M_x) grid -> truncated spectrum (..., N_z, N_x/2)."""
    mz, mx = f.shape[-2], f.shape[-1]
    big = np.fft.rfft2(f, axes=(-2, -1)) / (mx * mz)
    out = np.zeros(f.shape[:-2] + (nz, nx // 2), dtype=complex)
    h = nz // 2
    out[..., :h, :] = big[..., :h, :nx // 2]
    out[..., h + 1:, :] = big[..., mz - h + 1:, :nx // 2]
    return hermitian_fix_qp(out)


def to_physical(fh, nx, nz):
    """Spectral (..., N_z, N_x/2) -> real values on the unpadded (..., N_z, N_x) grid."""
    big = np.zeros(fh.shape[:-2] + (nz, nx // 2 + 1), dtype=complex)
    big[..., :, :nx // 2] = fh
    big[..., nz // 2, :] = 0.0
    return np.fft.irfft2(big, s=(nz, nx), axes=(-2, -1)) * (nx * nz)


def from_physical(f):
    """Real values on the (..., N_z, N_x) grid -> spectrum (..., N_z, N_x/2), Nyquist dropped."""
    nz, nx = f.shape[-2], f.shape[-1]
    big = np.fft.rfft2(f, axes=(-2, -1)) / (nx * nz)
    return hermitian_fix_qp(big[..., :, :nx // 2])
