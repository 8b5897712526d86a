"""Pins for oracle/fourier.py: the padded product against a brute-force convolution
sum, and the unpadded transforms against direct sums of exponentials."""
import numpy as np
import pytest

from oracle import fourier as fr


def random_spectrum(rng, nz, nkx, shape=()):
    f = rng.standard_normal(shape + (nz, nkx)) + 1j * rng.standard_normal(shape + (nz, nkx))
    return fr.hermitian_fix_qp(f)


def full_spectrum(fh, nx, nz):
    """dict (p, q) -> coefficient over signed p, q (using f real)."""
    out = {}
    sq = fr.signed_q(nz)
    for qi in range(nz):
        if qi == nz // 2:
            continue
        for p in range(nx // 2):
            q = int(sq[qi])
            out[(p, q)] = fh[qi, p]
            out[(-p, -q)] = np.conj(fh[qi, p])
    return out


def direct_physical(fh, nx, nz, lx, lz, x, z):
    alpha, beta = fr.wavenumbers(nx, nz, lx, lz)
    val = 0.0
    for (p, q), c in full_spectrum(fh, nx, nz).items():
        val += c * np.exp(1j * (2 * np.pi * p / lx * x + 2 * np.pi * q / lz * z))
    return val


@pytest.mark.parametrize("nx,nz", [(4, 4), (8, 4), (8, 8)])
def test_padded_product_is_truncated_convolution(nx, nz):
    rng = np.random.default_rng(nx * 10 + nz)
    f = random_spectrum(rng, nz, nx // 2)
    g = random_spectrum(rng, nz, nx // 2)
    mx, mz = 3 * nx // 2, 3 * nz // 2
    prod = fr.from_padded_physical(fr.to_padded_physical(f, mx, mz) * fr.to_padded_physical(g, mx, mz), nx, nz)
    F, G = full_spectrum(f, nx, nz), full_spectrum(g, nx, nz)
    sq = fr.signed_q(nz)
    for qi in range(nz):
        for p in range(nx // 2):
            if qi == nz // 2:
                assert prod[qi, p] == 0
                continue
            q = int(sq[qi])
            ref = 0.0
            for (p1, q1), c1 in F.items():
                c2 = G.get((p - p1, q - q1))
                if c2 is not None:
                    ref += c1 * c2
            if p == 0 and q < 0:
                continue  # overwritten by the Hermitian fix, checked via q > 0
            assert abs(prod[qi, p] - ref) < 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("nx,nz", [(4, 4), (8, 8), (16, 8)])
def test_unpadded_and_padded_inverse_are_direct_sums(nx, nz):
    rng = np.random.default_rng(3 + nx + nz)
    lx, lz = 2.67, 0.8
    fh = random_spectrum(rng, nz, nx // 2)
    phys = fr.to_physical(fh, nx, nz)
    for k in range(0, nz, 3):
        for i in range(0, nx, 3):
            ref = direct_physical(fh, nx, nz, lx, lz, i * lx / nx, k * lz / nz)
            assert abs(ref.imag) < 1e-12
            assert abs(phys[k, i] - ref.real) < 1e-12
    mx, mz = 3 * nx // 2, 3 * nz // 2
    pp = fr.to_padded_physical(fh, mx, mz)
    for k in range(0, mz, 5):
        for i in range(0, mx, 5):
            ref = direct_physical(fh, nx, nz, lx, lz, i * lx / mx, k * lz / mz)
            assert abs(pp[k, i] - ref.real) < 1e-12
    # forward transform inverts the inverse on resolved spectra
    assert np.allclose(fr.from_physical(phys), fh, atol=1e-14)
    assert np.allclose(fr.from_padded_physical(pp, nx, nz), fh, atol=1e-14)


def test_wavenumbers():
    a, b = fr.wavenumbers(8, 8, 2 * np.pi, np.pi)
    assert np.allclose(a, [0, 1, 2, 3])
    assert np.allclose(b, [0, 2, 4, 6, 0, -6, -4, -2])


def test_hermitian_fix_gives_real_field():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((8, 4)) + 1j * rng.standard_normal((8, 4))
    fh = fr.hermitian_fix_qp(f)
    big = np.zeros((8, 5), dtype=complex)
    big[:, :4] = fh
    assert np.abs(np.fft.ifft(big[:, 0]).imag).max() < 1e-16
    assert np.all(fh[4] == 0)
