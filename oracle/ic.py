"""Seeded initial conditions (oracle side).

TEST INFRASTRUCTURE: see ``oracle/__init__.py``.

The paper starts every episode from one of six stored turbulent fields
(§3.3, §4.2), which are not available here; a seeded synthetic field with the
paper's grid and Reynolds number stands in.  Recipe (a reading):

* mean profile: laminar U = 1.5 U_b (1 - r^2) with r the distance from the
  centreline of the closed channel (r = xi) or from the surface of the open
  one (r = 1 - y = (1 - xi)/2), or the Reichardt law of the wall in d^+ = d/nu, d the
  distance from the nearest wall, scaled to int U dxi = 2 U_b;
* perturbation on 0 < k, p <= 3, |q| <= 6, with the envelopes E_v, E_o:
  v-hat = E_v sum_{m<8} c_m T_m(xi),  omega_y-hat = E_o sum_{m<8} d_m T_m(xi);
  closed channel E_v = (1 - xi^2)^2, E_o = 1 - xi^2 (v = dv/dy = omega_y = 0 at
  both walls); open channel E_v = (1 + xi)^2 (1 - xi)^3, E_o = (1 + xi)(1 - xi)^2
  (the wall conditions at the bottom, v = d^2v/dy^2 = d omega_y/dy = 0 at the
  free-slip top); the real and imaginary parts
  of c_m, d_m are 2U - 1 with U = (x >> 11) 2^-53 from SplitMix64(seed)
  (Steele, Lea & Flood 2014), drawn in the loop order q (from -6 up), p,
  field (v, then omega_y), m, real part then imaginary part;
* the p = 0 column is made Hermitian (the q > 0 half is kept);
* the perturbation is scaled so that its root-mean-square velocity,
  sqrt(<u'^2 + v'^2 + w'^2> / 3) over the channel volume, equals
  ic_amp * U_cl with U_cl = 1.5 U_b.  The y integral is Clenshaw--Curtis
  quadrature on the nodes (DCT-I of the nodal values, then the integrals of
  T_n).

The library's reset implements the same recipe on its own; the parity tests
do not depend on it (they load the oracle's field through set_state).
"""
import numpy as np

from . import chebyshev as cheb
from . import fourier as fr
from .channel import IC_REICHARDT, State, reconstruct, zero_state

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood 2014), one 64-bit output per call."""

    def __init__(self, seed):
        self.state = int(seed) & MASK64

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next() >> 11) * (2.0 ** -53)


def reichardt(dplus, kappa=0.41):
    """Reichardt's law of the wall u^+(d^+)."""
    return (np.log1p(kappa * dplus) / kappa
            + 7.8 * (1.0 - np.exp(-dplus / 11.0) - (dplus / 11.0) * np.exp(-dplus / 3.0)))


def mean_profile(S):
    xi = S.y
    if S.cfg.ic_profile == IC_REICHARDT:
        d = S.wall_dist if S.open else np.minimum(1.0 + xi, 1.0 - xi)
        a = S.C @ reichardt(d / S.nu)
        return a * (2.0 * S.ub / (S.intw @ a))
    r = (1.0 - xi) / 2.0 if S.open else xi
    return S.C @ (1.5 * S.ub * (1.0 - r * r))


def volume_rms(S, st: State):
    """sqrt(<u^2 + v^2 + w^2> / 3) of the fluctuating part (mean pair excluded)."""
    u, v, w, _, _, _ = reconstruct(S, st)
    mult = np.where(np.arange(S.nkx) == 0, 1.0, 2.0)[None, :]
    total = 0.0
    for f in (u, v, w):
        f = f.copy()
        f[0, 0] = 0.0
        g = np.abs(f @ S.B.T) ** 2            # |f-hat|^2 at the nodes
        integ = (g @ S.C.T) @ S.intw          # int_{-1}^{1} dxi, per (q, p)
        total += np.sum(mult * integ)
    return np.sqrt(total / 2.0 / 3.0)


def initial_state(S, seed):
    st = zero_state(S)
    st.ubar = mean_profile(S)
    rng = SplitMix64(seed)
    xi = S.y
    if S.open:
        env_v = (1.0 + xi) ** 2 * (1.0 - xi) ** 3
        env_o = (1.0 + xi) * (1.0 - xi) ** 2
    else:
        env_v = (1.0 - xi * xi) ** 2
        env_o = 1.0 - xi * xi
    Tm = S.B[:, :8]                          # T_m(y_j), m < 8
    pmax = min(3, S.nkx - 1)
    qmax = min(6, S.nz // 2 - 1)
    for q in range(-qmax, qmax + 1):
        for p in range(0, pmax + 1):
            if p == 0 and q == 0:
                continue
            qi = q % S.nz
            for target, env in ((st.v, env_v), (st.om, env_o)):
                c = np.empty(8, dtype=complex)
                for m in range(8):
                    re = 2.0 * rng.uniform() - 1.0
                    im = 2.0 * rng.uniform() - 1.0
                    c[m] = complex(re, im)
                target[qi, p, :] = S.C @ (env * (Tm @ c))
    st.v = fr.hermitian_fix_qpy(st.v)
    st.om = fr.hermitian_fix_qpy(st.om)
    rms = volume_rms(S, st)
    if rms > 0:
        scale = S.cfg.ic_amp * 1.5 * S.ub / rms
        st.v *= scale
        st.om *= scale
    return st
