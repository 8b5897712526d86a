"""Pins for the oracle's three-dimensional non-linear coupling (paper §3.1: the
velocity--vorticity form of the solver, Kim, Moin & Moser 1987).

The two-dimensional and gradient-mode pins elsewhere leave these terms at zero:
h_g = i beta H_1 - i alpha H_3, the -v omega_x part of H_3, the spanwise mean forcing
H_3(0, 0) and the way the stage uses h_u and h_w.  Each is fixed here by an independent
fact:

* brute force: for a divergence-free field whose products are exactly representable
  (Chebyshev degree <= N/2 in y, stored Fourier modes in x and z), H = u x omega is the
  convolution of Chebyshev series (numpy.polynomial.chebyshev.chebmul) over the
  wavenumber pairs, truncated to the stored modes -- no FFT, no nodes, no DCT;
  h_g and h_v are checked against the vortex-stretching form of the vorticity equation,
  curl(u x omega) = (omega . grad) u - (u . grad) omega, evaluated the same way;
* u x omega does no work: at every Gauss--Lobatto node the plane sum of u . H is zero;
* Squire's theorem: an oblique Orr--Sommerfeld mode (alpha = beta = 1, Re = 10^4) evolves
  at the eigenvalue of the two-dimensional problem at k = sqrt(2), Re alpha / k, with
  omega_y following the lift-up (Squire) response solved by the test itself;
* mean momentum: over a very short time step dU/dt = <H_1> + nu U'' and dW/dt = <H_3>.

``test_planted_slips_are_caught`` edits the oracle's own source on the CPU (one sign or one
dropped term at a time) and checks that at least one of these pins fails."""
import inspect
import textwrap

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

import synth
from oracle import channel as ch
from tests.oracle_cases import cheb_colloc, orr_sommerfeld_mode


# ---------------------------------------------------------------------------
# Brute-force spectral fields: {(p, q) signed: Chebyshev coefficients} of a real field.
# ---------------------------------------------------------------------------

class Spec:
    def __init__(self, terms, alpha0, beta0):
        self.t = {k: np.asarray(c, dtype=complex) for k, c in terms.items()}
        self.a0, self.b0 = alpha0, beta0

    def _new(self, terms):
        return Spec(terms, self.a0, self.b0)

    def dx(self):
        return self._new({(p, q): 1j * p * self.a0 * c for (p, q), c in self.t.items()})

    def dz(self):
        return self._new({(p, q): 1j * q * self.b0 * c for (p, q), c in self.t.items()})

    def dy(self):
        return self._new({k: npc.chebder(c) if c.size > 1 else 0 * c for k, c in self.t.items()})

    def __add__(self, o):
        out = dict(self.t)
        for k, c in o.t.items():
            out[k] = npc.chebadd(out[k], c) if k in out else c
        return self._new(out)

    def __neg__(self):
        return self._new({k: -c for k, c in self.t.items()})

    def __sub__(self, o):
        return self + (-o)

    def __mul__(self, o):
        out = {}
        for (p1, q1), c1 in self.t.items():
            for (p2, q2), c2 in o.t.items():
                k = (p1 + p2, q1 + q2)
                prod = npc.chebmul(c1, c2)
                out[k] = npc.chebadd(out[k], prod) if k in out else prod
        return self._new(out)

    def scale(self, s):
        return self._new({k: s * c for k, c in self.t.items()})

    def stored(self, nz, nkx, ny):
        """(nz, nx/2, ny) array of the stored modes p = 0..nx/2-1, |q| < nz/2 (truncation)."""
        out = np.zeros((nz, nkx, ny), dtype=complex)
        for (p, q), c in self.t.items():
            if 0 <= p < nkx and abs(q) < nz // 2:
                if c.size > ny:
                    assert np.abs(c[ny:]).max() < 1e-14 * max(1.0, np.abs(c).max())
                out[q % nz, p, :min(ny, c.size)] += c[:ny]
        return out


def random_potential(rng, pmax, qmax, deg):
    """A real vector potential with |p| <= pmax, |q| <= qmax and Chebyshev degree <= deg."""
    comps = []
    for _ in range(3):
        terms = {}
        for p in range(0, pmax + 1):
            for q in range(-qmax, qmax + 1):
                if p == 0 and q < 0:
                    continue
                c = rng.normal(size=deg + 1) + 1j * rng.normal(size=deg + 1)
                c *= np.exp(-0.3 * np.arange(deg + 1))
                if p == 0 and q == 0:
                    c = c.real.astype(complex)
                terms[(p, q)] = c
                terms[(-p, -q)] = np.conj(c)
        comps.append(terms)
    return comps


def curl(ax, ay, az):
    return az.dy() - ay.dz(), ax.dz() - az.dx(), ay.dx() - ax.dy()


def coupling_case(seed=0):
    """Oracle setup, state and the brute-force fields of one exactly representable field."""
    cfg = ch.Config(nx=8, ny=17, nz=8, lx=2.5, lz=1.7, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0)
    S = ch.Setup(cfg)
    a0, b0 = 2 * np.pi / cfg.lx, 2 * np.pi / cfg.lz
    rng = np.random.default_rng(seed)
    A = [Spec(t, a0, b0) for t in random_potential(rng, 3, 3, S.N // 2)]
    u, v, w = curl(*A)                       # divergence-free by construction
    ox, oy, oz = curl(u, v, w)
    st = ch.zero_state(S)
    shape = (S.nz, S.nkx, S.ny)
    st.v = v.stored(*shape)
    st.om = oy.stored(*shape)
    U = u.stored(*shape)[0, 0]
    W = w.stored(*shape)[0, 0]
    assert np.abs(U.imag).max() < 1e-15 and np.abs(W.imag).max() < 1e-15
    st.ubar, st.wbar = U.real.copy(), W.real.copy()
    return S, st, (u, v, w), (ox, oy, oz)


def check_brute_force(seed=0):
    S, st, (u, v, w), (ox, oy, oz) = coupling_case(seed)
    shape = (S.nz, S.nkx, S.ny)
    Hbf = [(v * oz - w * oy).stored(*shape), (w * ox - u * oz).stored(*shape),
           (u * oy - v * ox).stored(*shape)]
    H = ch.nonlinear(S, st)
    scale = max(np.abs(h).max() for h in Hbf)
    for k in range(3):
        err = np.abs(H[k] - Hbf[k]).max() / scale
        assert err < 1e-13, f"H_{k + 1}: {err:.2e}"
    # vortex-stretching form: g = (omega . grad) u - (u . grad) omega = curl(u x omega)
    comps_u, comps_o = (u, v, w), (ox, oy, oz)

    def grad_dot(a, f):
        return a[0] * f.dx() + a[1] * f.dy() + a[2] * f.dz()

    g = [grad_dot(comps_o, comps_u[i]) - grad_dot(comps_u, comps_o[i]) for i in range(3)]
    hg_bf = g[1].stored(*shape)
    hv_bf = -(g[0].dz() - g[2].dx()).stored(*shape)   # -(curl g)_y = -(curl curl H)_y
    hv, hg, hu, hw = ch.explicit_terms(S, H)
    act = S.active[..., None]
    hg_bf = np.where(act, hg_bf, 0.0)
    hv_bf = np.where(act, hv_bf, 0.0)
    e_g = np.abs(hg - hg_bf).max() / np.abs(hg_bf).max()
    e_v = np.abs(hv - hv_bf).max() / np.abs(hv_bf).max()
    assert e_g < 1e-12, f"h_g: {e_g:.2e}"
    assert e_v < 1e-12, f"h_v: {e_v:.2e}"
    # mean forcing: the plane means of H_1 and H_3
    assert np.abs(hu - Hbf[0][0, 0].real).max() < 1e-13 * scale
    assert np.abs(hw - Hbf[2][0, 0].real).max() < 1e-13 * scale
    assert np.abs(Hbf[2][0, 0]).max() > 1e-2 * scale     # W forcing is exercised
    return S, st


def check_no_work(seed=7):
    """Plane sum of u . H at every node is zero (u . (u x omega) = 0 pointwise, and the
    truncation removes only modes that u does not carry)."""
    cfg = ch.Config(nx=16, ny=33, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0)
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    st.v, st.om, st.ubar, st.wbar, st.vw_old = synth.broadband_field(seed, S.nx, S.ny, S.nz, S.ub)
    u = ch.reconstruct(S, st)[:3]
    H = ch.nonlinear(S, st)
    mult = np.where(np.arange(S.nkx) == 0, 1.0, 2.0)[None, :]
    work = np.zeros(S.ny)
    size = np.zeros(S.ny)
    for f, h in zip(u, H):
        fv = npc.chebval(S.y, np.moveaxis(f, -1, 0))       # (nz, nkx, ny) values at the nodes
        hv = npc.chebval(S.y, np.moveaxis(h, -1, 0))
        work += np.einsum("qp,qpj->j", mult, (fv * np.conj(hv)).real)
        size += np.einsum("qp,qpj->j", mult, np.abs(fv) * np.abs(hv))
    rel = np.abs(work).max() / size.max()
    assert rel < 1e-13, f"plane work of u x omega: {rel:.2e}"


def squire_response(N, re, alpha, beta, lam, phi):
    """omega_y of the oblique mode: [lam + i alpha U - (D^2 - k^2)/Re] omega = -i beta U' v,
    omega(+-1) = 0, by collocation on the Gauss--Lobatto nodes (U = 1 - y^2)."""
    D, x = cheb_colloc(N)
    k2 = alpha * alpha + beta * beta
    L = lam * np.eye(N + 1) + 1j * alpha * np.diag(1 - x ** 2) - (D @ D - k2 * np.eye(N + 1)) / re
    rhs = -1j * beta * (-2 * x) * phi
    om = np.zeros(N + 1, dtype=complex)
    om[1:N] = np.linalg.solve(L[1:N, 1:N], rhs[1:N])
    return om


def check_oblique_mode(n1=60, n2=300):
    re, alpha, beta = 1.0e4, 1.0, 1.0
    k = np.hypot(alpha, beta)
    cfg = ch.Config(nx=4, ny=65, nz=4, lx=2 * np.pi / alpha, lz=2 * np.pi / beta, re_tau=180.0,
                    dt_plus=0.05, obs_y_plus=15.0, forcing=ch.CPG, px=2.0 / re,
                    nu_override=1.0 / re, dt_override=0.01)
    S = ch.Setup(cfg)
    lam2, phi = orr_sommerfeld_mode(S.N, re * alpha / k, k)   # Squire: 2-D problem at (k, Re alpha/k)
    lam3 = lam2 * alpha / k
    om = squire_response(S.N, re, alpha, beta, lam3, phi)
    st = ch.zero_state(S)
    st.ubar = S.C @ (1 - S.y ** 2)
    eps = 1e-6
    st.v[1, 1] = S.C @ (eps * phi)
    st.om[1, 1] = S.C @ (eps * om)
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    snaps = {}
    for n in range(n2 + 1):
        if n in (n1, n2):
            snaps[n] = (st.v[1, 1].copy(), st.om[1, 1].copy())
        if n < n2:
            st = ch.time_step(S, st, lambda r: zero)
    (v1, o1), (v2, o2) = snaps[n1], snaps[n2]
    g = np.vdot(v1, v2) / np.vdot(v1, v1)
    rate = np.log(g) / ((n2 - n1) * S.dt)
    err_rate = abs(rate - lam3) / abs(lam3)
    assert err_rate < 1e-6, f"oblique rate {rate} vs Squire {lam3}: {err_rate:.2e}"
    assert np.linalg.norm(v2 - g * v1) < 1e-6 * np.linalg.norm(g * v1)
    err_om = np.linalg.norm(o2 - g * o1) / np.linalg.norm(g * o1)
    assert err_om < 1e-6, f"omega_y does not follow the mode: {err_om:.2e}"
    # the lift-up response itself (relative to v, as in the eigenvector)
    ratio = np.vdot(S.C @ (eps * om), o1) / np.vdot(S.C @ (eps * om), S.C @ (eps * om))
    rv = np.vdot(S.C @ (eps * phi), v1) / np.vdot(S.C @ (eps * phi), S.C @ (eps * phi))
    assert abs(ratio / rv - 1.0) < 1e-5, f"omega_y / v = {ratio / rv}"
    assert np.linalg.norm(o1) > 1e-2 * eps   # omega_y is forced, not vanishing
    return lam3, rate


def check_mean_momentum(seed=2):
    """A time step of dt = 1e-8: (U(dt) - U)/dt = P_x + <H_1> + nu U'' and (W(dt) - W)/dt =
    <H_3> + nu W'' to O(dt).  The field is at rest at the walls (no wall velocity, v = v' =
    omega_y = 0), U = 1.5 U_b (1 - y^2) with P_x = 3 nu U_b and W = (1 - y^2)^3 (...), so that
    both rates vanish at the walls and the short step has no wall layer."""
    cfg = ch.Config(nx=16, ny=33, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                    forcing=ch.CPG, dt_override=1e-8)
    S0 = ch.Setup(cfg)
    cfg.px = 3.0 * S0.nu * S0.ub
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    v, om, _, _, _ = synth.broadband_field(seed, S.nx, S.ny, S.nz, S.ub, decay=8.0, amp_wall=0.0)
    st.v, st.om = v, om
    st.ubar = np.zeros(S.ny)
    st.ubar[:3] = [0.75 * S.ub, 0.0, -0.75 * S.ub]
    wpoly = npc.chebmul(npc.chebpow(-npc.chebfromroots([-1.0, 1.0]), 3),
                        np.random.default_rng(seed).normal(size=6) * 0.5)
    st.wbar = np.zeros(S.ny)
    st.wbar[:wpoly.size] = wpoly
    H = ch.nonlinear(S, st)
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    out = ch.time_step(S, st, lambda r: zero)
    for got, old, h, px in ((out.ubar, st.ubar, H[0][0, 0].real, cfg.px), (out.wbar, st.wbar, H[2][0, 0].real, 0.0)):
        rate = npc.chebval(S.y, (got - old) / S.dt)
        expect = px + npc.chebval(S.y, npc.chebadd(h, S.nu * npc.chebder(old, 2)))
        err = np.abs(rate - expect).max() / np.abs(expect).max()
        assert err < 1e-5, f"mean momentum: {err:.2e}"
        assert np.abs(npc.chebval(S.y, h)).max() > 0.1 * np.abs(expect).max()  # H matters


def test_nonlinear_term_against_brute_force_convolution():
    for seed in (0, 1):
        check_brute_force(seed)


def test_u_cross_omega_does_no_work():
    check_no_work()


def test_oblique_mode_follows_squire_theorem():
    lam3, rate = check_oblique_mode()
    print(f"  oblique mode: Squire {lam3:.10f}, oracle {rate:.10f}")


def test_mean_momentum_over_a_short_step():
    check_mean_momentum()


# ---------------------------------------------------------------------------
# Planted slips: each one edits one line of the oracle's source (in memory, on the CPU).
# ---------------------------------------------------------------------------

def _planted(fn, old, new):
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (fn.__name__, old)
    ns = dict(vars(ch))
    exec(compile(src.replace(old, new), f"<planted {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


SLIPS = [
    ("nonlinear", "H3 = U * OY - V * OX", "H3 = U * OY + V * OX"),
    ("nonlinear", "H3 = U * OY - V * OX", "H3 = U * OY"),
    ("nonlinear", "H1 = V * OZ - W * OY", "H1 = V * OZ + W * OY"),
    ("nonlinear", "H2 = W * OX - U * OZ", "H2 = W * OX"),
    ("explicit_terms", "ib * H1 - ia * H3", "ib * H1 + ia * H3"),
    ("explicit_terms", "ib * H1 - ia * H3", "- ia * H3"),
    ("explicit_terms", "(ia * H1 + ib * H3)", "(ia * H1 - ib * H3)"),
    ("explicit_terms", "H3[0, 0].real.copy()", "-H3[0, 0].real.copy()"),
    ("stage", "(g_r * hw + z_r * hw_p)", "(g_r * hw - z_r * hw_p)"),
    ("stage", "(g_r * hu + z_r * hu_p)", "0.0 * (g_r * hu + z_r * hu_p)"),
    ("stage", "(g_r * hg[act] + z_r * hg_p[act])", "(g_r * hg[act] - z_r * hg_p[act])"),
]

PINS = [check_brute_force, check_no_work, lambda: check_oblique_mode(40, 160), check_mean_momentum]


@pytest.mark.parametrize("fn,old,new", SLIPS)
def test_planted_slips_are_caught(monkeypatch, fn, old, new):
    monkeypatch.setattr(ch, fn, _planted(getattr(ch, fn), old, new))
    caught = []
    for pin in PINS:
        try:
            pin()
        except AssertionError as e:
            caught.append(str(e).splitlines()[0] if str(e) else pin.__name__)
    assert caught, f"slip {old!r} -> {new!r} passed every pin"
