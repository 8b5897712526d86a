"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds no arithmetic of the method: only random fields with the shapes and
statistics of the paper's workloads, handed identically to the oracle and to
the library.

* gaussian_action: the agents' wall-normal velocity request on the N_z x N_x
  wall grid.  The paper's exploration noise is zero-mean Gaussian with a spread
  of 0.1 u_tau (§3.2, DDPG paragraph; read as a standard deviation); with the
  plane mean removed it is the stand-in for a policy's action.
"""
import numpy as np


def gaussian_action(seed, nz, nx, sigma=0.1):
    """(nz, nx) float64, N(0, sigma^2) from numpy's PCG64(seed), plane mean removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.normal(0.0, sigma, size=(nz, nx))
    return a - a.mean()


def action_sequence(seed, count, nz, nx, sigma=0.1):
    """``count`` consecutive actions of one episode (seeds seed, seed+1, ...)."""
    return [gaussian_action(seed + k, nz, nx, sigma) for k in range(count)]



def broadband_field(seed, nx, ny, nz, ub, amp_v=1.0, amp_om=10.0, amp_w=0.5, amp_wall=0.1, decay=3.0,
                    top_freeslip=False):
    """A flow state with energy in every stored wavenumber pair and every Chebyshev degree.

    Returns (v, om, ubar, wbar, vw_old) in the state exchange shapes: v, om complex
    (nz, nx/2, ny) indexed [q mod nz][p][n]; ubar, wbar (ny,); vw_old complex (nz, nx/2).
    Everything is drawn from numpy's PCG64(seed) and shaped with numpy's Chebyshev series
    routines (the variable y is the Chebyshev variable, -1 the lower wall):

    * every pair (p, q) but (0, 0) and the Nyquist row q = nz/2 gets complex Gaussian
      coefficients g_m with spread exp(-decay m / N) / (1 + (p/(nx/2))^2 + (2|q|/nz)^2) under
      an envelope that meets the boundary conditions, so that the product fills every degree
      up to N: v = E_v(y) sum_m g_m T_m + v_w(p, q) b(y) and omega_y = E_o(y) sum_m h_m T_m.
      Closed channel: E_v = (1 - y^2)^2, E_o = 1 - y^2, b = (1 - y)^2 (2 + y)/4 (b(-1) = 1,
      b'(-1) = 0, b = b' = 0 at the top wall).  Open channel (free-slip top):
      E_v = (1 + y)^2 (1 - y)^3, E_o = (1 + y)(1 - y)^2, b = (1 - y)^3 (5 + 3y)/16 (b(-1) = 1,
      b'(-1) = 0, b = b'' = 0 at the top);
    * v and omega_y are scaled so that their sums of |coefficient|^2 over the pairs (p > 0
      counted twice, for the conjugate half) are amp_v^2 and amp_om^2; the wall term is added
      after the scaling, so v at the lower wall equals the old wall velocity;
    * the p = 0 column is made Hermitian (the q > 0 half kept), as for a real field;
    * U: the laminar profile 1.5 u_b (1 - r^2) (r = y closed, (1 - y)/2 open) plus E_m(y)
      times eight small random coefficients; W: E_m(y) times eight random coefficients of
      spread amp_w (a non-zero spanwise mean flow), E_m = 1 - y^2 (closed) or
      (1 + y)(1 - y)^2 (open, zero slope at the surface);
    * v_w,old: Gaussian of spread amp_wall on every pair but (0, 0) and the Nyquist row.
    """
    from numpy.polynomial import chebyshev as npc
    rng = np.random.Generator(np.random.PCG64(seed))
    N = ny - 1
    nkx = nx // 2
    one_m_y2 = -npc.chebfromroots([-1.0, 1.0])                      # 1 - y^2
    if top_freeslip:
        env_v = npc.chebmul(npc.chebpow([1.0, 1.0], 2), npc.chebpow([1.0, -1.0], 3))
        env_o = npc.chebmul([1.0, 1.0], npc.chebpow([1.0, -1.0], 2))
        bwall = npc.chebmul(npc.chebpow([1.0, -1.0], 3), [5.0, 3.0]) / 16.0
        lam = npc.chebmul([0.5, 0.5], [1.5, -0.5])                   # 1 - ((1 - y)/2)^2
        env_m = env_o
    else:
        env_v = npc.chebpow(one_m_y2, 2)
        env_o = one_m_y2
        bwall = npc.chebmul(npc.chebpow([1.0, -1.0], 2), [2.0, 1.0]) / 4.0
        lam = one_m_y2
        env_m = one_m_y2
    nv = N + 1 - (len(env_v) - 1)
    no = N + 1 - (len(env_o) - 1)
    v = np.zeros((nz, nkx, ny), dtype=complex)
    om = np.zeros((nz, nkx, ny), dtype=complex)
    vw = np.zeros((nz, nkx), dtype=complex)

    def gauss(n, spread):
        return (rng.normal(size=n) + 1j * rng.normal(size=n)) * spread / np.sqrt(2.0)

    def times(env, poly):
        out = np.zeros(ny, dtype=complex)
        prod = npc.chebmul(env, poly)
        out[:prod.size] = prod
        return out

    for qs in range(-(nz // 2 - 1), nz // 2):
        for p in range(nkx):
            if p == 0 and qs <= 0:
                continue
            q = qs % nz
            w = 1.0 / (1.0 + (p / nkx) ** 2 + (2.0 * abs(qs) / nz) ** 2)
            v[q, p] = times(env_v, gauss(nv, w * np.exp(-decay * np.arange(nv) / N)))
            om[q, p] = times(env_o, gauss(no, w * np.exp(-decay * np.arange(no) / N)))
            vw[q, p] = gauss(1, amp_wall)[0]
    mult = np.where(np.arange(nkx) == 0, 1.0, 2.0)[None, :, None]
    v *= amp_v / np.sqrt(np.sum(mult * np.abs(v) ** 2))
    om *= amp_om / np.sqrt(np.sum(mult * np.abs(om) ** 2))
    bw = np.zeros(ny)
    bw[:len(bwall)] = bwall
    v += vw[..., None] * bw[None, None, :]
    for q in range(1, nz // 2):
        v[nz - q, 0] = np.conj(v[q, 0])
        om[nz - q, 0] = np.conj(om[q, 0])
        vw[nz - q, 0] = np.conj(vw[q, 0])
    ubar = np.zeros(ny)
    ubar[:len(lam)] = 1.5 * ub * lam
    eu = npc.chebmul(env_m, rng.normal(size=8) * 0.2 * np.exp(-np.arange(8) / 2.0))
    ew = npc.chebmul(env_m, rng.normal(size=8) * amp_w * np.exp(-np.arange(8) / 2.0))
    ubar[:eu.size] += eu
    wbar = np.zeros(ny)
    wbar[:ew.size] += ew
    return v, om, ubar, wbar, vw
