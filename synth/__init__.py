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
