"""The request loop (continuous batching over resident channels) on the GPU: every channel's
results are bitwise those of the same requests served alone, and admission follows the HBM
footprint budget."""
import numpy as np
import pytest

from oracle import channel as ch
from synth import gaussian_action
from tests.gpu_helpers import grid_opts, to_device

pytestmark = pytest.mark.gpu

SPECS = [  # (nx, ny, nz, re_tau, controller, seed)
    (16, 65, 16, 180.0, ch.CTRL_OPPOSITION, 0),
    (32, 65, 32, 100.0, ch.CTRL_EXTERNAL, 1),
    (16, 65, 16, 100.0, ch.CTRL_EXTERNAL, 2),
    (8, 33, 8, 180.0, ch.CTRL_EXTERNAL, 3),
    (32, 65, 32, 180.0, ch.CTRL_OPPOSITION, 4),
]


def cfg_of(spec):
    nx, ny, nz, re, ctrl, _ = spec
    return ch.Config(nx=nx, ny=ny, nz=nz, lx=2.67, lz=0.8, re_tau=re, dt_plus=0.05, obs_y_plus=15.0,
                     controller=ctrl, ic_profile=ch.IC_REICHARDT, obs_mask=3)


def action(spec, k):
    if spec[4] != ch.CTRL_EXTERNAL:
        return None
    return to_device(gaussian_action(2000 + 17 * spec[-1] + k, spec[2], spec[0]))


def test_served_results_equal_alone():
    import paper_2301_09889_amd.binding as b
    from paper_2301_09889_amd.serve import ChannelServer
    server = ChannelServer(hbm_budget=1 << 40)
    for s in SPECS:
        grid, opts = grid_opts(cfg_of(s))
        assert server.admit(grid, opts, s[-1]) is not None
    alone = []
    for s in SPECS:
        grid, opts = grid_opts(cfg_of(s))
        e = b.ChanEnv(grid, opts)
        e.reset(s[-1])
        alone.append(e)
    # an irregular stream: some channels queue several requests, substep counts differ
    stream = [0, 1, 1, 2, 4, 3, 0, 3, 3, 1, 4, 2, 0]
    nsub = {0: 2, 1: 3, 2: 2, 3: 1, 4: 2}
    k_of = [0] * len(SPECS)
    reqs = []
    for c in stream:
        reqs.append(server.submit(c, action(SPECS[c], k_of[c]), nsub[c]))
        k_of[c] += 1
        if len(reqs) % 4 == 0:          # serve while requests keep arriving
            server.step_once()
    while server.has_pending():
        server.step_once()
    assert all(r.code == 0 for r in reqs)
    for c, s in enumerate(SPECS):
        for k in range(k_of[c]):
            alone[c].step(action(s, k), nsub[c])
        assert np.array_equal(alone[c].get_state(), server.channels[c].get_state()), c
        assert np.array_equal(alone[c].obs.cpu().numpy(), server.channels[c].obs.cpu().numpy()), c
        assert np.array_equal(alone[c].tau_w.cpu().numpy(), server.channels[c].tau_w.cpu().numpy()), c
        assert alone[c].drag.item() == server.channels[c].drag.item(), c
    server.close()
    for e in alone:
        e.close()


def test_admission_by_footprint():
    import paper_2301_09889_amd.binding as b
    from paper_2301_09889_amd.serve import ChannelServer
    grid, opts = grid_opts(cfg_of(SPECS[1]))
    need = b.chan_env_footprint_bytes(grid, opts)
    server = ChannelServer(hbm_budget=int(2.5 * need))
    ids = [server.admit(grid, opts, k) for k in range(3)]
    assert ids[:2] == [0, 1] and ids[2] is None
    assert server.used == 2 * need and server.rejected_channels == 1
    small, sopts = grid_opts(cfg_of(SPECS[3]))
    assert b.chan_env_footprint_bytes(small, sopts) <= server.budget - server.used
    assert server.admit(small, sopts, 9) == 2        # a smaller channel still fits
    server.close()
