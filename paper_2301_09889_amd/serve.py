"""Request loop for many RL workers: env-step requests on resident channels, served with
continuous batching.

Every channel's flow state stays on the device.  A channel is admitted only while the summed
HBM footprint (chan_env_footprint_bytes) of the admitted channels fits the server's budget.
Each iteration of the loop takes, for every channel with a pending request, its oldest one,
groups them by the number of time steps asked for, and advances each group with one
chan_batch_step_subset call over all resident channels of the batch; requests that arrive
while a call is on the GPU join the next iteration.  A request's latency runs from its
arrival to the end of the call that served it.  Every channel computes exactly what it would
compute alone (the batched launches run the same per-channel code), so a result does not
depend on what else was in the mix.
"""
import collections
import time

from . import binding as b


class Request:
    __slots__ = ("channel", "action", "n_substeps", "t_arrival", "t_done", "code")

    def __init__(self, channel, action, n_substeps, t_arrival):
        self.channel = channel
        self.action = action
        self.n_substeps = n_substeps
        self.t_arrival = t_arrival
        self.t_done = None
        self.code = None


class ChannelServer:
    """Resident channels behind one request queue.

    hbm_budget: bytes the channels' device allocations may take together.  Channels are
    ChanEnv objects (their obs / tau_w / drag tensors receive each served request's outputs).
    """

    def __init__(self, hbm_budget):
        self.budget = int(hbm_budget)
        self.used = 0
        self.channels = []          # ChanEnv, index = channel id
        self.footprint = []
        self.batch = None
        self.pending = collections.defaultdict(collections.deque)
        self.done = []
        self.rejected_channels = 0

    def admit(self, grid, opts, seed):
        """Create and reset a channel if its footprint fits the remaining budget; returns its id
        or None (not admitted)."""
        need = b.chan_env_footprint_bytes(grid, opts)
        if need == 0:
            raise ValueError("invalid grid or options")
        if self.used + need > self.budget:
            self.rejected_channels += 1
            return None
        env = b.ChanEnv(grid, opts)
        env.reset(seed)
        self.channels.append(env)
        self.footprint.append(need)
        self.used += need
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        return len(self.channels) - 1

    def _ensure_batch(self):
        if self.batch is None:
            self.batch = b.ChanBatch(self.channels)

    def submit(self, channel, action, n_substeps, t_arrival=None):
        """Queue an env step of a channel (action: float64 device tensor (nz, nx) or None)."""
        r = Request(channel, action, n_substeps, time.perf_counter() if t_arrival is None else t_arrival)
        self.pending[channel].append(r)
        return r

    def has_pending(self):
        return any(self.pending[c] for c in self.pending)

    def step_once(self):
        """One loop iteration: serve the oldest pending request of every channel that has one.
        Returns the requests completed."""
        heads = [q[0] for c, q in self.pending.items() if q]
        if not heads:
            return []
        self._ensure_batch()
        by_n = collections.defaultdict(list)
        for r in heads:
            by_n[r.n_substeps].append(r)
        served = []
        for n_sub, reqs in sorted(by_n.items()):
            reqs.sort(key=lambda r: r.channel)
            codes = self.batch.step_subset([r.channel for r in reqs], [r.action for r in reqs], n_sub)
            t = time.perf_counter()
            for r, code in zip(reqs, codes):
                r.code = code
                r.t_done = t
                self.pending[r.channel].popleft()
            served.extend(reqs)
        self.done.extend(served)
        return served

    def close(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        for e in self.channels:
            e.close()
        self.channels = []


def run_open_loop(server, arrivals, make_action, n_substeps=10):
    """Serve a fixed arrival schedule in real time: arrivals is a list of (t_offset_s, channel)
    sorted by time; make_action(channel, k) gives the k-th request's action for a channel.
    Requests are released when their time comes; the loop serves whatever is pending.
    Returns (completed requests, wall seconds)."""
    t0 = time.perf_counter()
    k_of = collections.Counter()
    nxt = 0
    completed = []
    while nxt < len(arrivals) or server.has_pending():
        now = time.perf_counter() - t0
        while nxt < len(arrivals) and arrivals[nxt][0] <= now:
            t_off, ch = arrivals[nxt]
            server.submit(ch, make_action(ch, k_of[ch]), n_substeps, t_arrival=t0 + t_off)
            k_of[ch] += 1
            nxt += 1
        if server.has_pending():
            completed.extend(server.step_once())
        elif nxt < len(arrivals):
            wait = arrivals[nxt][0] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    return completed, time.perf_counter() - t0
