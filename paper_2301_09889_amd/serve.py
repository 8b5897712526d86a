"""Request loop for many RL workers: env-step requests on resident channels, served with
continuous batching (the paper's EVOLVE request, §3.3, from many agents at once).

* Every channel's flow state stays on the device.  A channel is admitted while the summed HBM
  footprint (chan_env_footprint_bytes) of the admitted channels fits the server's budget;
  otherwise it waits (``admit(..., wait=True)``) and is admitted as soon as released channels
  have freed enough memory.
* A request carries its own output tensors (observation, wall shear, drag), written by the
  GPU; nothing of one request is overwritten by the next.
* The loop is asynchronous.  ``launch`` queues, each on the next of a few streams (lanes), one
  batch call per substep count and grid shape for the channels that have a pending request and
  no call in flight, and returns at once; ``poll`` finishes the calls whose work has ended.  Requests that arrive
  while calls are on the GPU are launched on another lane right away, so their work overlaps
  the calls in flight on the device.  A channel's requests run one at a time, in order (in RL
  the next action depends on the last observation anyway).
* Each channel computes exactly what it would alone (the batched launches run the same
  per-channel code), so a result does not depend on what else was in the mix.

A request's latency runs from its arrival to the poll that saw its call finished.
"""
import collections
import time

from . import binding as b


class Request:
    __slots__ = ("channel", "action", "n_substeps", "t_arrival", "t_launch", "t_done", "code",
                 "obs", "tau_w", "drag", "lane")

    def __init__(self, channel, action, n_substeps, t_arrival):
        self.channel = channel
        self.action = action
        self.n_substeps = n_substeps
        self.t_arrival = t_arrival
        self.t_launch = None
        self.t_done = None
        self.code = None
        self.obs = self.tau_w = self.drag = None
        self.lane = None


class ChannelServer:
    """Resident channels behind one request queue.

    hbm_budget: bytes the channels' device allocations may take together.  lanes: streams the
    batch calls are spread over (calls on different lanes run concurrently on the device).
    split_by_grid: one call per grid shape (and substep count), so that small channels cycle
    through short calls while a large channel's long call is in flight on another lane.
    Channel ids are never reused; ``channels`` maps the admitted ones to their ChanEnv.
    """

    def __init__(self, hbm_budget, lanes=2, split_by_grid=True):
        import torch
        self.split_by_grid = split_by_grid
        self.torch = torch
        self.budget = int(hbm_budget)
        self.used = 0
        self.channels = {}
        self.footprint = {}
        self.batch = None
        self.in_batch = set()
        self.streams = [torch.cuda.Stream() for _ in range(max(1, lanes))]
        self.lane = 0
        self.pending = collections.defaultdict(collections.deque)
        self.inflight = []              # (ChanCall, [Request])
        self.busy = set()               # channels with a call in flight
        self.to_release = set()
        self.waiting = collections.deque()   # (id, grid, opts, seed, need)
        self.done = []
        self.rejected_channels = 0
        self.next_id = 0

    # ---- admission and release ----
    def _create(self, cid, grid, opts, seed, need):
        env = b.ChanEnv(grid, opts)
        env.reset(seed)
        self.channels[cid] = env
        self.footprint[cid] = need
        self.used += need

    def _ensure_batch(self):
        """The batch holds every admitted channel: built at the first launch over the channels
        admitted so far (each grid shape's plane-pass tiling tuned on all its channels), later
        admissions join it."""
        if self.batch is None:
            self.batch = b.ChanBatch(list(self.channels.values()))
            self.in_batch = set(self.channels)
        for cid, env in self.channels.items():
            if cid not in self.in_batch:
                self.batch.add(env)
                self.in_batch.add(cid)

    def admit(self, grid, opts, seed, wait=False):
        """Create and reset a channel if its footprint fits the remaining budget; returns its id.
        If it does not fit: None, or with wait=True an id whose channel is created when enough
        memory has been released (``is_admitted`` tells)."""
        need = b.chan_env_footprint_bytes(grid, opts)
        if need == 0:
            raise ValueError("invalid grid or options")
        if need > self.budget:
            raise ValueError("channel larger than the whole budget")
        cid = self.next_id
        if self.used + need <= self.budget and not self.waiting:
            self.next_id += 1
            self._create(cid, grid, opts, seed, need)
            return cid
        if not wait:
            self.rejected_channels += 1
            return None
        self.next_id += 1
        self.waiting.append((cid, grid, opts, seed, need))
        return cid

    def is_admitted(self, cid):
        return cid in self.channels

    def _admit_waiting(self):
        while self.waiting and self.used + self.waiting[0][4] <= self.budget:
            cid, grid, opts, seed, need = self.waiting.popleft()
            self._create(cid, grid, opts, seed, need)

    def release(self, cid):
        """Remove a channel and free its memory (after its call in flight, if any, finishes);
        waiting channels that now fit are admitted.  Its pending requests are dropped."""
        if cid not in self.channels:
            raise KeyError(cid)
        self.pending.pop(cid, None)
        if cid in self.busy:
            self.to_release.add(cid)
            return
        env = self.channels.pop(cid)
        if cid in self.in_batch:
            self.batch.remove(env)
            self.in_batch.discard(cid)
        env.close()
        self.used -= self.footprint.pop(cid)
        self._admit_waiting()

    # ---- requests ----
    def submit(self, channel, action, n_substeps, t_arrival=None):
        """Queue an env step of a channel (action: float64 device tensor (nz, nx) or None)."""
        if channel not in self.channels and not any(w[0] == channel for w in self.waiting):
            raise KeyError(channel)
        r = Request(channel, action, n_substeps, time.perf_counter() if t_arrival is None else t_arrival)
        self.pending[channel].append(r)
        return r

    def has_pending(self):
        return any(self.pending[c] for c in self.pending) or bool(self.inflight)

    def launch(self):
        """Queue one call per substep count (and grid shape, with split_by_grid) for the admitted
        channels with a pending request and no call in flight, each call on the next lane.
        Returns the number of requests launched."""
        torch = self.torch
        heads = [q[0] for c, q in self.pending.items() if q and c in self.channels and c not in self.busy]
        if not heads:
            return 0
        self._ensure_batch()
        by_n = collections.defaultdict(list)
        for r in heads:
            g = self.channels[r.channel].grid
            key = (r.n_substeps, (g.nx, g.ny, g.nz) if self.split_by_grid else ())
            by_n[key].append(r)
        for (n_sub, _), reqs in sorted(by_n.items()):
            reqs.sort(key=lambda r: r.channel)
            lane = self.lane
            self.lane = (self.lane + 1) % len(self.streams)
            st = self.streams[lane]
            envs = [self.channels[r.channel] for r in reqs]
            with torch.cuda.stream(st):   # outputs allocated for the stream that writes them
                for r, e in zip(reqs, envs):
                    r.obs = torch.empty_like(e.obs)
                    r.tau_w = torch.empty_like(e.tau_w)
                    r.drag = torch.empty_like(e.drag)
            t = time.perf_counter()
            call = self.batch.launch(envs, [r.action for r in reqs], n_sub, [r.obs for r in reqs],
                                     [r.tau_w for r in reqs], [r.drag for r in reqs], stream=st)
            for r in reqs:
                r.t_launch = t
                r.lane = lane
                self.pending[r.channel].popleft()
                self.busy.add(r.channel)
            self.inflight.append((call, reqs))
        return len(heads)

    def poll(self, block=False):
        """Finish the calls whose work has ended (with block=True: wait for all in flight).
        Returns the requests completed."""
        served, keep = [], []
        for call, reqs in self.inflight:
            if block or call.done():
                codes = call.finish()
                t = time.perf_counter()
                for r, code in zip(reqs, codes):
                    r.code = code
                    r.t_done = t
                    self.busy.discard(r.channel)
                served.extend(reqs)
            else:
                keep.append((call, reqs))
        self.inflight = keep
        for cid in list(self.to_release):
            if cid not in self.busy:
                self.to_release.discard(cid)
                self.release(cid)
        self.done.extend(served)
        return served

    def step_once(self):
        """Launch what can be launched and wait for every call in flight; returns the requests
        completed (the synchronous form of one loop iteration)."""
        self.launch()
        return self.poll(block=True)

    def close(self):
        self.poll(block=True)
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        for e in self.channels.values():
            e.close()
        self.channels = {}


def run_open_loop(server, arrivals, make_action, n_substeps=10):
    """Serve a fixed arrival schedule in real time: arrivals is a list of (t_offset_s, channel)
    sorted by time; make_action(channel, k) gives the k-th request's action for a channel.
    Requests are submitted when their time comes and launched at once if their channel is
    free; finished calls are polled without blocking.  Returns (completed requests, wall s)."""
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
        launched = server.launch()
        got = server.poll()
        completed.extend(got)
        if not launched and not got:
            if server.inflight:
                time.sleep(0.0001)
            elif nxt < len(arrivals):
                wait = arrivals[nxt][0] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
    return completed, time.perf_counter() - t0
