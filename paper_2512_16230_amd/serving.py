"""Continuous-batching request loop over the C ABI.

Requests (a lattice, a model, a grid, a step count and initial fields) arrive
over time.  At every chunk boundary the server

  1. admits waiting requests in arrival order while their device footprint
     fits the HBM budget (strict FIFO: a request that does not fit blocks the
     ones behind it, so large requests cannot starve);
  2. advances every resident solve by up to ``max_chunk`` steps (never past
     its own step count) with one ``mrtlb_batch_step`` call -- one kernel
     launch per step for each group of solves sharing lattice, model and
     storage, so requests of one group run in the same launch, and a solve
     that finishes inside the chunk drops out of the later launches;
  3. retires the solves that reached their step count: reads their moments
     back, frees their memory and records the latency (arrival -> result on
     the host).

Populations of resident solves stay in HBM between chunks.  ``GpuExecutor`` runs on the
library; ``SimExecutor`` replays the same schedule in simulated time (bytes /
bandwidth) for tests of the scheduling logic without a GPU.
"""

from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import workloads as W

STORE_BYTES = {"fp64": 8, "fp32": 4, "fp32_dev": 4, "fp16_dev": 2, "bf16_dev": 2, "i16_dev": 2, "fp32_dev_f64": 4}
B_OF = {"rD2Q25": 25, "rD2Q13": 13, "rD3Q53": 53, "rD3Q33": 33}


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the window
    card: W.Card
    eq: str
    shape: tuple
    steps: int
    storage: str
    rates: W.Rates
    seed: int
    D0: float = 0.0
    D2: float = 0.0
    adv_u: tuple = (0.0, 0.0, 0.0)
    with_force: bool = False
    payload: dict = None           # rho_or_phi, u, force (filled by the producer)
    payload_error: str = None      # set by the producer if the payload could not be made

    @property
    def nodes(self):
        return int(np.prod(self.shape))


def make_payload(req: Request) -> dict:
    """Initial fields of a request (what a client would send)."""
    card = req.card
    if req.eq == "NCDE":
        return {"rho_or_phi": W.gaussian_hill(card, req.shape), "u": None, "force": None}
    if card.d == 2:
        p, u = W.taylor_green_2d(card, req.shape, 0.05)
        return {"rho_or_phi": 1.0 + p / card.cs2, "u": u, "force": None}
    rho, u = W.taylor_green_3d(card, req.shape, 0.05, 1e-2)
    F = W.sinusoidal_force(card, req.shape, 1e-5, seed=req.seed) if req.with_force else None
    return {"rho_or_phi": rho, "u": u, "force": F}


def request_stream(n, rate, seed=0, storage="i16_dev", mix=(1 / 3, 1 / 3, 1 / 3), steps=(200, 2000),
                   q25=(64, 2048), q13=(128, 1024), q33=(32, 128)):
    """Poisson arrivals at ``rate`` per second mixing rD2Q25 NSE (sides in
    ``q25``), rD2Q13 NCDE (``q13``) and rD3Q33 NSE with a body force
    (``q33``); sides log-uniform, step counts uniform integers in ``steps``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        kind = rng.choice(3, p=np.asarray(mix) / np.sum(mix))
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        if kind == 0:
            side = int(round(np.exp(rng.uniform(np.log(q25[0]), np.log(q25[1])))))
            out.append(Request(i, t, W.Q25_RECT, "NSE_INC", (side, side), nsteps, storage, W.rates_tau(0.8), i))
        elif kind == 1:
            side = int(round(np.exp(rng.uniform(np.log(q13[0]), np.log(q13[1])))))
            wl = W.ncde_hill((4, 4))
            adv = tuple(rng.uniform(-0.05, 0.05, size=2)) + (0.0,)
            out.append(Request(i, t, W.Q13_SQUARE, "NCDE", (side, side), nsteps, storage, wl.rates, i,
                               D0=wl.D0, D2=wl.D2, adv_u=adv))
        else:
            side = int(round(np.exp(rng.uniform(np.log(q33[0]), np.log(q33[1])))))
            out.append(Request(i, t, W.Q33_CUBIC, "NSE_COMP", (side, side, side), nsteps, storage,
                               W.rates_tau(0.8), i, with_force=True))
    return out


def footprint_bytes(req: Request) -> int:
    """Device bytes of a resident request (populations, force, phi history)."""
    b = B_OF[req.card.kind]
    n = req.nodes
    real = 8 if req.storage == "fp64" else 4
    out = 2 * b * n * STORE_BYTES[req.storage]
    if req.with_force:
        out += req.card.d * n * real
    if req.eq == "NCDE":
        out += 2 * n * real
    return out + 4096


# --------------------------------------------------------------------------
# executors
# --------------------------------------------------------------------------

class PinnedPool:
    """Page-locked float64 host buffers from the library (mrtlb_host_alloc),
    reused across requests in power-of-two size classes: uploads from them
    and read-backs into them run at DMA speed instead of through the
    runtime's pageable staging."""

    def __init__(self, H):
        self._H = H
        self._free = {}
        self._all = []
        self._lock = threading.Lock()

    def get(self, n):
        cap = 1 << max(10, int(n - 1).bit_length())
        with self._lock:
            lst = self._free.get(cap)
            b = lst.pop() if lst else None
        if b is None:
            b = self._H.HostBuffer(cap)
            with self._lock:
                self._all.append(b)
        return b

    def put(self, b):
        with self._lock:
            self._free.setdefault(b.n, []).append(b)

    @staticmethod
    def array(b, shape):
        n = int(np.prod(shape))
        return b.array[:n].reshape(shape)

    def close(self):
        with self._lock:
            for b in self._all:
                b.close()
            self._all, self._free = [], {}


class GpuExecutor:
    """Runs solves on the HIP library.  The producer thread stages request
    payloads in page-locked memory together with the flow bounds of the
    int16 storage (``prepare``); results are read back into page-locked
    buffers."""

    def __init__(self, device=0, stream=None, hbm_budget=0, pinned=True):
        from . import _mrtlb as H
        self.H = H
        self.ctx = H.Context(device, stream=stream, hbm_budget=hbm_budget)
        self._lat = {}
        self.pool = PinnedPool(H) if pinned else None

    def prepare(self, req):
        """Producer side: the payload (what a client uploads), its flow
        bounds, and page-locked copies of its fields."""
        p = make_payload(req)
        if req.storage == "i16_dev":
            p["bounds"] = W.flow_bounds(req.eq, p["rho_or_phi"], p["u"], p["force"], req.steps, adv_u=req.adv_u,
                                          cs2=req.card.cs2)
        if self.pool is not None:
            p["_pinned"] = []
            for key in ("rho_or_phi", "u", "force"):
                a = p[key]
                if a is None:
                    continue
                t = self.pool.get(a.size)
                view = self.pool.array(t, a.shape)
                np.copyto(view, a)
                p[key] = view
                p["_pinned"].append(t)
        return p

    def recycle(self, payload):
        if self.pool is not None:
            for t in payload.get("_pinned", ()):
                self.pool.put(t)

    def budget(self):
        return self.ctx.memory()[1]

    def _lattice(self, card):
        if card not in self._lat:
            self._lat[card] = self.H.Lattice(card.kind, card.c, card.cs2, card.free)
        return self._lat[card]

    def footprint(self, req):
        return self.H.footprint(self._lattice(req.card), req.shape, req.storage, req.eq, req.with_force)

    def create(self, req):
        H = self.H
        r = req.rates
        p = req.payload
        ub = db = 0.0
        if req.storage == "i16_dev":
            ub, db = p.get("bounds") or W.flow_bounds(req.eq, p["rho_or_phi"], p["u"], p["force"], req.steps,
                                                       adv_u=req.adv_u, cs2=req.card.cs2)
        md = H.model_desc(req.eq, s0=r.s0, s1=r.s1, s_shear=r.s_shear, s_bulk=r.s_bulk, s3=r.s3, s_high=r.s_h,
                          D0=req.D0, D2=req.D2, adv_u=req.adv_u, u_bound=ub, dev_bound=db)
        s = H.Solve(self.ctx, self._lattice(req.card), md, req.shape, req.storage, has_force=req.with_force)
        s.init_fields(p["rho_or_phi"], p["u"], p["force"])
        return s

    def step(self, handles, counts):
        self.H.batch_step(handles, counts)

    def read(self, handle, req, keep=True):
        """Moments of a finished solve; with keep=False they land in reused
        page-locked buffers and are not returned (the bench discards them)."""
        with_u = req.eq != "NCDE"
        if self.pool is None:
            out = handle.read_moments(with_u=with_u)
            return out if with_u else (out, None)
        tr = self.pool.get(handle.N)
        tu = self.pool.get(handle.d * handle.N) if with_u else None
        r = tr.array[:handle.N]
        u = tu.array[:handle.d * handle.N] if with_u else None
        res = handle.read_moments(out=(r, u))
        if keep:
            res = (res[0].copy(), res[1].copy()) if with_u else (res.copy(), None)
        else:
            res = None
        self.pool.put(tr)
        if tu is not None:
            self.pool.put(tu)
        return res

    def release(self, handle):
        handle.close()

    def now(self):
        return time.perf_counter()

    def close(self):
        if self.pool is not None:
            self.pool.close()
        self.ctx.close()


class SimExecutor:
    """Simulated device: a chunk takes sum(bytes moved) / bandwidth seconds;
    creation and read-back are free.  Handles are the requests."""

    needs_payload = False

    def __init__(self, hbm_budget, bandwidth=5.5e12, fail_on=None):
        self._budget = hbm_budget
        self.bw = bandwidth
        self.t = 0.0
        self.fail_on = fail_on or set()
        self.steps_done = {}

    def budget(self):
        return self._budget

    def footprint(self, req):
        return footprint_bytes(req)

    def create(self, req):
        if req.rid in self.fail_on:
            raise RuntimeError("device error on request %d" % req.rid)
        self.steps_done[req.rid] = 0
        return req

    def step(self, handles, counts):
        moved = sum(2 * B_OF[h.card.kind] * STORE_BYTES[h.storage] * h.nodes * n for h, n in zip(handles, counts))
        self.t += moved / self.bw
        for h, n in zip(handles, counts):
            self.steps_done[h.rid] += n

    def read(self, handle, req, keep=True):
        return self.steps_done[handle.rid], None

    def release(self, handle):
        pass

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)

    def close(self):
        pass


# --------------------------------------------------------------------------
# the loop
# --------------------------------------------------------------------------

@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    nodes: int
    steps: int
    value: object = None
    error: str = None

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class ServeStats:
    results: list = field(default_factory=list)
    wall: float = 0.0
    max_resident: int = 0
    max_bytes: int = 0
    chunks: int = 0
    t_create: float = 0.0      # host time in admission (allocation, upload, init kernel)
    t_step: float = 0.0        # host time in batched steps (includes the device time)
    t_read: float = 0.0        # host time in read-back and release
    t_wait: float = 0.0        # time waiting for payloads or arrivals

    def latencies(self):
        return np.array([r.latency for r in self.results if r.error is None])

    def summary(self):
        lat = self.latencies()
        work = sum(r.nodes * r.steps for r in self.results if r.error is None)
        return {"requests": len(self.results), "failed": sum(r.error is not None for r in self.results),
                "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_s": float(lat.mean()) if len(lat) else None,
                "mlups": work / self.wall / 1e6 if self.wall > 0 else None,
                "wall_s": self.wall, "max_resident": self.max_resident, "max_bytes": self.max_bytes,
                "chunks": self.chunks, "t_create_s": self.t_create, "t_step_s": self.t_step,
                "t_read_s": self.t_read, "t_wait_s": self.t_wait}


class Server:
    def __init__(self, executor, max_chunk=64, keep_values=False, lookahead=32, producers=4):
        self.ex = executor
        self.max_chunk = max_chunk
        self.keep_values = keep_values
        self.lookahead = lookahead
        self.producers = producers

    def _start_producer(self, reqs):
        """Fill request payloads ahead of their arrival (the clients' uploads)
        with ``producers`` threads, at most ``lookahead`` requests ahead of
        admission."""
        events = {r.rid: threading.Event() for r in reqs}
        if not getattr(self.ex, "needs_payload", True):
            for e in events.values():
                e.set()
            return events, None
        room = threading.Semaphore(self.lookahead)
        nxt = iter(reqs)
        take = threading.Lock()

        def produce():
            while True:
                room.acquire()
                with take:
                    r = next(nxt, None)
                if r is None:
                    room.release()
                    return
                try:
                    if r.payload is None:
                        prepare = getattr(self.ex, "prepare", None)
                        r.payload = prepare(r) if prepare is not None else make_payload(r)
                except Exception as e:       # the request fails alone; admission must not wait forever
                    r.payload = None
                    r.payload_error = "payload: %s: %s" % (type(e).__name__, e)
                finally:
                    events[r.rid].set()

        for _ in range(self.producers):
            threading.Thread(target=produce, daemon=True).start()
        return events, room

    def run(self, requests, real_time=True):
        ex = self.ex
        reqs = sorted(requests, key=lambda r: r.arrival)
        events, room = self._start_producer(reqs)
        budget = ex.budget()
        pending = deque(reqs)
        active = []          # [handle, req, remaining, admitted_at, bytes]
        used = 0
        stats = ServeStats()
        t0 = ex.now()
        clock = (lambda: ex.now() - t0)

        def consumed(req):
            recycle = getattr(ex, "recycle", None)
            if recycle is not None and req.payload is not None:
                recycle(req.payload)
            req.payload = None
            if room is not None:
                room.release()

        while pending or active:
            now = clock()
            # 1. admission, strict FIFO, by footprint
            while pending and pending[0].arrival <= now:
                req = pending[0]
                fp = ex.footprint(req)
                if fp > budget:
                    pending.popleft()
                    events[req.rid].wait()
                    consumed(req)
                    stats.results.append(Result(req.rid, req.arrival, now, clock(), req.nodes, 0,
                                                error="footprint %d B exceeds the HBM budget" % fp))
                    continue
                if used + fp > budget:
                    break
                pending.popleft()
                tw = clock()
                events[req.rid].wait()
                tc = clock()
                stats.t_wait += tc - tw
                if getattr(req, "payload_error", None):
                    consumed(req)
                    stats.results.append(Result(req.rid, req.arrival, now, clock(), req.nodes, 0,
                                                error=req.payload_error))
                    continue
                try:
                    h = ex.create(req)
                except Exception as e:           # the failing request only
                    consumed(req)
                    stats.results.append(Result(req.rid, req.arrival, now, clock(), req.nodes, 0, error=str(e)))
                    continue
                consumed(req)
                stats.t_create += clock() - tc
                used += fp
                active.append([h, req, req.steps, now, fp])
            stats.max_resident = max(stats.max_resident, len(active))
            stats.max_bytes = max(stats.max_bytes, used)
            if not active:
                if pending:
                    nxt = pending[0].arrival
                    stats.t_wait += max(0.0, nxt - clock())
                    if real_time:
                        time.sleep(max(0.0, min(nxt - clock(), 0.05)))
                    else:
                        ex.sleep_until(t0 + nxt)
                continue
            # 2. one chunk for every resident solve
            counts = [min(self.max_chunk, a[2]) for a in active]
            ts = clock()
            ex.step([a[0] for a in active], counts)
            stats.t_step += clock() - ts
            stats.chunks += 1
            for a, k in zip(active, counts):
                a[2] -= k
            # 3. retire
            tr = clock()
            still = []
            for a in active:
                if a[2] == 0:
                    h, req, _, adm, fp = a
                    val = ex.read(h, req, keep=self.keep_values)
                    ex.release(h)
                    used -= fp
                    stats.results.append(Result(req.rid, req.arrival, adm, clock(), req.nodes, req.steps,
                                                value=val if self.keep_values else None))
                else:
                    still.append(a)
            active = still
            stats.t_read += clock() - tr
        stats.wall = clock()
        stats.results.sort(key=lambda r: r.rid)
        return stats
