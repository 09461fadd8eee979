"""Continuous-batching ensemble server for the ES-DGSEM stepper.

Requests (ensemble members) arrive over time, each a mesh of its own size
and order with a seeded initial state and a number of LSRK(5,4) steps.  The
server

* admits arrived requests while their device footprint fits the HBM budget
  (FIFO with backfill: a request that does not fit does not block smaller
  ones behind it), keeping every member's state resident on the device; a
  member's mesh, initial state and time step are prepared off the
  scheduler's thread, which meanwhile keeps launching the buckets' steps;
* groups members by (N, precision) into buckets; each bucket is one packed
  launch per stage over all its members (``esdg.Pack``: a device descriptor
  table, one step = 5 packed stage kernels + a parity flip captured in a
  HIP graph) on its own stream, so buckets overlap on the device;
* advances each bucket on its own: as soon as a bucket's step completes, its
  members' latencies are recorded, finished members retire (freeing memory
  for the queue), new members join, and the bucket's next step is launched
  -- a bucket of small members is not held back by a bucket of large ones;
* picks elements per workgroup per (N, precision) from an autotuner that
  times the compiled variants and caches the choice in JSON;
* reports per-member step latency (completion of step s minus completion of
  step s-1, or of the admission for s = 1) as p50/p99 over all member-steps,
  aggregate DOF*RHS/s (sum of nodes x 5 x steps / makespan), queue waits and
  end-to-end latency.

The scheduler is written against a small executor interface: ``GpuExecutor``
drives the library; ``FakeExecutor`` simulates step durations from a cost
model so that admission, packing, eviction and the statistics are testable
on a machine without a GPU.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import json
import math
import os
import threading
import time
import weakref
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import workloads as W

FP64, FP32_MIXED = 0, 1

# Packed stepping runs the fused kernels, which cover orders up to 8; the
# server rejects requests of higher order.
PACK_MAX_N = 8


class NonPhysicalState(RuntimeError):
    """A member met rho <= 0, p <= 0 or NaN; it was evicted, the others run on."""


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                  # "bubble" | "channel"
    K: Tuple[int, int, int]
    N: int
    precision: int             # FP64 | FP32_MIXED
    seed: int
    steps: int
    arrival: float = 0.0       # seconds after the start of the run
    # failure-isolation tests: write a negative density at this node index
    # (element 0, flat node index) of the initial state
    nonphysical_node: Optional[int] = None

    def spec(self) -> W.MeshSpec:
        if self.kind == "bubble":
            return W.rising_bubble(N=self.N, K=self.K).mesh
        if self.kind == "channel":
            return W.channel(N=self.N, K=self.K).mesh
        raise ValueError(self.kind)

    @property
    def nodes(self) -> int:
        return self.K[0] * self.K[1] * self.K[2] * (self.N + 1) ** 3

    @property
    def key(self):
        return (self.N, self.precision)


def footprint_bytes(req: Request) -> int:
    """Steady device footprint of a member: two state buffers and dq
    (3 x 40 B per node), the mesh's reduction partials (4 doubles per 256
    nodes), and for FP32-mixed the FP32 reference and R(q_r) momentum
    (20 B per node)."""
    n = req.nodes
    b = 120 * n + 4 * 8 * (n // 256 + 1) + 4096
    if req.precision == FP32_MIXED:
        b += 20 * n
    return b


def request_stream(n=96, seed=0, mean_interarrival=0.05, steps=50, kmin=8, kmax=40,
                   orders=(3, 4, 5, 7)):
    """Seeded ensemble request stream: Poisson arrivals, kind bubble/channel
    with probability 1/2, elements per dimension ~ U{kmin..kmax} independently,
    N uniform over `orders`, FP64 or FP32-mixed with probability 1/2, seed =
    request id."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(mean_interarrival))
        kind = "bubble" if rng.uniform() < 0.5 else "channel"
        K = tuple(int(k) for k in rng.integers(kmin, kmax + 1, size=3))
        N = int(rng.choice(orders))
        prec = FP32_MIXED if rng.uniform() < 0.5 else FP64
        out.append(Request(i, kind, K, N, prec, i, steps, t))
    return out


# ---------------------------------------------------------------------------
# Autotuner
# ---------------------------------------------------------------------------

class Autotuner:
    """Elements per workgroup per (N, precision), chosen by timing the
    compiled variants on a bubble mesh of about `target_nodes` nodes and
    cached in a JSON file."""

    def __init__(self, cache_path: Optional[str] = None, target_nodes: float = 2.0e6):
        self.cache_path = cache_path
        self.target_nodes = target_nodes
        self.table: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = json.load(f)

    @staticmethod
    def _key(N, precision):
        return f"N{N}_{'mixed' if precision == FP32_MIXED else 'fp64'}"

    def epw(self, N: int, precision: int) -> int:
        k = self._key(N, precision)
        if k not in self.table:
            self.table[k] = self.tune(N, precision)
            self.save()
        return int(self.table[k]["epw"])

    def save(self):
        if self.cache_path:
            d = os.path.dirname(os.path.abspath(self.cache_path))
            os.makedirs(d, exist_ok=True)
            with open(self.cache_path, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)

    def tune(self, N: int, precision: int, reps: int = 5) -> dict:
        import torch
        from . import esdg
        opts = esdg.epw_options(N, precision)
        k = max(2, int(round((self.target_nodes / (N + 1) ** 3) ** (1.0 / 3.0))))
        req = Request(-1, "bubble", (k, k, k), N, precision, 0, 1)
        timings = {}
        for e in opts:
            m, q, _ = _make_member_mesh(req, epw=e)
            r = torch.empty_like(q)
            for _ in range(2):
                m.rhs(q, r)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                m.rhs(q, r)
            b.record()
            torch.cuda.synchronize()
            timings[str(e)] = a.elapsed_time(b) / reps
            m.close()
            del q, r
        best = min(timings, key=timings.get)
        return {"epw": int(best), "ms": timings, "nodes": req.nodes}


def _make_member_mesh(req: Request, epw: int = 0, retire=None):
    """Library mesh, initial state (built in device memory) and the FP32-mixed
    reference arrays of a request.  The FP64 mesh that supplies the node
    coordinates of an FP32-mixed request is destroyed here, or handed to
    `retire(mesh)` to be destroyed later (destroying a mesh waits for the
    device)."""
    import torch
    from . import esdg
    spec = req.spec()
    if req.precision == FP32_MIXED:
        probe = esdg.Mesh(spec, epw=0)
        xyz = probe.coords()
        if retire is None:
            probe.close()
        else:
            retire(probe)
        rr, pr = W.reference_state(xyz, spec, req.kind)
        m = esdg.Mesh(spec, precision=esdg.FP32_MIXED, ref_rho=rr.contiguous(),
                      ref_p=pr.contiguous(), epw=epw)
        m._refs = None  # the library copied the reference at creation
    else:
        m = esdg.Mesh(spec, epw=epw)
        xyz = m.coords()
    q = W.make_state(req.kind, xyz, spec, seed=req.seed).contiguous()
    if req.nonphysical_node is not None:
        q[0, 0, req.nonphysical_node] = -1.0
    return m, q, xyz


# ---------------------------------------------------------------------------
# Executors
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Member:
    req: Request
    footprint: int
    handle: object = None          # executor's per-member object
    admitted: float = 0.0          # host time of admission
    last_done: float = 0.0         # device time of the last completed step (or admission)
    steps_done: int = 0
    latencies: List[float] = dataclasses.field(default_factory=list)
    finished: float = 0.0
    error: Optional[Exception] = None  # set when the member was evicted


class GpuExecutor:
    """Drives libesdg: one Pack and one stream per (N, precision) bucket."""

    def __init__(self, autotuner: Optional[Autotuner] = None, keep_results: bool = False,
                 admission_threads: int = 2):
        import torch
        self.torch = torch
        self.autotuner = autotuner or Autotuner()
        self.keep_results = keep_results
        self.buckets: Dict[tuple, dict] = {}
        self.t0_host = time.perf_counter()
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev0.record()
        torch.cuda.synchronize()
        # host seconds spent per activity, and device seconds of the steps
        self.times = {"admission_s": 0.0, "set_members_s": 0.0, "launch_and_capture_s": 0.0,
                      "flag_reads_s": 0.0, "release_s": 0.0, "device_step_s": 0.0}
        # meshes of released members, destroyed in batches: destroying one
        # synchronises its stream and frees device memory, which waits for
        # the device, so it is done when the budget needs the bytes or when
        # no step is in flight
        self._retired: List[object] = []
        self._retired_bytes = 0
        self._lock = threading.Lock()
        # admissions run on worker threads: building a member's mesh and
        # state and reading its time step wait for the device, and the
        # scheduler's thread keeps launching steps meanwhile
        self.device = torch.cuda.current_device()
        self._pool = concurrent.futures.ThreadPoolExecutor(
            max_workers=max(1, int(admission_threads)), thread_name_prefix="esdg-admission")
        # the admission threads end with the executor
        self._pool_finalizer = weakref.finalize(self, self._pool.shutdown, wait=False)
        # each admission thread's work goes to a stream of its own (not the
        # null stream, whose implicit ordering with other streams would
        # invalidate a graph capture running on the scheduler's thread)
        self._tls = threading.local()

    def now(self) -> float:
        return time.perf_counter() - self.t0_host

    def close(self):
        """Wait for the admission threads, end them, and destroy the meshes of
        released members."""
        self._pool.shutdown(wait=True)
        self._pool_finalizer.detach()
        self.flush_retired()

    def _dev_time(self, ev) -> float:
        return self.ev0.elapsed_time(ev) * 1e-3

    def admit_async(self, req: Request) -> concurrent.futures.Future:
        """Prepare a member on an admission thread; the future's result is
        what `admit` returns.  The elements per workgroup are looked up (and,
        the first time for an (N, precision), tuned) on the calling thread,
        which also captures the packs' graphs: tuning synchronises the
        device."""
        epw = self.autotuner.epw(req.N, req.precision)
        return self._pool.submit(self.admit, req, epw)

    def admit(self, req: Request, epw: Optional[int] = None):
        """Mesh, initial state, ping-pong and dq buffers and time step of a
        new member, complete on the device when this returns."""
        torch = self.torch
        t0 = time.perf_counter()
        if epw is None:
            epw = self.autotuner.epw(req.N, req.precision)
        torch.cuda.set_device(self.device)
        stream = getattr(self._tls, "stream", None)
        if stream is None:
            stream = self._tls.stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = self._admit(req, epw)
        with self._lock:
            self.times["admission_s"] += time.perf_counter() - t0
        return out

    def _admit(self, req: Request, epw: int):
        torch = self.torch
        m, q, xyz = _make_member_mesh(req, epw=epw, retire=self._retire_mesh)
        del xyz
        try:
            dt = m.cfl_dt(q, 0.5)
        except Exception:
            # a state without a finite wave speed still enters and is evicted
            # by its flag after its first step; its time step is immaterial
            dt = 1e-3
        q1 = torch.empty_like(q)
        dq = torch.zeros_like(q)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        ev.synchronize()
        return ({"mesh": m, "bufs": [q, q1], "dq": dq, "dt": dt, "parity": 0, "ready": ev},
                self._dev_time(ev))

    def set_bucket(self, key, members: List[Member]):
        from . import esdg
        torch = self.torch
        t0 = time.perf_counter()
        b = self.buckets.get(key)
        if b is None:
            stream = torch.cuda.Stream()
            b = {"stream": stream, "pack": None}
            self.buckets[key] = b
        with torch.cuda.stream(b["stream"]):
            if b["pack"] is None:
                b["pack"] = esdg.Pack(b["stream"])
            # initial states are written on the admission thread's stream:
            # the bucket stream waits for each member's admission event (a
            # no-op once it has completed, as it has when admit returned)
            hs = [mb.handle for mb in members]
            for h in hs:
                if h.get("ready") is not None:
                    b["stream"].wait_event(h["ready"])
                    h["ready"] = None
            b["pack"].set_members([h["mesh"] for h in hs], [h["bufs"][0] for h in hs],
                                  [h["bufs"][1] for h in hs], [h["dq"] for h in hs],
                                  [h["dt"] for h in hs], [h["parity"] for h in hs])
        b["members"] = list(members)
        # pinned host buffer that each step's flags are copied into (the
        # copy is enqueued behind the step, so reading it needs no sync)
        if b.get("hflags") is None or b["hflags"].numel() < len(members):
            b["hflags"] = torch.zeros(max(8, 2 * len(members)), dtype=torch.int32,
                                      pin_memory=True)
        self.times["set_members_s"] += time.perf_counter() - t0

    def drop_bucket(self, key):
        b = self.buckets.pop(key, None)
        if b and b["pack"] is not None:
            b["pack"].close()

    def launch_step(self, key):
        torch = self.torch
        t0 = time.perf_counter()
        b = self.buckets[key]
        with torch.cuda.stream(b["stream"]):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(b["stream"])
            b["pack"].step(1)  # the first step after set_members captures the graph
            b["pack"].flags_async(b["hflags"])
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(b["stream"])
        for mb in b["members"]:
            mb.handle["parity"] ^= 1
        b["ev_start"] = ev0
        self.times["launch_and_capture_s"] += time.perf_counter() - t0
        return ev

    def failed_members(self, key) -> List[Member]:
        """Members of the bucket's completed step whose own non-physical flag
        is set (the flags were gathered, and cleared, behind the step; its
        completion event covers the copy, so nothing waits here)."""
        t0 = time.perf_counter()
        b = self.buckets[key]
        if b.get("ev_start") is not None:
            self.times["device_step_s"] += b["ev_start"].elapsed_time(b["ev_done"]) * 1e-3 \
                if b.get("ev_done") is not None else 0.0
        flags = b["hflags"][:len(b["members"])].tolist()
        self.times["flag_reads_s"] += time.perf_counter() - t0
        return [mb for mb, f in zip(b["members"], flags) if f]

    def poll(self, tokens: Dict[tuple, object], until: Optional[float] = None) -> Dict[tuple, float]:
        """Device completion times of the in-flight steps that have finished;
        waits until at least one has, or until host time `until`."""
        while True:
            out = {}
            for key, ev in tokens.items():
                if ev.query():
                    out[key] = self._dev_time(ev)
                    self.buckets[key]["ev_done"] = ev
            if out or (until is not None and self.now() >= until):
                return out
            time.sleep(5e-5)

    def release(self, mb: Member, keep: bool = True):
        t0 = time.perf_counter()
        h = mb.handle
        result = None
        if self.keep_results and keep:
            result = h["bufs"][h["parity"]].cpu().numpy()
        self._retire_mesh(h["mesh"])
        mb.handle = None
        self.times["release_s"] += time.perf_counter() - t0
        return result

    def _retire_mesh(self, m):
        with self._lock:
            self._retired.append(m)
            self._retired_bytes += m.footprint

    def retired_bytes(self) -> int:
        """Device bytes still held by the meshes of released members (and by
        the coordinate meshes of admitted FP32-mixed members)."""
        return self._retired_bytes

    def flush_retired(self):
        """Destroy the meshes of released members."""
        with self._lock:
            ms, self._retired, self._retired_bytes = self._retired, [], 0
        if not ms:
            return
        t0 = time.perf_counter()
        for m in ms:
            m.close()
        self.times["release_s"] += time.perf_counter() - t0


class FakeExecutor:
    """Simulated device: a step of a bucket needs overhead + sum over its
    members of nodes x cost(N, precision) of device time; the steps in flight
    share the device equally (processor sharing, as concurrent streams share
    the CUs).  Time is virtual."""

    def __init__(self, cost_per_node=None, overhead=20e-6, admit_cost=1e-3, fail_on=None,
                 nonphysical_on=None, retire_fraction=0.0):
        self.cost = cost_per_node or (lambda N, prec: 5 * 1e-10 * (1.0 if prec == FP64 else 0.8))
        self.overhead = overhead
        self.admit_cost = admit_cost
        self.clock = 0.0
        self.running: Dict[tuple, float] = {}   # bucket -> remaining device time
        self.finished: Dict[tuple, float] = {}  # bucket -> completion time
        self.buckets: Dict[tuple, List[Member]] = {}
        self.fail_on = fail_on or set()
        # request id -> step (1-based) after which its flag reads non-physical
        self.nonphysical_on = dict(nonphysical_on or {})
        self.times = {}
        # device bytes: live members, and the part of released members'
        # footprints (retire_fraction) held until flush_retired, as the GPU
        # executor holds released meshes; peak_bytes is their largest sum
        self.retire_fraction = retire_fraction
        self.live_bytes = self.retired = self.peak_bytes = 0
        self.flushes = 0

    def now(self) -> float:
        return self.clock

    def _run_until(self, t):
        while self.running and self.clock < t:
            n = len(self.running)
            step = min(self.running.values()) * n
            if self.clock + step > t:
                for k in self.running:
                    self.running[k] -= (t - self.clock) / n
                self.clock = t
                return
            self.clock += step
            least = min(self.running.values())
            for k in list(self.running):
                self.running[k] -= least
                if self.running[k] <= 1e-15:
                    del self.running[k]
                    self.finished[k] = self.clock
        self.clock = max(self.clock, t)

    def advance_to(self, t):
        self._run_until(t)

    def admit(self, req: Request):
        if req.rid in self.fail_on:
            raise RuntimeError(f"simulated failure admitting request {req.rid}")
        self._run_until(self.clock + self.admit_cost)
        self.live_bytes += footprint_bytes(req)
        self.peak_bytes = max(self.peak_bytes, self.live_bytes + self.retired)
        return {"parity": 0}, self.clock

    def admit_async(self, req: Request) -> concurrent.futures.Future:
        """Admission completes at once (its cost advances the virtual clock)."""
        fut = concurrent.futures.Future()
        try:
            fut.set_result(self.admit(req))
        except Exception as ex:  # noqa: BLE001 -- handed to the scheduler
            fut.set_exception(ex)
        return fut

    def set_bucket(self, key, members):
        self.buckets[key] = list(members)

    def drop_bucket(self, key):
        self.buckets.pop(key, None)

    def launch_step(self, key):
        ms = self.buckets[key]
        self.running[key] = self.overhead + sum(mb.req.nodes * self.cost(*key) for mb in ms)
        return key

    def poll(self, tokens, until=None):
        while True:
            done = {k: self.finished.pop(k) for k in list(tokens) if k in self.finished}
            if done:
                return done
            if not self.running:
                return {}
            n = len(self.running)
            t_next = self.clock + min(self.running.values()) * n
            if until is not None and until < t_next:
                self._run_until(until)
                return {k: self.finished.pop(k) for k in list(tokens) if k in self.finished}
            self._run_until(t_next)

    def failed_members(self, key):
        return [mb for mb in self.buckets.get(key, [])
                if mb.req.rid in self.nonphysical_on
                and mb.steps_done + 1 >= self.nonphysical_on[mb.req.rid]]

    def release(self, mb, keep: bool = True):
        fp = footprint_bytes(mb.req)
        self.live_bytes -= fp
        self.retired += int(self.retire_fraction * fp)
        return None

    def retired_bytes(self) -> int:
        return self.retired

    def flush_retired(self):
        if self.retired:
            self.flushes += 1
        self.retired = 0


# ---------------------------------------------------------------------------
# Scheduler
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class RunStats:
    n_requests: int
    n_completed: int
    n_rejected: int
    makespan_s: float
    aggregate_dof_rhs_per_s: float
    step_latency_p50_ms: float
    step_latency_p99_ms: float
    queue_wait_p50_ms: float
    queue_wait_p99_ms: float
    e2e_latency_mean_s: float
    peak_footprint_bytes: int
    hbm_budget_bytes: int
    bucket_steps: int
    max_concurrent_members: int
    buckets_seen: int
    n_failed: int = 0
    time_breakdown: Optional[dict] = None

    def as_dict(self):
        return dataclasses.asdict(self)


class RequestHandle:
    """What `Server.submit` returns: the request's final state (host array,
    when the executor keeps results) and its own latency figures once a
    `Server.run_until_idle` call has served it."""

    def __init__(self, server: "Server", req: Request):
        self._server = server
        self.req = req

    def done(self) -> bool:
        """True once the request has completed or failed."""
        mb = self._server.members.get(self.req.rid)
        return mb is not None and (mb.steps_done >= self.req.steps or mb.error is not None)

    def error(self) -> Optional[Exception]:
        """The error that evicted the request (e.g. NonPhysicalState), or None."""
        mb = self._server.members.get(self.req.rid)
        return None if mb is None else mb.error

    def result(self):
        if not self.done():
            raise RuntimeError(f"request {self.req.rid} has not completed "
                               "(call Server.run_until_idle)")
        err = self.error()
        if err is not None:
            raise err
        return self._server.results.get(self.req.rid)

    def stats(self) -> dict:
        if not self.done():
            raise RuntimeError(f"request {self.req.rid} has not completed")
        mb = self._server.members[self.req.rid]
        if mb.error is not None:
            raise mb.error
        lat = np.array(mb.latencies)
        return {"steps": mb.steps_done, "queue_wait_s": mb.admitted - self.req.arrival,
                "e2e_latency_s": mb.finished - self.req.arrival,
                "step_latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
                "step_latency_p99_ms": float(np.percentile(lat, 99) * 1e3)}


class Server:
    """Continuous-batching ensemble server.  Either hand `run` a whole
    request stream with arrival times, or `submit` requests one by one and
    call `run_until_idle`; `stats` returns the figures of the last run."""

    def __init__(self, hbm_budget_bytes: int, executor=None, autotuner: Optional[Autotuner] = None):
        self.budget = int(hbm_budget_bytes)
        self.ex = executor if executor is not None else GpuExecutor(autotuner)
        self.results: Dict[int, object] = {}
        self.members: Dict[int, Member] = {}
        self._submitted: List[Request] = []
        self._last: Optional[RunStats] = None

    def submit(self, req: Request) -> RequestHandle:
        """Queue a request (its `arrival` offset, in seconds after the start
        of the next `run_until_idle`, is kept; 0 = at once)."""
        if req.rid in self.members or any(r.rid == req.rid for r in self._submitted):
            raise ValueError(f"request id {req.rid} already submitted")
        self._submitted.append(req)
        return RequestHandle(self, req)

    def run_until_idle(self, realtime: bool = True) -> RunStats:
        """Serve every submitted request to completion."""
        reqs, self._submitted = self._submitted, []
        return self.run(reqs, realtime=realtime)

    def stats(self) -> dict:
        return self._last.as_dict() if self._last is not None else {}

    def run(self, requests: List[Request], realtime: bool = True) -> RunStats:
        """Serve the stream until every request has completed (or was
        rejected for exceeding the whole budget)."""
        ex = self.ex
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: List[Request] = []
        active: Dict[tuple, List[Member]] = {}
        dirty = set()
        used = peak = 0
        rejected = 0
        done: List[Member] = []
        failed: List[Member] = []
        steps_launched = max_conc = 0
        buckets_seen = set()
        retired = getattr(ex, "retired_bytes", lambda: 0)
        flush = getattr(ex, "flush_retired", lambda: None)
        inflight: Dict[tuple, object] = {}      # bucket -> completion token of its step
        stepping: Dict[tuple, List[Member]] = {}  # bucket -> members of that step
        admitting: List[tuple] = []             # (future, request, footprint)
        t_start = ex.now()
        while pending or queue or admitting or any(active.values()) or inflight:
            now = ex.now() - t_start
            while pending and pending[0].arrival <= now:
                r = pending.pop(0)
                if footprint_bytes(r) > self.budget or r.N > PACK_MAX_N:
                    rejected += 1
                    continue
                queue.append(r)
            # admission: FIFO with backfill; the footprint is reserved at
            # once, the member is prepared by the executor (asynchronously on
            # the GPU) and joins its bucket when ready
            for r in list(queue):
                fp = footprint_bytes(r)
                if used + fp > self.budget:
                    continue
                if used + retired() + fp > self.budget:
                    flush()
                queue.remove(r)
                used += fp
                peak = max(peak, used)
                admitting.append((ex.admit_async(r), r, fp))
            for item in list(admitting):
                fut, r, fp = item
                if not fut.done():
                    continue
                admitting.remove(item)
                try:
                    handle, t_adm = fut.result()
                except Exception:
                    used -= fp
                    rejected += 1
                    continue
                mb = Member(r, fp, handle, admitted=ex.now() - t_start, last_done=t_adm)
                active.setdefault(r.key, []).append(mb)
                self.members[r.rid] = mb
                dirty.add(r.key)
            n_act = sum(len(v) for v in active.values())
            max_conc = max(max_conc, n_act)
            # idle buckets take their membership changes and launch a step
            for key in list(dirty):
                if key in inflight:
                    continue
                if active.get(key):
                    ex.set_bucket(key, active[key])
                    buckets_seen.add(key)
                else:
                    ex.drop_bucket(key)
                    active.pop(key, None)
                dirty.discard(key)
            for key, ms in active.items():
                if ms and key not in inflight:
                    inflight[key] = ex.launch_step(key)
                    stepping[key] = list(ms)  # members admitted later join after this step
                    steps_launched += 1
            if not inflight:
                if admitting:
                    # nothing to step until a member is ready
                    concurrent.futures.wait([a[0] for a in admitting], timeout=0.05,
                                            return_when=concurrent.futures.FIRST_COMPLETED)
                    continue
                flush()
                if not pending and not queue:
                    break
                if pending:
                    wait = pending[0].arrival - (ex.now() - t_start)
                    if wait > 0:
                        if realtime and hasattr(ex, "torch"):
                            time.sleep(min(wait, 0.05))
                        elif hasattr(ex, "advance_to"):
                            ex.advance_to(t_start + pending[0].arrival)
                        else:
                            time.sleep(min(wait, 0.05))
                continue
            until = t_start + pending[0].arrival if pending else None
            if admitting:
                # look again soon for members that have become ready
                soon = ex.now() + 1e-3
                until = soon if until is None else min(until, soon)
            for key, t_end in ex.poll(inflight, until).items():
                del inflight[key]
                # failure isolation: a member whose own flag reports a
                # non-physical state is evicted with an error; the others
                # (which share no data with it) carry on
                bad = {id(mb) for mb in ex.failed_members(key)}
                for mb in stepping.pop(key):
                    if id(mb) in bad:
                        mb.error = NonPhysicalState(
                            f"request {mb.req.rid}: non-physical state (rho <= 0, p <= 0 or "
                            f"NaN) in step {mb.steps_done + 1}")
                        mb.finished = ex.now() - t_start
                        ex.release(mb, keep=False)
                        mb.handle = None
                        active[key].remove(mb)
                        used -= mb.footprint
                        failed.append(mb)
                        dirty.add(key)
                        continue
                    mb.latencies.append(t_end - mb.last_done)
                    mb.last_done = t_end
                    mb.steps_done += 1
                    if mb.steps_done >= mb.req.steps:
                        mb.finished = ex.now() - t_start
                        self.results[mb.req.rid] = ex.release(mb)
                        active[key].remove(mb)
                        used -= mb.footprint
                        done.append(mb)
                        dirty.add(key)
        for key in list(active):
            ex.drop_bucket(key)
        flush()
        makespan = max((mb.finished for mb in done), default=0.0)
        first = min((r.arrival for r in requests), default=0.0)
        span = max(makespan - first, 1e-12)
        lat = np.array([x for mb in done for x in mb.latencies]) if done else np.zeros(1)
        waits = np.array([mb.admitted - mb.req.arrival for mb in done]) if done else np.zeros(1)
        e2e = np.array([mb.finished - mb.req.arrival for mb in done]) if done else np.zeros(1)
        work = sum(mb.req.nodes * 5 * mb.steps_done for mb in done)
        self._last = RunStats(
            n_requests=len(requests), n_completed=len(done), n_rejected=rejected,
            makespan_s=span, aggregate_dof_rhs_per_s=work / span,
            step_latency_p50_ms=float(np.percentile(lat, 50) * 1e3),
            step_latency_p99_ms=float(np.percentile(lat, 99) * 1e3),
            queue_wait_p50_ms=float(np.percentile(waits, 50) * 1e3),
            queue_wait_p99_ms=float(np.percentile(waits, 99) * 1e3),
            e2e_latency_mean_s=float(e2e.mean()), peak_footprint_bytes=int(peak),
            hbm_budget_bytes=self.budget, bucket_steps=steps_launched, max_concurrent_members=max_conc,
            buckets_seen=len(buckets_seen), n_failed=len(failed),
            time_breakdown=dict(getattr(ex, "times", {}) or {}) or None)
        return self._last
