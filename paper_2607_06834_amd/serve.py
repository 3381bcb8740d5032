"""Serving many independent PTA data sets on one GPU with continuous batching.

Each request is one data set (any shape within the library limits) with a
fixed-step HMC job: n_chains chains, n_traj trajectories of n_leapfrog
steps.  Admitted requests run side by side, each on its own HIP stream, and
advance by quanta of trajectories (one captured HIP-graph replay per
trajectory).  A request is admitted, first come first served, as soon as a
slot is free and its device footprint fits the memory budget next to the
requests already running; a finished request releases its slot and memory at
once, so the next one starts while the others are still running.  The
footprint is known before any allocation (ptafs_estimate plus the server's
own per-request buffers); a request that could never fit is rejected at
submission.

Every request's arithmetic depends only on its own data set, start point,
seed and TOA-pass tuning: its samples are bit-identical whether it runs
alone or in a mix.  The tuning is fixed by the caller, or else a fixed
function of the request's shape (autotune.serving_tuning), never a timing
taken under the load of other requests.

Two threads share the work.  The admission thread creates each admitted
request's data set, workspace and first evaluation on the request's own
stream; the scheduler thread only collects finished quanta and launches the
next ones, so admitting or retiring a request never stalls the others (the
library synchronises nothing device-wide: its memory comes from a
stream-ordered pool that is reused across requests, and a data set waits
only for its own work when it is released).
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np
import torch

from . import api, autotune

class Rejected(RuntimeError):
    """The request can never fit the server's memory budget (or its
    descriptor is invalid)."""


class Cancelled(RuntimeError):
    """Raised by ``poll``/``wait`` for a request that was cancelled."""


@dataclasses.dataclass
class _Req:
    rid: int
    desc: dict
    n_traj: int
    n_leapfrog: int
    eps: float
    seed: int
    x0: np.ndarray
    inv_mass: np.ndarray | None
    keep: str
    footprint: int
    t_arrival: float
    tuning: tuple = ()
    t_admit: float = float("nan")
    t_done: float = float("nan")
    status: str = "queued"
    error: str | None = None
    cancel: bool = False
    # running state
    ds: object = None
    stream: object = None
    x: object = None
    lp: object = None
    gr: object = None
    acc: object = None
    bad: object = None
    im: object = None
    smp: object = None
    done_traj: int = 0
    pending: int = 0
    event: object = None
    out: list = dataclasses.field(default_factory=list)
    result: dict | None = None


class Server:
    """``Server(budget_bytes, max_slots).submit(desc, ...) -> id``;
    ``poll(id)`` returns None until the request has finished, then a dict with
    the samples (n_traj, n_chains, n_theta or d), final log p, acceptance and
    invalid-evaluation counts and the arrival / admission / completion times
    (``time.perf_counter`` seconds).  ``cancel(id)`` withdraws a queued request
    or stops a running one at its next quantum boundary, freeing its memory."""

    def __init__(self, budget_bytes: int, max_slots: int = 8, quantum: int = 10, device: int = 0,
                 tuning=None, use_graph: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("the server needs a HIP GPU")
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.quantum = max(1, int(quantum))
        self.device = int(device)
        self.tuning = tuning
        self.use_graph = bool(use_graph)
        self._lock = threading.Condition()
        self._queue: collections.deque[_Req] = collections.deque()
        self._reqs: dict[int, _Req] = {}
        self._next = 0
        self._used = 0
        self.max_used = 0
        self.max_active = 0
        self._stop = False
        self._err = None
        self._n_cu = torch.cuda.get_device_properties(self.device).multi_processor_count
        self._to_admit: collections.deque[_Req] = collections.deque()
        self._ready: collections.deque[_Req] = collections.deque()
        self._admitting = 0
        self._thread = threading.Thread(target=self._run, name="ptafs-serve", daemon=True)
        self._admit_thread = threading.Thread(target=self._admit_loop, name="ptafs-admit", daemon=True)
        self._admit_thread.start()
        self._thread.start()

    # ------------------------------------------------------------------ API
    def footprint(self, desc, n_chains: int) -> int:
        """Device bytes a request holds while it runs."""
        est = api.ptafs_estimate(desc, n_chains)
        d = int(est.d)
        own = 8 * (2 * n_chains * d + 2 * n_chains + d + self.quantum * n_chains * d) + 8 * 2 * n_chains
        return int(est.dataset_bytes + est.workspace_bytes + est.hmc_bytes) + own + (1 << 20)

    def submit(self, desc, *, x0, n_traj: int, n_leapfrog: int = 20, eps: float, seed: int,
               inv_mass=None, keep: str = "theta") -> int:
        """Queue a request.  ``x0`` (n_chains, d) start points; ``keep`` is
        "theta" (hyper-parameter samples) or "all" (whole vectors)."""
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        if x0.ndim != 2:
            raise ValueError("x0 must be (n_chains, d)")
        try:
            fp = self.footprint(desc, x0.shape[0])
        except RuntimeError as e:
            raise Rejected(str(e)) from e
        if fp > self.budget:
            raise Rejected(f"footprint {fp} B exceeds the budget {self.budget} B")
        t_arrival = time.perf_counter()
        with self._lock:
            if self._err is not None:
                raise RuntimeError("server stopped after an error") from self._err
            rid = self._next
            self._next += 1
            r = _Req(rid, desc, int(n_traj), int(n_leapfrog), float(eps), int(seed), x0,
                     None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64),
                     keep, fp, t_arrival)
            self._reqs[rid] = r
            self._queue.append(r)
            self._lock.notify_all()
        return rid

    def poll(self, rid: int):
        with self._lock:
            r = self._reqs[rid]
            if r.status == "error":
                raise RuntimeError(f"request {rid} failed: {r.error}")
            if r.status == "cancelled":
                raise Cancelled(f"request {rid} was cancelled after {r.done_traj} trajectories")
            return r.result if r.status == "done" else None

    def cancel(self, rid: int) -> bool:
        """Cancel a request.  A queued request leaves the queue at once; an
        admitted one stops at its next quantum boundary (the quantum in flight
        finishes on its own stream), and its device memory and budget are
        released then.  Returns False if the request had already finished."""
        with self._lock:
            r = self._reqs[rid]
            if r.status in ("done", "error", "cancelled"):
                return False
            if r.status == "queued" and r in self._queue:
                self._queue.remove(r)
                r.status = "cancelled"
                self._lock.notify_all()
                return True
            r.cancel = True
            return True

    def wait(self, rid: int, timeout: float | None = None):
        t_end = None if timeout is None else time.perf_counter() + timeout
        with self._lock:
            while True:
                r = self._reqs[rid]
                if r.status in ("done", "error", "cancelled") or self._err is not None:
                    break
                left = None if t_end is None else t_end - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError(f"request {rid} not finished")
                self._lock.wait(left if left is not None else 0.5)
        return self.poll(rid)

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        self._thread.join()
        self._admit_thread.join()
        if self._err is not None:
            raise RuntimeError("server stopped after an error") from self._err

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ scheduler
    def _admit(self, r: _Req):
        """Create the request's device state on its own stream (admission
        thread); the scheduler launches its first quantum once it is ready."""
        r.t_admit = time.perf_counter()
        torch.cuda.set_device(self.device)
        r.stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(r.stream):
            r.ds = api.Dataset(r.desc, stream=r.stream)
            C, d = r.x0.shape[0], r.ds.d
            if r.x0.shape[1] != d:
                raise ValueError(f"x0 has {r.x0.shape[1]} columns, the data set needs {d}")
            tuning = self.tuning if self.tuning is not None else \
                autotune.serving_tuning(r.ds.toa_offsets, C, self._n_cu)
            r.ds.ptafs_set_tuning(*tuning)
            r.tuning = r.ds.ptafs_get_tuning()
            r.ds.ptafs_reserve(C)
            dev = torch.device("cuda", self.device)
            r.x = torch.tensor(r.x0, device=dev)
            r.lp, r.gr, _ = r.ds.ptafs_logp_grad(r.x, stream=r.stream)
            r.acc = torch.zeros(C, dtype=torch.int64, device=dev)
            r.bad = torch.zeros(C, dtype=torch.int64, device=dev)
            r.im = None if r.inv_mass is None else torch.tensor(r.inv_mass, device=dev)
            r.smp = torch.empty((self.quantum, C, d), dtype=torch.float64, device=dev)
        r.status = "running"

    def _admit_loop(self):
        try:
            torch.cuda.set_device(self.device)
            while True:
                with self._lock:
                    while not self._to_admit and not self._stop:
                        self._lock.wait(0.05)
                    if not self._to_admit and self._stop:
                        return
                    r = self._to_admit.popleft()
                try:
                    self._admit(r)
                    with self._lock:
                        self._ready.append(r)
                        self._admitting -= 1
                        self._lock.notify_all()
                except Exception as e:  # this request only
                    if r.ds is not None:
                        r.ds.close()
                    with self._lock:
                        self._admitting -= 1
                    self._release(r, "error", repr(e))
        except Exception as e:  # a failure of the admission thread itself
            with self._lock:
                self._err = e
                self._lock.notify_all()

    def _launch(self, r: _Req):
        q = min(self.quantum, r.n_traj - r.done_traj)
        with torch.cuda.stream(r.stream):
            r.ds.ptafs_hmc_run(r.x, r.lp, r.gr, r.acc, n_traj=q, n_leapfrog=r.n_leapfrog, eps=r.eps,
                               seed=r.seed, traj0=r.done_traj, inv_mass=r.im, samples=r.smp[:q],
                               n_invalid=r.bad, use_graph=self.use_graph, stream=r.stream)
            r.event = torch.cuda.Event()
            r.event.record(r.stream)
        r.pending = q

    def _collect(self, r: _Req):
        # copies on the request's own stream (idle now): no wait on the others
        q = r.pending
        s = r.smp[:q]
        if r.keep == "theta":
            s = s[:, :, : r.ds.layout.n_theta]
        with torch.cuda.stream(r.stream):
            r.out.append(s.cpu().numpy())
        r.done_traj += q
        r.pending = 0

    def _finish(self, r: _Req):
        with torch.cuda.stream(r.stream):
            r.result = dict(
                samples=np.concatenate(r.out) if r.out else np.zeros((0,)),
                logp=r.lp.cpu().numpy(), n_accept=r.acc.cpu().numpy(),
                n_invalid=r.bad.cpu().numpy(), x=r.x.cpu().numpy(),
                t_arrival=r.t_arrival, t_admit=r.t_admit, t_done=time.perf_counter(),
                footprint=r.footprint, tuning=tuple(r.tuning))
        r.t_done = r.result["t_done"]
        r.result["latency"] = r.t_done - r.t_arrival
        self._drop(r)

    def _drop(self, r: _Req):
        # the data set waits for its own last work before its memory goes back
        r.ds.close()
        r.ds = r.stream = r.x = r.lp = r.gr = r.acc = r.bad = r.im = r.smp = r.event = None
        r.out = []

    def _release(self, r: _Req, status: str, error: str | None = None):
        with self._lock:
            r.status, r.error = status, error
            self._used -= r.footprint
            self._lock.notify_all()

    def _run(self):
        torch.cuda.set_device(self.device)
        active: list[_Req] = []
        try:
            while True:
                # admission (first come first served, by slot and footprint):
                # the admission thread builds the device state, and the request
                # joins the active set when it is ready
                started = []
                with self._lock:
                    if self._err is not None:
                        raise self._err
                    while self._queue and len(active) + self._admitting + len(self._ready) < self.max_slots \
                            and self._used + self._queue[0].footprint <= self.budget:
                        r = self._queue.popleft()
                        self._used += r.footprint
                        self.max_used = max(self.max_used, self._used)
                        self._admitting += 1
                        self._to_admit.append(r)
                        self._lock.notify_all()
                    while self._ready:
                        started.append(self._ready.popleft())
                    if not active and not started:
                        if self._stop and not self._queue and not self._admitting:
                            return
                        self._lock.wait(0.002)
                        continue
                for r in started:
                    if r.cancel:   # cancelled while it was being admitted
                        self._drop(r)
                        self._release(r, "cancelled")
                        continue
                    active.append(r)
                    self._launch(r)
                self.max_active = max(self.max_active, len(active))
                # progress: collect finished quanta, launch the next ones
                progressed = False
                for r in list(active):
                    if r.event is not None and r.event.query():
                        self._collect(r)
                        if r.cancel and r.done_traj < r.n_traj:
                            self._drop(r)
                            active.remove(r)
                            self._release(r, "cancelled")
                        elif r.done_traj >= r.n_traj:
                            self._finish(r)
                            active.remove(r)
                            self._release(r, "done")
                        else:
                            self._launch(r)
                        progressed = True
                if not progressed:
                    time.sleep(2e-4)
        except Exception as e:  # a failure of the scheduler itself
            with self._lock:
                self._err = e
                self._stop = True
                for r in active + list(self._queue) + list(self._ready):
                    r.status, r.error = "error", repr(e)
                self._lock.notify_all()
