"""Continuous-batching query server over resident scenes.

Scenes (Gaussians + visibility field) stay resident on the device.  Requests
ask for the uncertainty scores of a set of candidate views of one scene.  The
server keeps a FIFO of pending requests and a fixed number of slots (HIP
streams).  Whenever a slot is free it forms a batch from the oldest pending
request plus the following pending requests of the same scene (up to a view
budget), asks the backend for the workspace bytes of that batch, and admits
it if the bytes fit in the free memory budget; otherwise it waits for memory
to come back (the oldest request is never bypassed, so large requests do not
starve).  A request whose exact bytes exceed the whole budget is served in
chunks of its views (halved until each fits; a view's score does not depend
on the other views of its call), and only a single view that does not fit
is rejected.  Batches of different scenes run concurrently on different
slots.  Completion is detected by polling the slot's event; each request's
latency is completion time minus arrival time.

The backend is an interface, so the scheduling logic is tested on the CPU
with a simulated backend (memory budget, completion times, failures) and
runs on the GPU with `GpuBackend`.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np

PENDING, RUNNING, DONE, FAILED, CANCELLED, REJECTED = "pending", "running", "done", "failed", "cancelled", "rejected"


@dataclass(eq=False)                      # compared by identity (chunks share their request's id)
class Request:
    rid: int
    scene_id: Any
    cams: Any                 # scenes.Cameras
    t_arrival: float
    status: str = PENDING
    t_start: Optional[float] = None
    t_done: Optional[float] = None
    scores: Optional[np.ndarray] = None
    error: Optional[str] = None
    parent: Optional["Request"] = None   # set on a chunk of a request too large for the budget
    offset: int = 0                      # a chunk's first view within its request
    parts_left: int = 0                  # on a split request: chunks not yet done

    @property
    def n_views(self) -> int:
        return int(self.cams.n)

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_arrival


@dataclass(eq=False)
class Batch:
    reqs: List[Request]
    slot: int
    handle: Any
    nbytes: int
    t_launch: float


class BackendError(RuntimeError):
    pass


class Server:
    def __init__(self, backend, memory_budget: int, n_slots: int = 4, max_batch_views: int = 512,
                 stuck_timeout: float = 30.0):
        self.be = backend
        self.budget = int(memory_budget)
        self.in_use = 0
        self.n_slots = n_slots
        self.free_slots = list(range(n_slots))
        self.max_batch_views = max_batch_views
        self.stuck_timeout = stuck_timeout
        self.pending: deque = deque()
        self.running: List[Batch] = []
        self.requests: Dict[int, Request] = {}
        self._next = 0
        self.batches_launched = 0
        self.merged_requests = 0
        self.split_requests = 0

    # ---------------------------------------------------------------- client side
    def submit(self, scene_id, cams, t_arrival: Optional[float] = None) -> int:
        rid = self._next
        self._next += 1
        r = Request(rid, scene_id, cams, self.be.now() if t_arrival is None else t_arrival)
        self.requests[rid] = r
        self.pending.append(r)
        return rid

    def cancel(self, rid: int) -> bool:
        """Cancels a request none of whose views has started."""
        r = self.requests.get(rid)
        if r is None or r.status != PENDING:
            return False
        r.status = CANCELLED
        self._drop_pending(r)
        return True

    def _drop_pending(self, root: Request) -> None:
        """Removes a request and every pending chunk of it from the queue."""
        self.pending = deque(x for x in self.pending if x is not root and x.parent is not root)

    # ---------------------------------------------------------------- scheduling
    def _form_batch(self):
        """The oldest request plus the following requests of its scene, while
        the batch stays within the view budget and its workspace within a
        slot's share of the memory budget (so that the slots can overlap);
        returns (batch, its workspace bytes)."""
        head = self.pending[0]
        batch, views = [head], head.n_views
        nbytes = self.be.plan_bytes(head.scene_id, [head.cams])
        share = self.budget // max(self.n_slots, 1)
        for r in list(self.pending)[1:]:
            if r.scene_id != head.scene_id or views + r.n_views > self.max_batch_views or nbytes >= share:
                continue
            b = self.be.plan_bytes(head.scene_id, [x.cams for x in batch] + [r.cams])
            if b <= share:
                batch.append(r)
                views += r.n_views
                nbytes = b
        return batch, nbytes

    def _admit(self) -> None:
        while self.free_slots and self.pending:
            free = self.budget - self.in_use
            try:
                batch, nbytes = self._form_batch()
                if nbytes > self.budget:
                    # a request whose estimate exceeds the whole budget may
                    # still fit at its exact size (asked once per request:
                    # the backend keeps it while the request waits)
                    nbytes = self.be.plan_bytes(batch[0].scene_id, [batch[0].cams], limit=self.budget)
            except BackendError as e:
                self._fail([self.pending[0]], str(e))
                continue
            if nbytes > self.budget:
                head = batch[0]                          # never merged: it alone exceeds a share
                if head.n_views > 1:
                    self._split(head)
                else:
                    self._end(head, REJECTED, self.be.now(), msg=f"a view needs {nbytes} bytes, budget {self.budget}")
                continue
            if nbytes > self.budget - self.in_use:
                return                                   # wait for memory (FIFO head is not bypassed)
            slot = self.free_slots.pop(0)
            try:
                handle = self.be.launch(batch[0].scene_id, [r.cams for r in batch], slot, nbytes)
            except BackendError as e:
                self.free_slots.append(slot)
                self._fail(batch, str(e))
                continue
            t = self.be.now()
            for r in batch:
                self.pending.remove(r)
                r.status, r.t_start = RUNNING, t
                if r.parent is not None and r.parent.status == PENDING:
                    r.parent.status, r.parent.t_start = RUNNING, t
            self.in_use += nbytes
            self.running.append(Batch(batch, slot, handle, nbytes, t))
            self.batches_launched += 1
            self.merged_requests += len(batch) - 1

    def _split(self, r: Request) -> None:
        """Replaces the pending head r (a request or a chunk of one) by two
        chunks holding the first and the second half of its views."""
        root = r.parent or r
        h = r.n_views // 2
        parts = [Request(root.rid, r.scene_id, r.cams.subset(np.arange(lo, hi)), r.t_arrival,
                         parent=root, offset=r.offset + lo) for lo, hi in ((0, h), (h, r.n_views))]
        if r.parent is None:
            root.scores = np.zeros(root.n_views)
            root.parts_left = 2
            self.split_requests += 1
        else:
            root.parts_left += 1
        assert self.pending[0] is r
        self.pending.popleft()
        self.pending.appendleft(parts[1])
        self.pending.appendleft(parts[0])

    def _end(self, r: Request, status: str, t: float, scores=None, msg=None) -> None:
        """Settles a request or a chunk: a chunk writes its scores into its
        request, which is done when its last chunk is; a chunk that fails or
        is rejected ends its request so, and the request's pending chunks are
        dropped."""
        if r.status in (PENDING, RUNNING):
            r.status, r.t_done, r.error = status, t, msg
            if scores is not None and r.parent is None:
                r.scores = np.asarray(scores)
        if r in self.pending:
            self.pending.remove(r)
        root = r.parent
        if root is None:
            return
        if root.status not in (PENDING, RUNNING):
            return                                   # the request already ended (a chunk failed)
        if status != DONE:
            root.status, root.t_done, root.error = status, t, msg
            self._drop_pending(root)
            return
        root.scores[r.offset:r.offset + r.n_views] = scores
        root.parts_left -= 1
        if root.parts_left == 0:
            root.status, root.t_done = DONE, t

    def _fail(self, batch: List[Request], msg: str) -> None:
        t = self.be.now()
        for r in batch:
            self._end(r, FAILED, t, msg=msg)

    def _retire(self, b: Batch, status: str, scores=None, msg=None) -> None:
        t = self.be.now()
        off = 0
        for r in b.reqs:
            if r.status == RUNNING:          # requests already failed by a time-out stay failed
                self._end(r, status, t, scores=None if scores is None else scores[off:off + r.n_views], msg=msg)
            off += r.n_views
        self.in_use -= b.nbytes
        self.free_slots.append(b.slot)
        self.be.release(b.handle)

    def _poll(self) -> List[Request]:
        """Retires the batches that completed; returns the requests that
        ended (a split request once its last chunk has)."""
        finished = []
        for b in list(self.running):
            try:
                ready = self.be.done(b.handle)
            except BackendError as e:
                self.running.remove(b)
                self._retire(b, FAILED, msg=str(e))
                finished += b.reqs
                continue
            if ready:
                self.running.remove(b)
                try:
                    self._retire(b, DONE, scores=self.be.result(b.handle))
                except BackendError as e:
                    self._retire(b, FAILED, msg=str(e))
                finished += b.reqs
            elif self.be.now() - b.t_launch > self.stuck_timeout:
                # the device work cannot be recalled; its requests fail and its
                # slot and memory stay reserved until the backend reports done
                for r in b.reqs:
                    if r.status == RUNNING:
                        self._end(r, FAILED, self.be.now(), msg="timed out")
        return finished

    def step(self) -> List[Request]:
        done = []
        for r in self._poll():
            root = r.parent or r
            if root.status not in (PENDING, RUNNING) and all(x is not root for x in done):
                done.append(root)
        self._admit()
        return done

    def idle(self) -> bool:
        return not self.pending and not self.running

    def run_until_idle(self, timeout: float = 60.0, sleep: float = 0.0) -> None:
        t0 = self.be.now()
        while not self.idle():
            self.step()
            if self.be.now() - t0 > timeout:
                raise TimeoutError("server did not drain")
            self.be.wait(sleep)

    # ---------------------------------------------------------------- stats
    def stats(self) -> dict:
        done = [r for r in self.requests.values() if r.status == DONE]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        views = sum(r.n_views for r in done)
        if done:
            span = max(r.t_done for r in done) - min(r.t_arrival for r in done)
        else:
            span = 0.0
        return {"requests_done": len(done), "views_done": views,
                "p50_latency_ms": float(np.percentile(lat, 50) * 1e3) if done else None,
                "p99_latency_ms": float(np.percentile(lat, 99) * 1e3) if done else None,
                "views_per_s": views / span if span > 0 else None,
                "batches": self.batches_launched, "merged_requests": self.merged_requests,
                "split_requests": self.split_requests,
                "failed": sum(r.status == FAILED for r in self.requests.values()),
                "rejected": sum(r.status == REJECTED for r in self.requests.values())}


def replay(server: Server, arrivals, timeout: float = 120.0) -> dict:
    """Submits (t_offset, scene_id, cams) requests at their arrival times
    (relative to the start, on the backend's clock), stepping the server in
    between, and returns its statistics once everything has drained."""
    be = server.be
    t0 = be.now()
    queue = sorted(arrivals, key=lambda a: a[0])
    i = 0
    while i < len(queue) or not server.idle():
        now = be.now() - t0
        while i < len(queue) and queue[i][0] <= now:
            server.submit(queue[i][1], queue[i][2], t_arrival=t0 + queue[i][0])
            i += 1
        server.step()
        if be.now() - t0 > timeout:
            raise TimeoutError("replay did not drain")
        if i < len(queue) and server.idle():
            be.wait(min(queue[i][0] - (be.now() - t0), 1e-3))
    return server.stats()


# ==================================================================== GPU backend

@dataclass
class ResidentScene:
    dsc: Any                  # api.DeviceScene
    gamma: Any                # torch tensor [K, n]
    sh_degree: int
    n_train: int


class GpuBackend:
    """Runs batches through the C ABI, one HIP stream per slot.

    Admission needs a batch's workspace bytes before anything runs; they are
    computed on the host.  Per resident scene and image size the backend
    keeps the largest records and instances per view seen so far (`rates`)
    and plans a batch as the sum over its views of those rates times `slack`
    (Context.query_plan: no device pass, nothing allocated).  A batch holding
    an image size the scene has not been seen at, or a request whose estimate
    exceeds the whole budget, is sized exactly by the library's counting pass
    (synchronous; once per scene and size, once per such request).
    The workspace is allocated when the batch is launched, after admission;
    an allocation failure is a BackendError.  At completion every batch's
    workspace status gives its exact record and instance counts, which
    raise the rates; a batch that overflowed its plan (the kernels then skip
    their writes and flag it) is planned exactly and launched again on its
    slot, once.  Such a re-launch may hold more bytes than were admitted for
    the batch until it completes."""

    def __init__(self, ctx, n_slots: int = 4, params=None, slack: float = 1.25):
        import torch
        from . import _lib
        self.torch = torch
        self.ctx = ctx
        self.scenes: Dict[Any, ResidentScene] = {}
        self.n_slots = n_slots
        self._streams = None      # created on first use (the planning logic runs without a device)
        self.params = params if params is not None else _lib.default_uq_params()
        self.slack = float(slack)
        self.rates: Dict[tuple, list] = {}      # (scene, w, h) -> [records per view, instances per view]
        self.exact_sizings = 0
        self.relaunches = 0
        self._exact_plans: Dict[tuple, Any] = {}   # exact plans of batches whose estimate did not fit

    def add_scene(self, scene_id, dsc, gamma, sh_degree: int, n_train: int) -> None:
        self.scenes[scene_id] = ResidentScene(dsc, gamma, sh_degree, n_train)

    @property
    def streams(self):
        if self._streams is None:
            self._streams = [self.torch.cuda.Stream() for _ in range(self.n_slots + 1)]
        return self._streams

    @property
    def plan_stream(self):
        return self.streams[-1]

    def now(self) -> float:
        return time.perf_counter()

    def wait(self, dt: float) -> None:
        if dt > 0:
            time.sleep(dt)

    def _cams(self, cams_list):
        from .scenes import Cameras
        return cams_list[0] if len(cams_list) == 1 else Cameras.concat(cams_list)

    @staticmethod
    def _sizes(cams):
        return [(int(w), int(h)) for w, h in cams.wh]

    def _exact(self, sc, cams):
        """Exact capacities of `cams` by the library's counting pass."""
        from ._lib import GvError
        try:
            ws_plan = self.ctx.query_plan_exact(sc.dsc, cams, self.params, sc.sh_degree, stream=self.plan_stream)
        except GvError as e:
            raise BackendError(str(e))
        self.exact_sizings += 1
        return ws_plan

    def _learn(self, scene_id, cams, records: int, instances: int) -> None:
        """Raises the per-view rates of the image sizes in `cams` so that
        they cover `records` and `instances` spread over its views by the
        current rates (evenly for sizes without one)."""
        sizes = self._sizes(cams)
        keys = [(scene_id,) + wh for wh in sizes]
        est_r = sum(self.rates.get(k, [0.0, 0.0])[0] for k in keys)
        est_m = sum(self.rates.get(k, [0.0, 0.0])[1] for k in keys)
        n = len(keys)
        for k in set(keys):
            r = self.rates.setdefault(k, [0.0, 0.0])
            r[0] = max(r[0], records / n if est_r <= 0 else r[0] * records / est_r)
            r[1] = max(r[1], instances / n if est_m <= 0 else r[1] * instances / est_m)

    def _plan(self, scene_id, cams):
        sc = self.scenes[scene_id]
        keys = [(scene_id,) + wh for wh in self._sizes(cams)]
        missing = sorted({k[1:] for k in keys if k not in self.rates})
        for wh in missing:       # first sight of an image size: one exact pass over its views
            sub = cams.subset([i for i, k in enumerate(keys) if k[1:] == wh])
            p = self._exact(sc, sub)
            self._learn(scene_id, sub, int(p.max_records), int(p.max_instances))
        rec = sum(self.rates[k][0] for k in keys) * self.slack
        ins = sum(self.rates[k][1] for k in keys) * self.slack
        return self.ctx.query_plan(sc.dsc, cams, sc.sh_degree, int(np.ceil(rec)) + 64, int(np.ceil(ins)) + 256)

    def plan_bytes(self, scene_id, cams_list, limit: Optional[int] = None) -> int:
        """Workspace bytes of a batch from the learnt rates; when that
        estimate exceeds `limit` (the free budget), the exact bytes instead
        (one counting pass, kept for the batch's launch and for later asks
        while it waits for memory)."""
        key = (scene_id, tuple(id(c) for c in cams_list))
        if key in self._exact_plans:          # the entry holds the cameras, so their ids stay theirs
            return int(self._exact_plans[key][1].bytes)
        cams = self._cams(cams_list)
        plan = self._plan(scene_id, cams)
        if limit is not None and plan.bytes > limit:
            plan = self._exact(self.scenes[scene_id], cams)
            if len(self._exact_plans) >= 64:
                self._exact_plans.pop(next(iter(self._exact_plans)))
            self._exact_plans[key] = (list(cams_list), plan)
        return int(plan.bytes)

    def _alloc(self, plan):
        torch = self.torch
        try:
            return self.ctx.alloc_workspace(plan)
        except (torch.cuda.OutOfMemoryError, RuntimeError) as e:
            raise BackendError(f"workspace allocation of {int(plan.bytes)} bytes failed: {e}")

    def _run(self, h) -> None:
        from ._lib import GvError
        torch = self.torch
        sc = self.scenes[h["scene"]]
        s = h["stream"]
        s.wait_stream(self.plan_stream)
        with torch.cuda.stream(s):
            try:
                self.ctx.vf_query_views(sc.dsc, sc.gamma, sc.sh_degree, sc.n_train, h["cams"], self.params,
                                        h["ws"], scores=h["scores"], stream=s)
            except GvError as e:
                raise BackendError(str(e))
            ev = torch.cuda.Event()
            ev.record(s)
        h["ev"] = ev

    def launch(self, scene_id, cams_list, slot: int, nbytes: int):
        torch = self.torch
        cams = self._cams(cams_list)
        ent = self._exact_plans.pop((scene_id, tuple(id(c) for c in cams_list)), None)
        plan = ent[1] if ent is not None else self._plan(scene_id, cams)
        ws = self._alloc(plan)
        scores = torch.empty(cams.n, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        h = {"scene": scene_id, "cams": cams, "ws": ws, "scores": scores, "stream": self.streams[slot],
             "relaunched": False}
        self._run(h)
        return h

    def done(self, h) -> bool:
        from ._lib import GV_ERR_CAPACITY
        if not h["ev"].query():
            return False
        st, counts = self.ctx.check_workspace(h["ws"], stream=h["stream"])
        self._learn(h["scene"], h["cams"], counts[0], counts[1])
        if st == GV_ERR_CAPACITY and not h["relaunched"]:
            sc = self.scenes[h["scene"]]
            plan = self._exact(sc, h["cams"])
            h["ws"] = self._alloc(plan)
            h["relaunched"] = True
            self.relaunches += 1
            self._run(h)
            return False
        if st != 0:
            raise BackendError(f"query failed with status {st} (records {counts[0]}, instances {counts[1]})")
        return True

    def result(self, h):
        return h["scores"].cpu().numpy()

    def release(self, h) -> None:
        h.clear()
