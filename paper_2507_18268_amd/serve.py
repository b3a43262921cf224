"""Serving loop for parametric heat-equation solves (snapshot generation).

A request is (cube side n, DT, dt, number of steps, T0); its answer is T after
every step.  The server keeps the meshes (one per side, shared by all requests
of that side) and every admitted request's fields resident on the device, and
runs continuous batching over several launch slots, each a stream with its own
batched-kernel task table:

* admission: a queued request is admitted when its device bytes (snapshot
  buffer, plus a problem workspace unless an idle one of its side can be
  re-used, plus its mesh if that is not resident yet) fit the HBM budget; idle
  problems, then resident meshes no admitted request uses, are evicted first
  when memory is short;
* launch: whenever a slot is free, the admitted requests not yet running
  (largest first, up to a slot's capacity, one workgroup size per launch) go
  into that slot's persistent batched kernel, so requests that arrive while
  others run start on free slots and their work overlaps on the device;
* completion: a finished slot's snapshots are copied to the host, the
  requests' problems go back to a per-side pool (destroying a problem frees
  pinned host memory, which waits for the whole device, so problems are
  re-targeted with lf_problem_reset instead), and the latency (arrival to
  results on the host) is recorded.

Large requests can instead take the direct lane: up to direct_workers of them
at a time, each with its own pool of problems, run all their steps with the
multi-kernel solver (many workgroups per problem, coefficients in the band
layout where the mesh allows), T being copied after each step into the
snapshot buffer.  By default the lane is a group (lf_group): every kernel of
the running direct requests' steps goes out as one launch for all of them that
need it, so a mid-size request no longer pays a dependent launch per kernel of
its own; T0 goes up and the snapshots come down on a few lane streams.  A request's run
starts when it is admitted (lf_group_add) and every scheduling pass advances
the group as far as its finished device work allows (lf_group_poll, which
never waits), so a small request does not wait for a large one's steps.
(direct_group=False runs each request alone with lf_step_begin/lf_step_poll
on a stream of its own.)
One workgroup is far too little for a large mesh, so this cuts both their
latency and the time the batched slots spend waiting for them.  The lane runs
on the scheduling thread: polling returns at once, and no second host thread
has to share the interpreter with the scheduler.

A batched workgroup occupies its compute unit for the whole of its problem,
so with the direct lane on the server keeps at most batch_max_running batched
problems in flight (3/4 of the CUs by default) and the direct lane's kernels
always find free CUs.

The server uses n_slots + direct_workers + 1 streams.  The process needs at
least that many hardware queues (HIP's GPU_MAX_HW_QUEUES, 4 by default, set
before the runtime starts): streams that share a queue run in order, so a
direct-lane kernel would wait behind a whole persistent batched launch.

Every request's result is independent of what it shares the GPU with: the
batched kernel solves each problem inside one workgroup with fixed-order sums,
and the workgroup size comes from the autotuner's table for the request's
size; the direct lane's kernels use fixed-order reductions too, and which lane
a request takes depends only on its size.
"""
import collections
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import autotune
from . import lapfoam as L


@dataclass
class Request:
    rid: int
    n: int
    DT: float
    dt: float
    steps: int
    T0: np.ndarray
    bcs: list
    arrival: float = 0.0           # seconds on the server clock
    # filled by the server
    admitted: float = None
    launched: float = None
    done: float = None
    snapshots: np.ndarray = None   # [steps, N]
    stats: list = None
    error: str = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


@dataclass
class _Live:
    req: Request
    problem: object
    snap: object                   # device tensor [steps * N]
    snap_bytes: int
    key: tuple                     # problem pool of the request: (side, lane)


@dataclass
class _Direct:
    req: Request
    problem: object
    snap: object                   # device tensor [steps, N]
    snap_bytes: int
    key: tuple
    worker: int                    # direct-lane slot (its stream)
    step: int = 0
    stats: list = None


class Server:
    def __init__(self, mesh_for_side, budget_bytes, n_slots=4, slot_capacity=64, max_steps=10,
                 tuning=None, direct_min_side=None, direct_workers=4, batch_max_running=None,
                 direct_use_graph=True, direct_group=True, direct_streams=4, group_iters=0):
        import torch
        self.torch = torch
        # A batched workgroup holds its CU for a whole problem; with the direct
        # lane on, at most this many batched problems run at once so that
        # direct-lane kernels always find free CUs (default: 3/4 of the CUs).
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        if batch_max_running is None:
            batch_max_running = (3 * n_cu) // 4 if direct_min_side is not None else n_slots * slot_capacity
        self.batch_max_running = max(1, int(batch_max_running))
        self.mesh_for_side = mesh_for_side          # side -> mesh description (host arrays)
        self.budget = int(budget_bytes)
        self.used = 0
        self.slot_capacity = slot_capacity
        self.max_steps = max_steps
        self.tuning = tuning if tuning is not None else autotune.load()
        self.admit_stream = torch.cuda.Stream()     # set-up work of batched-lane problems
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.batches = [L.Batch(slot_capacity, max_steps, stream=s) for s in self.streams]
        self.slot_live: List[Optional[List[_Live]]] = [None] * n_slots
        # requests with side >= direct_min_side take the direct lane (None: never)
        self.direct_min_side = direct_min_side
        self.direct_use_graph = direct_use_graph
        nd = direct_workers if direct_min_side is not None else 0
        # grouped lane: the running direct requests' kernels share launches
        # (lf_group, on its own stream); their uploads and downloads go to a
        # few streams, worker k on stream k % direct_streams
        self.group = None
        if nd and direct_group:
            self.group_stream = torch.cuda.Stream()
            self.group = L.Group(nd, iters_per_block=group_iters, stream=self.group_stream)
            ns = max(1, min(nd, int(direct_streams)))
            pool = [torch.cuda.Stream() for _ in range(ns)]
            self.direct_streams = [pool[k % ns] for k in range(nd)]
        else:
            self.direct_streams = [torch.cuda.Stream() for _ in range(nd)]
        self.direct_slot: List[Optional[_Direct]] = [None] * nd
        self.draining = []                            # direct results on their way to the host
        self.idle: Dict[tuple, List[object]] = collections.defaultdict(list)   # key -> idle problems
        self.meshes: Dict[int, object] = {}          # side -> L.Mesh
        self.mesh_bytes: Dict[int, int] = {}
        self.mesh_users: Dict[int, int] = collections.defaultdict(int)
        self.mesh_last_use: Dict[int, float] = {}
        self.queue = collections.deque()              # arrived, not admitted
        self.ready: List[_Live] = []                  # admitted, not launched
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.mesh_builds = 0                          # device meshes created
        self.evictions = 0                            # idle problems and meshes freed for room
        self.t0 = time.perf_counter()

    # ------------------------------------------------------------------ clock
    def now(self):
        return time.perf_counter() - self.t0

    # -------------------------------------------------------------- memory
    def _is_direct(self, req):
        return self.direct_min_side is not None and req.n >= self.direct_min_side

    def _opts(self, direct, mesh):
        # band layout where the mesh has one; the batched kernel takes it for
        # 3-band (structured 3-D) meshes only
        banded = mesh.n_bands == 3 or (direct and mesh.n_bands > 0)
        layout = L.LF_LAYOUT_AUTO if banded else L.LF_LAYOUT_ROWS
        graph = 1 if (not direct or self.direct_use_graph) else 0
        return L.make_opts(precision=L.LF_PREC_MIXED, layout=layout, use_graph=graph)

    def idle_bytes(self):
        return sum(P.ws_bytes for ps in self.idle.values() for P in ps)

    def preload_mesh(self, side):
        """Make a side's mesh resident (counted in the budget)."""
        if side in self.meshes:
            return self.meshes[side]
        m = L.Mesh(self.mesh_for_side(side))
        self.mesh_builds += 1
        self.meshes[side] = m
        self.mesh_bytes[side] = m.ws_bytes
        self.used += m.ws_bytes
        self.mesh_last_use[side] = self.now()
        return m

    def _close_idle(self, key):
        for P in self.idle.pop(key, []):
            self.used -= P.ws_bytes
            self.evictions += 1
            P.close()

    def _evict(self, need, keep_side):
        """Free idle problems, then idle meshes (least recently used sides
        first, the requesting side last) until `need` more bytes fit."""
        order = sorted(self.meshes, key=lambda s: (s == keep_side, self.mesh_last_use.get(s, 0.0)))
        for side in order:
            if self.used + need <= self.budget:
                return
            for key in [k for k in self.idle if k[0] == side]:
                self._close_idle(key)
        for side in order:
            if self.used + need <= self.budget:
                return
            if side != keep_side and self.mesh_users[side] == 0 and not any(
                    k[0] == side and ps for k, ps in self.idle.items()):
                self.meshes.pop(side).close()
                self.evictions += 1
                self.used -= self.mesh_bytes.pop(side)
                self.mesh_last_use.pop(side, None)

    # -------------------------------------------------------------- requests
    def submit(self, req: Request):
        if req.steps > self.max_steps:
            req.error = f"at most {self.max_steps} steps per request"
            self.rejected.append(req)
            return
        self.queue.append(req)

    def _reject(self, req, why):
        self.queue.popleft()
        req.error = why
        self.rejected.append(req)

    def _admit(self):
        while self.queue:
            req = self.queue[0]
            direct = self._is_direct(req)
            worker = -1
            if direct:
                free = [k for k, d in enumerate(self.direct_slot) if d is None]
                if not free:
                    return                   # in arrival order: wait for a direct slot
                worker = free[0]
            key = (req.n, worker)
            if req.n not in self.meshes:
                # size the mesh from its description before building it
                mbytes = L.lf_mesh_workspace_bytes(_desc_of(self.mesh_for_side(req.n))[0])
                self._evict(mbytes, req.n)
                if self.used + mbytes > self.budget:
                    if not self._anything_live():
                        self._reject(req, "mesh larger than the device-memory budget")
                        continue
                    return
                mesh = self.preload_mesh(req.n)
            else:
                mesh = self.meshes[req.n]
            snap_bytes = 8 * req.steps * mesh.n_cells
            new_bytes = L.lf_problem_workspace_bytes(mesh.h, self._opts(direct, mesh))
            need = snap_bytes if self.idle.get(key) else snap_bytes + new_bytes
            if self.used + need > self.budget:
                self._evict(need, req.n)
                need = snap_bytes if self.idle.get(key) else snap_bytes + new_bytes
            if self.used + need > self.budget:
                if not self._anything_live():
                    self._reject(req, "request larger than the device-memory budget")
                    continue
                return
            self.queue.popleft()
            self.used += need
            self.mesh_users[req.n] += 1
            req.admitted = self.now()
            P = self.idle[key].pop() if self.idle.get(key) else None
            if direct:
                self._start_direct(req, mesh, P, snap_bytes, key, worker)
                continue
            with self.torch.cuda.stream(self.admit_stream):
                if P is None:
                    P = L.Problem(mesh, req.bcs, req.DT, req.dt, self._opts(False, mesh),
                                  stream=self.admit_stream)
                else:
                    P.reset(req.bcs, req.DT, req.dt)
                self._upload_T(P, req.T0)
                snap = self.torch.empty(req.steps * mesh.n_cells, dtype=self.torch.float64,
                                        device="cuda")
                self.admit_stream.synchronize()      # T in place before any slot uses it
            self.ready.append(_Live(req, P, snap, snap_bytes, key))

    # Host transfers go through pinned buffers on the lane's own stream: a copy
    # from or to pageable host memory can wait for work on other streams, i.e.
    # for whole persistent batched launches.
    def _upload_T(self, P, T0):
        torch = self.torch
        h = torch.from_numpy(np.ascontiguousarray(T0, dtype=np.float64)).pin_memory()
        d = torch.empty(h.shape, dtype=torch.float64, device="cuda")
        d.copy_(h, non_blocking=True)
        P.set_T(d)                                   # device copy on the problem's stream

    def _download(self, dev):
        torch = self.torch
        h = torch.empty(dev.shape, dtype=dev.dtype, pin_memory=True)
        h.copy_(dev, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        return h.numpy()

    def _anything_live(self):
        return bool(self.ready) or any(d is not None for d in self.direct_slot) or \
            any(s is not None for s in self.slot_live) or bool(self.draining)

    # -------------------------------------------------------------- batched lane
    def _launch(self):
        for k, live in enumerate(self.slot_live):
            if live is not None or not self.ready:
                continue
            room = self.batch_max_running - sum(len(g) for g in self.slot_live if g is not None)
            if room <= 0:
                return
            # largest first; one workgroup size and one step count per launch
            self.ready.sort(key=lambda x: -x.problem.mesh.n_cells)
            bs = autotune.block_threads_for(self.ready[0].req.n, self.tuning)
            steps = self.ready[0].req.steps
            group = [x for x in self.ready
                     if autotune.block_threads_for(x.req.n, self.tuning) == bs
                     and x.req.steps == steps][: min(self.slot_capacity, room)]
            for x in group:
                self.ready.remove(x)
            self.batches[k].launch([x.problem for x in group], steps, block_threads=bs,
                                   snapshots=[x.snap for x in group])
            t = self.now()
            for x in group:
                x.req.launched = t
            self.slot_live[k] = group

    def _finish(self, req, snap_bytes):
        req.done = self.now()
        self.finished.append(req)
        self.used -= snap_bytes
        self.mesh_users[req.n] -= 1
        self.mesh_last_use[req.n] = req.done

    def _collect(self):
        for k, live in enumerate(self.slot_live):
            if live is None or not self.batches[k].poll():
                continue
            stats, _ = self.batches[k].stats()
            with self.torch.cuda.stream(self.streams[k]):
                host = [self._download(x.snap) for x in live]
            for x, st, h in zip(live, stats, host):
                x.req.snapshots = h.reshape(x.req.steps, -1)
                x.req.stats = st
                self.idle[x.key].append(x.problem)
                self._finish(x.req, x.snap_bytes)
            self.slot_live[k] = None

    # -------------------------------------------------------------- direct lane
    def _start_direct(self, req, mesh, P, snap_bytes, key, k):
        torch = self.torch
        st = self.direct_streams[k]
        with torch.cuda.stream(st):
            if P is None:
                P = L.Problem(mesh, req.bcs, req.DT, req.dt, self._opts(True, mesh), stream=st)
            else:
                P.reset(req.bcs, req.DT, req.dt)
            snap = torch.empty((req.steps, mesh.n_cells), dtype=torch.float64, device="cuda")
            if self.group is not None:
                # T0 goes up on the lane's stream and the group copies it into
                # the problem there: no wait on the host
                h = torch.from_numpy(np.ascontiguousarray(req.T0, dtype=np.float64)).pin_memory()
                T0 = torch.empty(h.shape, dtype=torch.float64, device="cuda")
                T0.copy_(h, non_blocking=True)
                self.group.add(P, req.steps, snap, T0=T0)   # the whole run; _step_direct advances the group
            else:
                self._upload_T(P, req.T0)
                P.step_begin(req.steps, snap)        # the whole run; _step_direct advances it
        req.launched = self.now()
        self.direct_slot[k] = _Direct(req, P, snap, snap_bytes, key, k, 0, [])

    def _step_direct(self):
        """Advance every running direct-lane request as far as its finished device
        work allows (lf_step_poll: no waiting) and finish those whose last step
        is done."""
        torch = self.torch
        if self.group is not None:
            # snapshots on their way to the host: finished once their copy is
            for item in list(self.draining):
                ev, req, snap, host, snap_bytes = item
                if not ev.query():
                    continue
                self.draining.remove(item)
                req.snapshots = host.numpy().reshape(req.steps, -1)
                self._finish(req, snap_bytes)
            done = self.group.poll()
            if not done:
                return
            by_problem = {id(d.problem): k for k, d in enumerate(self.direct_slot) if d is not None}
            for P, stats in done:
                k = by_problem[id(P)]
                d = self.direct_slot[k]
                req = d.req
                self.idle[d.key].append(d.problem)
                self.direct_slot[k] = None
                if any(st["nonfinite"] for st in stats):
                    req.error = "direct lane: non-finite residual"
                    self._finish(req, d.snap_bytes)
                    continue
                req.stats = stats
                st = self.direct_streams[k]
                host = torch.empty(d.snap.shape, dtype=d.snap.dtype, pin_memory=True)
                with torch.cuda.stream(st):
                    host.copy_(d.snap, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(st)
                self.draining.append((ev, req, d.snap, host, d.snap_bytes))
            return
        for k, d in enumerate(self.direct_slot):
            if d is None:
                continue
            _, finished, stats, status = d.problem.step_poll()
            if not finished:
                continue
            req = d.req
            failed = status == L.LF_ENONFINITE
            if failed:
                req.error = "direct lane: non-finite residual"
            else:
                with torch.cuda.stream(self.direct_streams[k]):
                    req.snapshots, req.stats = self._download(d.snap), stats
            self.idle[d.key].append(d.problem)
            self._finish(req, d.snap_bytes)
            self.direct_slot[k] = None

    # -------------------------------------------------------------- loop
    def pump(self):
        """One scheduling pass: collect finished work, admit, launch, and advance
        the running direct-lane requests."""
        self._collect()
        self._admit()
        self._launch()
        self._step_direct()

    def idle_now(self):
        return not self.queue and not self._anything_live()

    def run(self, requests: List[Request], poll_s=0.0002, progress=None, every=64):
        """Serve requests whose `arrival` times (seconds) are on this server's clock,
        starting now.  Returns the requests finished by this call.  progress(done,
        total) is called each time another `every` requests have finished."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        self.finished = []
        i = 0
        reported = 0
        while i < len(pending) or not self.idle_now():
            t = self.now()
            while i < len(pending) and pending[i].arrival <= t:
                self.submit(pending[i])
                i += 1
            self.pump()
            if progress is not None and len(self.finished) >= reported + every:
                reported = len(self.finished) // every * every
                progress(len(self.finished), len(pending))
            if poll_s:
                time.sleep(poll_s)
        return self.finished

    def close(self):
        if self.group is not None:
            self.group.close()
            self.group = None
        for key in list(self.idle):
            self._close_idle(key)
        for b in self.batches:
            b.close()
        for m in self.meshes.values():
            m.close()
        self.meshes.clear()


def _desc_of(mesh):
    """lf_mesh_desc of a host mesh (keeps its arrays alive while in use)."""
    keep = dict(
        owner=np.ascontiguousarray(mesh.owner, dtype=np.int32),
        neighbour=np.ascontiguousarray(mesh.neighbour, dtype=np.int32),
        cell_volume=np.ascontiguousarray(mesh.cell_volume, dtype=np.float64),
        cell_centre=np.ascontiguousarray(mesh.cell_centre, dtype=np.float64),
        face_area=np.ascontiguousarray(mesh.face_area, dtype=np.float64),
        patch_start=np.ascontiguousarray(mesh.patch_start, dtype=np.int32),
        bface_cell=np.ascontiguousarray(mesh.bface_cell, dtype=np.int32),
        bface_area=np.ascontiguousarray(mesh.bface_area, dtype=np.float64),
        bface_centre=np.ascontiguousarray(mesh.bface_centre, dtype=np.float64))
    d = L.lf_mesh_desc()
    d.n_cells, d.n_faces = mesh.n_cells, mesh.n_faces
    d.n_patches = keep["patch_start"].size - 1
    for k, v in keep.items():
        setattr(d, k, v.ctypes.data)
    return d, keep


def summarize(finished, t_first_arrival=0.0):
    lat = sorted(r.latency for r in finished if r.latency is not None)
    if not lat:
        return {}
    end = max(r.done for r in finished)
    pct = lambda q: lat[min(len(lat) - 1, int(round(q / 100.0 * (len(lat) - 1))))]
    return {"requests": len(lat), "solves_per_s": len(lat) / max(end - t_first_arrival, 1e-9),
            "p50_latency_s": pct(50), "p99_latency_s": pct(99), "max_latency_s": lat[-1],
            "mean_latency_s": float(np.mean(lat))}
