"""Serving loop for parametric heat-equation solves (snapshot generation).

A request is (cube side n, DT, dt, number of steps, T0); its answer is T after
every step.  The server keeps the meshes (one per side, shared by all requests
of that side) and every admitted request's fields resident on the device, and
runs continuous batching over several launch slots, each a stream with its own
batched-kernel task table:

* admission: a queued request is admitted when its device bytes (problem
  workspace + snapshot buffer, plus its mesh if that is not resident yet) fit
  the HBM budget; resident meshes no admitted request uses are evicted first
  when memory is short;
* launch: whenever a slot is free, the admitted requests not yet running
  (largest first, up to a slot's capacity, one workgroup size per launch) go
  into that slot's persistent batched kernel, so requests that arrive while
  others run start on free slots and their work overlaps on the device;
* completion: a finished slot's snapshots are copied to the host, its
  requests' memory returns to the budget, and their latency (arrival to
  results on the host) is recorded.

Every request's result is independent of what it shares the GPU with: the
batched kernel solves each problem inside one workgroup with fixed-order sums,
and the workgroup size comes from the autotuner's table for the request's
size.
"""
import collections
import time
from dataclasses import dataclass, field
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
    nbytes: int


class Server:
    def __init__(self, mesh_for_side, budget_bytes, n_slots=4, slot_capacity=64, max_steps=10,
                 tuning=None):
        import torch
        self.torch = torch
        self.mesh_for_side = mesh_for_side          # side -> mesh description (host arrays)
        self.budget = int(budget_bytes)
        self.used = 0
        self.slot_capacity = slot_capacity
        self.max_steps = max_steps
        self.tuning = tuning if tuning is not None else autotune.load()
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.batches = [L.Batch(slot_capacity, max_steps, stream=s) for s in self.streams]
        self.slot_live: List[Optional[List[_Live]]] = [None] * n_slots
        self.meshes: Dict[int, object] = {}          # side -> L.Mesh
        self.mesh_bytes: Dict[int, int] = {}
        self.mesh_users: Dict[int, int] = collections.defaultdict(int)
        self.mesh_last_use: Dict[int, float] = {}
        self.queue = collections.deque()              # arrived, not admitted
        self.ready: List[_Live] = []                  # admitted, not launched
        self.finished: List[Request] = []
        self.t0 = time.perf_counter()
        self.rejected: List[Request] = []

    # ------------------------------------------------------------------ clock
    def now(self):
        return time.perf_counter() - self.t0

    # -------------------------------------------------------------- memory
    def _request_bytes(self, req, mesh):
        opts = L.make_opts(precision=L.LF_PREC_MIXED, layout=L.LF_LAYOUT_ROWS)
        return L.lf_problem_workspace_bytes(mesh.h, opts) + 8 * req.steps * mesh.n_cells

    def preload_mesh(self, side):
        """Make a side's mesh resident (counted in the budget)."""
        if side in self.meshes:
            return self.meshes[side]
        m = L.Mesh(self.mesh_for_side(side))
        self.meshes[side] = m
        self.mesh_bytes[side] = m.ws_bytes
        self.used += m.ws_bytes
        self.mesh_last_use[side] = self.now()
        return m

    def _evict_meshes(self, need):
        idle = sorted((t, s) for s, t in self.mesh_last_use.items()
                      if self.mesh_users[s] == 0 and s in self.meshes)
        for _, s in idle:
            if self.used + need <= self.budget:
                break
            self.meshes.pop(s).close()
            self.used -= self.mesh_bytes.pop(s)
            self.mesh_last_use.pop(s, None)

    # -------------------------------------------------------------- requests
    def submit(self, req: Request):
        if req.steps > self.max_steps:
            req.error = f"at most {self.max_steps} steps per request"
            self.rejected.append(req)
            return
        self.queue.append(req)

    def _admit(self):
        while self.queue:
            req = self.queue[0]
            mesh_new = req.n not in self.meshes
            if mesh_new:
                # size the mesh from its description before building it
                desc = self.mesh_for_side(req.n)
                d = _desc_of(desc)
                mbytes = L.lf_mesh_workspace_bytes(d[0])
            else:
                mbytes = 0
            if mesh_new:
                self._evict_meshes(mbytes)
                if self.used + mbytes > self.budget:
                    if not self._anything_live():
                        self.queue.popleft()
                        req.error = "mesh larger than the device-memory budget"
                        self.rejected.append(req)
                        continue
                    return
                mesh = self.preload_mesh(req.n)
            else:
                mesh = self.meshes[req.n]
            need = self._request_bytes(req, mesh)
            if self.used + need > self.budget:
                self._evict_meshes(need)
            if self.used + need > self.budget:
                if not self._anything_live():
                    self.queue.popleft()
                    req.error = "request larger than the device-memory budget"
                    self.rejected.append(req)
                    continue
                return
            self.queue.popleft()
            P = L.Problem(mesh, req.bcs, req.DT, req.dt,
                          L.make_opts(precision=L.LF_PREC_MIXED, layout=L.LF_LAYOUT_ROWS))
            P.set_T(req.T0)
            snap = self.torch.empty(req.steps * mesh.n_cells, dtype=self.torch.float64, device="cuda")
            self.used += need
            self.mesh_users[req.n] += 1
            req.admitted = self.now()
            self.ready.append(_Live(req, P, snap, need))

    def _anything_live(self):
        return bool(self.ready) or any(s is not None for s in self.slot_live)

    def _launch(self):
        for k, live in enumerate(self.slot_live):
            if live is not None or not self.ready:
                continue
            # largest first; one workgroup size and one step count per launch
            self.ready.sort(key=lambda x: -x.problem.mesh.n_cells)
            bs = autotune.block_threads_for(self.ready[0].req.n, self.tuning)
            steps = self.ready[0].req.steps
            group = [x for x in self.ready
                     if autotune.block_threads_for(x.req.n, self.tuning) == bs
                     and x.req.steps == steps][: self.slot_capacity]
            for x in group:
                self.ready.remove(x)
            # the problems' set-up (workspace clearing, T) finished synchronously
            # on their own stream when they were admitted
            self.batches[k].launch([x.problem for x in group], steps, block_threads=bs,
                                   snapshots=[x.snap for x in group])
            t = self.now()
            for x in group:
                x.req.launched = t
            self.slot_live[k] = group

    def _collect(self):
        for k, live in enumerate(self.slot_live):
            if live is None or not self.batches[k].poll():
                continue
            stats, _ = self.batches[k].stats()
            with self.torch.cuda.stream(self.streams[k]):
                host = [x.snap.to("cpu", non_blocking=False) for x in live]
            t = self.now()
            for x, st, h in zip(live, stats, host):
                x.req.snapshots = h.numpy().reshape(x.req.steps, -1)
                x.req.stats = st
                x.req.done = t
                self.finished.append(x.req)
                x.problem.close()
                self.used -= x.nbytes
                self.mesh_users[x.req.n] -= 1
                self.mesh_last_use[x.req.n] = t
            self.slot_live[k] = None

    def pump(self):
        """One scheduling pass: collect finished slots, admit, launch."""
        self._collect()
        self._admit()
        self._launch()

    def idle(self):
        return not self.queue and not self._anything_live()

    def run(self, requests: List[Request], poll_s=0.0002):
        """Serve requests whose `arrival` times (seconds) are on this server's clock,
        starting now.  Returns when every request has finished."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        while i < len(pending) or not self.idle():
            t = self.now()
            while i < len(pending) and pending[i].arrival <= t:
                self.submit(pending[i])
                i += 1
            self.pump()
            if poll_s:
                time.sleep(poll_s)
        return self.finished

    def close(self):
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
