"""Serving form: a request loop with continuous batching.

Each request asks for one assembly + sensitivity + compliance (Sec. 3.2,
Appendix D) on a structured Q1 mesh (2D n x n quads or 3D n x n x n hexes)
with its own densities, penalisation p and displacement field.  The loop

* keeps one CSR pattern/plan per distinct mesh resident on the device (built
  the first time the mesh is seen: the once-per-mesh work of Sec. 3.2.2);
* admits waiting requests in arrival order while a stream slot is free and
  the HBM footprint of the admitted requests stays within a budget;
* runs each admitted request on its own stream, so requests that arrive
  while others are on the GPU overlap with them on the device;
* retires requests whose completion event has fired, freeing their slot and
  memory, and records latency = completion - arrival; when no waiting request
  can be admitted it blocks on the oldest request's completion event instead
  of polling.

Each request is one soptx_step call (assembly with the mesh's Dirichlet
table bound once, dc and c) into outputs allocated before the run: one K
buffer per stream slot, and dc and c per request.

Every kernel sums in a fixed order and no request shares an output with
another, so a request's result is bitwise the same alone and in any mix.

The scheduling logic (Scheduler) is host code over an executor interface so
it can be tested without a GPU; GpuExecutor runs the library.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

__all__ = ["Request", "Result", "Scheduler", "GpuExecutor", "make_requests", "latency_stats", "serve"]


@dataclasses.dataclass
class Request:
    rid: int
    kind: str            # "quad" (n x n Q1 quads) or "hex" (n x n x n Q1 hexes)
    n: int
    p: float
    arrival: float = 0.0  # seconds from the start of the run
    seed: int = 0

    @property
    def mesh_key(self) -> Tuple[str, int]:
        return (self.kind, self.n)

    @property
    def n_cells(self) -> int:
        return self.n ** 2 if self.kind == "quad" else self.n ** 3


@dataclasses.dataclass
class Result:
    rid: int
    n_cells: int
    arrival: float
    start: float
    finish: float
    dc: object = None     # device tensor [n_cells]
    c: object = None      # device tensor [2]: u^T K u, f^T u (0 here)
    K: object = None      # device tensor [nnz] (the executor's keep_K), else None

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def request_footprint(kind: str, n: int) -> int:
    """Device bytes a request holds while admitted: K values, rho, u, dc, c."""
    if kind == "quad":
        nn, nc, d = (n + 1) ** 2, n * n, 2
        nnz = 4 * (3 * n + 1) ** 2
    else:
        nn, nc, d = (n + 1) ** 3, n ** 3, 3
        nnz = 9 * (3 * n + 1) ** 3
    return nnz * 8 + nc * 8 * 2 + nn * d * 8 + 16


class Scheduler:
    """Continuous batching over an executor.

    executor.launch(req, slot) -> handle   (asynchronous; slot in [0, slots))
    executor.done(handle) -> bool
    executor.wait(handle)                  (blocks until done)
    executor.finish(handle) -> (dc, c) or (dc, c, K)   (called once done)
    executor.now() -> seconds
    """

    def __init__(self, executor, slots: int, hbm_budget: int, footprint: Callable[[Request], int] = None):
        if slots < 1 or hbm_budget <= 0:
            raise ValueError("need at least one slot and a positive HBM budget")
        self.ex = executor
        self.slots = slots
        self.budget = hbm_budget
        self.footprint = footprint or (lambda r: request_footprint(r.kind, r.n))
        self.in_use = 0
        self.free_slots = list(range(slots))
        self.admission_log: List[Tuple[int, int]] = []  # (rid, bytes in use after admission)

    def run(self, requests: List[Request], poll_sleep: float = 0.0) -> List[Result]:
        for r in requests:
            if self.footprint(r) > self.budget:
                raise ValueError(f"request {r.rid} needs {self.footprint(r)} bytes > budget {self.budget}")
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        waiting: List[Request] = []
        inflight: Dict[int, Tuple[Request, object, int, float]] = {}
        results: List[Result] = []
        i = 0
        while i < len(pending) or waiting or inflight:
            now = self.ex.now()
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            # retire
            for rid in [k for k, v in inflight.items() if self.ex.done(v[1])]:
                req, h, slot, t0 = inflight.pop(rid)
                out = self.ex.finish(h)
                results.append(Result(rid, req.n_cells, req.arrival, t0, self.ex.now(), out[0], out[1],
                                      out[2] if len(out) > 2 else None))
                self.in_use -= self.footprint(req)
                self.free_slots.append(slot)
            # admit in arrival order (no overtaking: the head waits for room)
            while waiting and self.free_slots and self.in_use + self.footprint(waiting[0]) <= self.budget:
                req = waiting.pop(0)
                slot = self.free_slots.pop(0)
                self.in_use += self.footprint(req)
                self.admission_log.append((req.rid, self.in_use))
                inflight[req.rid] = (req, self.ex.launch(req, slot), slot, self.ex.now())
            if not inflight and not waiting and i < len(pending):
                self.ex.wait_until(pending[i].arrival)
            elif inflight and waiting and (i >= len(pending) or pending[i].arrival > self.ex.now()):
                # the head of the queue waits for a slot or for memory: block
                # on the oldest request in flight
                self.ex.wait(min(inflight.values(), key=lambda v: v[3])[1])
            elif poll_sleep > 0:
                time.sleep(poll_sleep)
        return sorted(results, key=lambda r: r.rid)


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    span = max(r.finish for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "elements_per_s": float(sum(r.n_cells for r in results) / span), "makespan_s": float(span)}


def make_requests(count: int, rate_elems_per_s: Optional[float] = None, first_rid: int = 0) -> List[Request]:
    """Seeded requests (inputs.serving_request); Poisson arrivals whose mean
    offered load is rate_elems_per_s, or all at t = 0 (burst) when None."""
    from . import inputs as I
    reqs = []
    for k in range(count):
        rid = first_rid + k
        kind, n, p, _ = I.serving_request(rid)
        reqs.append(Request(rid, kind, n, p, 0.0, seed=rid))
    if rate_elems_per_s:
        mean_elems = float(np.mean([r.n_cells for r in reqs]))
        rng = np.random.default_rng(4999)
        gaps = rng.exponential(mean_elems / rate_elems_per_s, size=count)
        t = np.cumsum(gaps) - gaps[0]
        for r, a in zip(reqs, t):
            r.arrival = float(a)
    return reqs


class GpuExecutor:
    """Runs requests through the library on a pool of streams.

    prepare() builds the resident meshes (pattern, plan and the bound
    Dirichlet table of each distinct mesh), puts every request's inputs in
    HBM (or, with pcie=True, in pinned host memory, copied to the slot's
    device buffers at launch), and allocates the outputs: one K buffer per
    slot (the largest request's size) and dc and c per request.  A launch then
    allocates nothing and makes one library call.  keep_K gives every request
    a K of its own, returned in its Result (for tests)."""

    def __init__(self, slots: int, device: int = 0, pcie: bool = False, keep_K: bool = False):
        import torch

        from . import api
        self.torch, self.api = torch, api
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]  # default priority
        self.meshes: Dict[Tuple[str, int], tuple] = {}
        self.t0 = time.perf_counter()
        self.pcie, self.keep_K = pcie, keep_K
        self.staged: Dict[int, tuple] = {}
        self.outputs: Dict[int, tuple] = {}
        self.slot_bufs: List[Optional[tuple]] = [None] * slots

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float):
        d = t - self.now()
        if d > 0:
            time.sleep(d)

    def resident(self, key):
        """(pattern, Dirichlet table, mesh, host mask), built once per distinct mesh."""
        if key not in self.meshes:
            from . import inputs as I
            kind, n = key
            mesh = I.quad_grid(n, n) if kind == "quad" else I.hex_grid(n, n, n)
            mask, _ = I.mbb_bc(mesh) if kind == "quad" else I.clamp_x0_bc(mesh)
            pat = self.api.Pattern.from_mesh(mesh)
            self.meshes[key] = (pat, self.api.Dirichlet(pat, mask), mesh, mask)
        return self.meshes[key]

    def request_inputs(self, req: Request):
        """Host inputs of a request: rho ~ U(0.001, 1), u ~ N(0, 1) zero on fixed dofs."""
        from . import inputs as I
        mesh, mask = self.resident(req.mesh_key)[2:]
        _, _, _, rng = I.serving_request(req.rid)
        return rng.uniform(0.001, 1.0, mesh.n_cells), I.synthetic_u(rng, mask)

    def prepare(self, requests: List[Request]):
        """Resident meshes, staged inputs and preallocated outputs, ahead of the timed run."""
        torch = self.torch
        nnz_max = cells_max = dof_max = 0
        for r in requests:
            pat = self.resident(r.mesh_key)[0]
            nnz_max, cells_max, dof_max = max(nnz_max, pat.nnz), max(cells_max, pat.n_cells), max(dof_max, pat.ndof)
            rho, u = self.request_inputs(r)
            if self.pcie:
                self.staged[r.rid] = (torch.from_numpy(rho).pin_memory(), torch.from_numpy(u).pin_memory())
            else:
                self.staged[r.rid] = (torch.from_numpy(rho).to(self.dev), torch.from_numpy(u).to(self.dev))
            self.outputs[r.rid] = (torch.empty(pat.n_cells, dtype=torch.float64, device=self.dev),
                                   torch.empty(2, dtype=torch.float64, device=self.dev),
                                   torch.empty(pat.nnz, dtype=torch.float64, device=self.dev) if self.keep_K else None)
        for k in range(len(self.streams)):
            cur = self.slot_bufs[k]
            if cur is None or cur[0].numel() < nnz_max or cur[1].numel() < cells_max or cur[2].numel() < dof_max:
                self.slot_bufs[k] = (torch.empty(nnz_max, dtype=torch.float64, device=self.dev),
                                     torch.empty(cells_max, dtype=torch.float64, device=self.dev),
                                     torch.empty(dof_max, dtype=torch.float64, device=self.dev))
        torch.cuda.synchronize(self.dev)

    def launch(self, req: Request, slot: int):
        torch = self.torch
        st = self.streams[slot]
        pat, bc = self.resident(req.mesh_key)[:2]
        if req.rid not in self.staged:
            self.prepare([req])
        rho_h, u_h = rho, u = self.staged.pop(req.rid)
        dc, c, Kown = self.outputs.pop(req.rid)
        Kslot, rho_slot, u_slot = self.slot_bufs[slot]
        if self.pcie:
            # asynchronous copies from pinned memory into the slot's buffers
            rho = self._h2d(rho_h, rho_slot, st)
            u = self._h2d(u_h, u_slot, st)
        K = Kown if Kown is not None else Kslot[: pat.nnz]
        mat = self.api.Material(E0=1.0, Emin=1e-9, nu=0.3, p=req.p)
        pat.step(mat, rho, u, bc=bc, K=K, dc=dc, c=c, stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        return (ev, dc, c, Kown, rho, u, rho_h, u_h)  # inputs (and pinned sources) live until the work is done

    def _h2d(self, src, buf, st):
        with self.torch.cuda.stream(st):
            return buf[: src.numel()].copy_(src, non_blocking=True)

    def done(self, h) -> bool:
        return h[0].query()

    def wait(self, h):
        h[0].synchronize()

    def finish(self, h):
        return h[1], h[2], h[3]


def serve(requests: List[Request], slots: int = 4, hbm_budget: int = 32 << 30, executor=None, keep_K: bool = False):
    """Run requests through a Scheduler on the GPU; returns (results, stats)."""
    ex = executor or GpuExecutor(slots, keep_K=keep_K)
    ex.prepare(requests)
    ex.t0 = time.perf_counter()
    sched = Scheduler(ex, slots, hbm_budget)
    results = sched.run(requests)
    return results, latency_stats(results)
