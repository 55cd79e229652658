"""Continuous-batching request loop over libgeneo.

Requests arrive at seeded Poisson times.  A request is either a new problem
(device Q1 assembly + GenEO setup + PCG solve; the operator then stays
resident on the device) or a repeat solve of a resident operator with a
batch of right-hand sides.  The dispatcher admits a request as soon as a
worker slot is free and its estimated device-memory footprint fits in the
budget (resident operators count against it; the oldest resident operator
is evicted when a new setup would not fit otherwise).  Each worker thread
owns its own HIP stream, so admitted requests overlap on the device; the
library calls release the GIL.  Latency = completion - arrival.

All numerical work runs in libgeneo's kernels; this module only schedules.
"""
import heapq
import threading
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import geneo as G


def _part_sizes(n, parts, ovl):
    base, extra = divmod(n, parts)
    out, lo = [], 0
    for p in range(parts):
        sz = base + (1 if p < extra else 0)
        elo, ehi = max(0, lo - ovl), min(n, lo + sz + ovl)
        out.append((elo, ehi))
        lo += sz
    return out


def footprint_bytes(prob):
    """Upper estimate of the device memory a setup + solve of ``prob`` needs:
    the assembled system, the local Cholesky factors with their inverted
    diagonal tiles, the transient shifted factors and eigen blocks, and the
    coarse data."""
    sizes = G.geneo_q1_sizes(G.grid_from_problem(prob))
    axes = [_part_sizes(prob.ne[a], prob.parts[a], prob.ovl) for a in range(prob.dim)]
    tot_loc = 0
    for idx in np.ndindex(*[len(a) for a in axes]):
        nn = prob.ncomp
        for a, i in enumerate(idx):
            elo, ehi = axes[a][i]
            nn *= (ehi - elo + 1)
        nt = (nn + 31) // 32
        tiles = nt * (nt + 1) // 2 * 1024
        loc_factor = tiles * (4 if prob.precision == "mixed" else 8)
        shifted = tiles * 8 * 2                 # factor + scratch copy
        eig = nt * 32 * 64 * 8 * 4              # U, W, T, Y at the largest block
        tot_loc += loc_factor + nt * 1024 * 8 + shifted + eig
    system = sizes["nnz"] * 12 + sizes["ndof"] * 64 + sizes["nnz_loc"] * 20 + sizes["nloc"] * 40
    nc = prob.nsub * (prob.nev_max if prob.tau else prob.nev)
    coarse = 3 * nc * nc * 8
    return int(system + tot_loc + coarse)


def resident_bytes(prob):
    """Device memory an operator keeps after its setup: the system, the local
    Cholesky factors (and their inverted diagonal tiles), the coarse basis
    and the coarse inverse."""
    sizes = G.geneo_q1_sizes(G.grid_from_problem(prob))
    axes = [_part_sizes(prob.ne[a], prob.parts[a], prob.ovl) for a in range(prob.dim)]
    fac = 0
    for idx in np.ndindex(*[len(a) for a in axes]):
        nn = prob.ncomp
        for a, i in enumerate(idx):
            elo, ehi = axes[a][i]
            nn *= (ehi - elo + 1)
        nt = (nn + 31) // 32
        fac += (nt * (nt + 1) // 2 + nt) * 1024 * (4 if prob.precision == "mixed" else 8)
    system = sizes["nnz"] * 12 + sizes["ndof"] * 64 + sizes["nnz_loc"] * 20 + sizes["nloc"] * 40
    nc = prob.nsub * (prob.nev_max if prob.tau else prob.nev)
    return int(system + fac + 2 * nc * nc * 8)


@dataclass(order=True)
class Request:
    arrival: float
    rid: int
    kind: str = field(compare=False)                 # "new" or "repeat"
    problem: object = field(compare=False, default=None)
    op_id: Optional[int] = field(compare=False, default=None)
    rhs: Optional[np.ndarray] = field(compare=False, default=None)   # (nrhs, n)
    result: dict = field(compare=False, default_factory=dict)


class Operator:
    def __init__(self, op_id, prob, sysm, handle, nbytes):
        self.op_id, self.prob, self.sysm, self.handle, self.nbytes = op_id, prob, sysm, handle, nbytes
        self.lock = threading.Lock()   # one solve at a time on the handle
        self.pins = 0                  # dispatched repeat requests not yet finished


class Server:
    """Admission-controlled, multi-stream executor of GenEO-PCG requests."""

    def __init__(self, hbm_budget_bytes, slots=4, keep_solutions=False):
        import torch
        self.budget = int(hbm_budget_bytes)
        self.slots = slots
        self.keep_solutions = keep_solutions
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.used = 0
        self.resident = {}          # op_id -> Operator (insertion order = age)
        self.cv = threading.Condition()
        self.free_slots = list(range(slots))
        self.done = []
        self.errors = []
        self.inflight_new = set()    # rids of new-problem requests still running
        self.peak_used = 0

    # ------------------------------------------------------------ workers
    def _run_new(self, req, stream):
        import torch
        prob = req.problem
        with torch.cuda.stream(stream):
            coeff = torch.as_tensor(prob.coeff, dtype=torch.float64, device="cuda")
            sysm = G.geneo_assemble_q1(G.grid_from_problem(prob), coeff, stream=stream)
            opts = G.opts_from_problem(prob)
            h = G.geneo_setup(sysm.csr(), sysm.subdomains(), sysm.neumann(), sysm.overlap(),
                              opts, stream=stream)
            x = torch.zeros_like(sysm.b)
            info = G.pcg_solve(sysm.csr(), h, sysm.b, x, rtol=prob.rtol, maxit=prob.maxit,
                               stream=stream)
            stream.synchronize()
        req.result.update(iters=info["iters"], converged=info["converged"],
                          relres=info["relres"], ndof=prob.ndof)
        if self.keep_solutions:
            req.result["x"] = x.cpu().numpy()
        return Operator(req.rid, prob, sysm, h, resident_bytes(prob))

    def _run_repeat(self, req, stream, op):
        import torch
        with op.lock, torch.cuda.stream(stream):
            nrhs, n = req.rhs.shape
            b = torch.as_tensor(req.rhs.reshape(-1), dtype=torch.float64, device="cuda")
            x = torch.zeros_like(b)
            infos = G.pcg_solve(op.sysm.csr(), op.handle, b, x, rtol=op.prob.rtol,
                                maxit=op.prob.maxit, nrhs=nrhs, stream=stream)
            stream.synchronize()
        infos = infos if isinstance(infos, list) else [infos]
        req.result.update(iters=[i["iters"] for i in infos],
                          converged=all(i["converged"] for i in infos), ndof=n * nrhs)
        if self.keep_solutions:
            req.result["x"] = x.cpu().numpy().reshape(nrhs, n)
        return None

    def _worker(self, req, slot, need, pinned):
        t_start = time.perf_counter()
        op = None
        try:
            if req.kind == "new":
                op = self._run_new(req, self.streams[slot])
            else:
                self._run_repeat(req, self.streams[slot], pinned)
        except Exception as e:  # recorded, not raised in the worker thread
            self.errors.append((req.rid, repr(e)))
        t_end = time.perf_counter()
        req.result["t_start"] = t_start
        req.result["t_end"] = t_end
        with self.cv:
            self.used -= need
            self.inflight_new.discard(req.rid)
            if pinned is not None:
                pinned.pins -= 1
            if op is not None:
                self.resident[op.op_id] = op
                self.used += op.nbytes
                self.peak_used = max(self.peak_used, self.used)
            self.free_slots.append(slot)
            self.done.append(req)
            self.cv.notify_all()

    # --------------------------------------------------------- dispatcher
    def _evict_for(self, need, keep):
        """Evict the oldest idle resident operators until `need` fits: never
        one pinned by a dispatched repeat request (pins are taken and dropped
        under self.cv, like this call), nor one in `keep`, which requests not
        yet dispatched still use."""
        for op_id in list(self.resident):
            if self.used + need <= self.budget:
                return
            op = self.resident[op_id]
            if op.pins or op_id in keep:
                continue
            del self.resident[op_id]
            self.used -= op.nbytes
            op.handle.close()

    def run(self, requests, t0=None):
        """Serve `requests` (sorted by arrival, seconds relative to t0)."""
        pending = list(requests)
        heapq.heapify(pending)
        wanted = {}                      # op_id -> repeat requests not yet dispatched
        for r in pending:
            if r.kind == "repeat":
                wanted[r.op_id] = wanted.get(r.op_id, 0) + 1
        t0 = time.perf_counter() if t0 is None else t0
        threads = []
        while pending:
            req = pending[0]
            now = time.perf_counter() - t0
            if req.arrival > now:
                time.sleep(min(req.arrival - now, 0.002))
                continue
            need = footprint_bytes(req.problem) if req.kind == "new" else 0
            skip = False
            with self.cv:
                while True:
                    if req.kind == "new":
                        if need > self.budget:
                            raise RuntimeError("request %d needs %d bytes > budget"
                                               % (req.rid, need))
                        self._evict_for(need, {k for k, v in wanted.items() if v > 0})
                    elif req.op_id not in self.resident and req.op_id not in self.inflight_new:
                        skip = True      # its operator failed or is gone
                        break
                    ready = req.kind == "new" or req.op_id in self.resident
                    if ready and self.free_slots and self.used + need <= self.budget:
                        break
                    self.cv.wait(0.01)
                pinned = None
                if not skip:
                    slot = self.free_slots.pop()
                    self.used += need
                    self.peak_used = max(self.peak_used, self.used)
                    if req.kind == "new":
                        self.inflight_new.add(req.rid)
                    else:
                        pinned = self.resident[req.op_id]
                        pinned.pins += 1
            heapq.heappop(pending)
            if req.kind == "repeat":
                wanted[req.op_id] -= 1
            if skip:
                self.errors.append((req.rid, "operator %d not available" % req.op_id))
                continue
            req.result["t_arrival"] = t0 + req.arrival
            th = threading.Thread(target=self._worker, args=(req, slot, need, pinned), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return self.stats()

    def stats(self):
        lat = np.array([r.result["t_end"] - r.result["t_arrival"] for r in self.done])
        span = (max(r.result["t_end"] for r in self.done) -
                min(r.result["t_arrival"] for r in self.done)) if self.done else 0.0
        dofs = sum(r.result.get("ndof", 0) for r in self.done)
        return {"requests": len(self.done), "errors": len(self.errors),
                "peak_bytes": self.peak_used, "budget_bytes": self.budget,
                "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
                "solves_per_s": len(self.done) / span if span > 0 else None,
                "dof_per_s": dofs / span if span > 0 else None}

    def close(self):
        for op in self.resident.values():
            op.handle.close()
        self.resident.clear()


def make_stream(seed=0, count=200, rate=None, mean_service_s=0.05, sizes2d=(128, 256, 512, 1024),
                sizes3d=(48, 64, 96), mix=(0.60, 0.25, 0.15), nrhs=8):
    """Seeded request stream shaped like the serving workload: 60% new 2D
    Darcy problems (GRF + inclusions, 32^2-element subdomains, overlap 2),
    25% new 3D layered problems (12^3-element subdomains, overlap 1), 15%
    repeat solves of an earlier operator with `nrhs` random right-hand sides.
    Arrivals are Poisson with `rate` per second (default 0.8/mean_service_s)."""
    import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    rate = rate if rate is not None else 0.8 / mean_service_s
    t, reqs, news = 0.0, [], []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        if u < mix[2] and news:
            src = news[int(rng.integers(len(news)))]
            n = src.problem.ndof
            rhs = rng.normal(size=(nrhs, n))
            reqs.append(Request(t, rid, "repeat", problem=src.problem, op_id=src.rid, rhs=rhs))
            continue
        if u < mix[2] + mix[1]:
            n = int(rng.choice(sizes3d))
            parts = max(1, n // 12)
            p = synth.layers_3d(seed=int(rng.integers(1 << 30)), n=n, parts=parts, ovl=1,
                                     nev=12, precision="mixed")
        else:
            n = int(rng.choice(sizes2d))
            parts = max(1, n // 32)
            p = synth.grf_2d(seed=int(rng.integers(1 << 30)), n=n, parts=parts, ovl=2,
                                  precision="mixed", inclusions=max(1, (24 * n * n) // (512 * 512)))
        r = Request(t, rid, "new", problem=p)
        reqs.append(r)
        news.append(r)
    return reqs
