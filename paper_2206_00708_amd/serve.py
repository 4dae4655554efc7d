"""Serving form: a continuous-batching request loop of transmission solves.

Each request carries two meshes of one closed surface, wavenumbers, densities
and 1-16 plane-wave directions.  `Server` keeps `slots` workers, each owning a
context with its own HIP stream, so the device work of admitted requests
overlaps.  A free worker takes the next request in arrival order, builds its
mesh tables and asks for admission: the request enters when it is the oldest
waiting one and its device footprint (bem_problem_footprint: operators,
projections, Krylov state, assembly scratch) fits beside the footprints
already admitted, within the HBM budget; otherwise it waits until a finishing
request frees memory.  Operators
and Krylov state stay resident in HBM while the request runs; all its
directions are solved together (one matrix-core product per step for the
complex64 form).  Latency is completion time minus arrival time.
"""
import threading
import time

import numpy as np
import torch

from . import api as A


class Request:
    def __init__(self, rid, t_arrival, ext, inte, k_ext, k_int, rho_ext, rho_int, dirs):
        self.id, self.t_arrival = rid, t_arrival
        self.ext, self.inte = ext, inte
        self.k_ext, self.k_int, self.rho_ext, self.rho_int = k_ext, k_int, rho_ext, rho_int
        self.dirs = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)


class Result:
    def __init__(self, rid):
        self.id = rid
        self.traces = None
        self.stats = None
        self.code = None
        self.error = None
        self.footprint = 0
        self.slot = -1
        self.t_arrival = self.t_admit = self.t_done = 0.0

    @property
    def latency(self):
        return self.t_done - self.t_arrival


class Server:
    """Worker contexts on one device, admission by footprint, arrival-order queue."""

    def __init__(self, device=0, slots=4, hbm_budget_bytes=None, precision=A.C64_MIXED, tol=1e-6, maxit=500):
        self.device, self.slots, self.precision, self.tol, self.maxit = device, slots, precision, tol, maxit
        if hbm_budget_bytes is None:
            free, total = torch.cuda.mem_get_info(device)
            hbm_budget_bytes = int(0.8 * free)
        self.budget = hbm_budget_bytes
        self.streams = [torch.cuda.Stream(device) for _ in range(slots)]
        self.ctx = [A.Context(device, stream=s) for s in self.streams]
        self._cv = threading.Condition()
        self._in_use = 0
        self._waiting = []   # request ids in arrival order, not yet admitted

    # -- admission ----------------------------------------------------------
    def _admit(self, rid, nbytes):
        """Block until the request is at the head of the waiting line and its
        footprint fits beside the admitted ones."""
        with self._cv:
            if nbytes > self.budget:
                self._waiting.remove(rid)
                self._cv.notify_all()
                raise A.BemError(-5, f"request needs {nbytes} bytes, above the budget {self.budget}")
            while not (self._waiting[0] == rid and self._in_use + nbytes <= self.budget):
                self._cv.wait()
            self._waiting.pop(0)
            self._in_use += nbytes
            self._cv.notify_all()

    def _release(self, nbytes):
        with self._cv:
            self._in_use -= nbytes
            self._cv.notify_all()

    # -- one request ----------------------------------------------------------
    def _serve(self, req, res, slot):
        """Runs on the worker thread that owns `slot` (its context and stream);
        the library calls release the GIL (ctypes)."""
        ctx = self.ctx[slot]
        me = mi = p = None
        admitted = False
        res.slot = slot
        try:
            with torch.cuda.stream(self.streams[slot]):
                me = A.Mesh(ctx, *req.ext)
                mi = A.Mesh(ctx, *req.inte)
                p = A.Problem(ctx, me, mi, req.k_ext, req.k_int, req.rho_ext, req.rho_int, precision=self.precision)
                res.footprint = p.footprint(len(req.dirs), self.maxit)
                self._admit(req.id, res.footprint)
                admitted = True
                res.t_admit = time.perf_counter()
                p.assemble_operators()
                p.assemble_projection()
                out, stats, code = p.solve(req.dirs, tol=self.tol, maxit=self.maxit, batch=len(req.dirs))
                res.traces = out.cpu().numpy()
            res.stats, res.code = stats, code
        except Exception as e:   # the request fails alone; the loop goes on
            res.error = f"{type(e).__name__}: {e}"
            with self._cv:
                if req.id in self._waiting:
                    self._waiting.remove(req.id)
                    self._cv.notify_all()
        finally:
            for h in (p, mi, me):
                if h is not None:
                    h.close()
            if admitted:
                ctx.trim()   # the assembly scratch counts in this request's footprint only
            res.t_done = time.perf_counter()
            if admitted:
                self._release(res.footprint)

    # -- a stream ------------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve `requests` (arrival times in seconds from the start).  With
        realtime, each request is released at its arrival time; otherwise all
        are available at once.  Returns (results by id, summary)."""
        results = {r.id: Result(r.id) for r in requests}
        order = sorted(requests, key=lambda r: r.t_arrival)
        queue, qcv = [], threading.Condition()
        done_feeding = [False]
        t0 = time.perf_counter()

        def feeder():
            for r in order:
                if realtime:
                    dt = t0 + r.t_arrival - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                results[r.id].t_arrival = t0 + r.t_arrival if realtime else t0
                with self._cv:
                    self._waiting.append(r.id)
                with qcv:
                    queue.append(r)
                    qcv.notify()
            with qcv:
                done_feeding[0] = True
                qcv.notify_all()

        def worker(w):
            while True:
                with qcv:
                    while not queue and not done_feeding[0]:
                        qcv.wait()
                    if not queue:
                        return
                    r = queue.pop(0)
                self._serve(r, results[r.id], w)

        threads = [threading.Thread(target=feeder)] + [threading.Thread(target=worker, args=(w,))
                                                      for w in range(self.slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        makespan = time.perf_counter() - t0
        ok = [results[r.id] for r in requests if results[r.id].error is None]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        solves = sum(len(r.dirs) for r in requests if results[r.id].error is None)
        summary = {
            "requests": len(requests), "completed": len(ok),
            "not_converged": sum(1 for r in ok if r.code == A.W_NOCONV),
            "errors": sum(1 for r in results.values() if r.error is not None),
            "solves": solves, "makespan_s": round(makespan, 3),
            "solves_per_s": round(solves / makespan, 3), "requests_per_s": round(len(ok) / makespan, 3),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 1),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 1),
            "slots": self.slots, "budget_bytes": self.budget,
        }
        return results, summary

    def close(self):
        for c in self.ctx:
            c.close()
