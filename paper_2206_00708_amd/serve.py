"""Serving form: a continuous-batching request loop of transmission solves.

Each request carries two meshes of one closed surface, wavenumbers, densities
and 1-16 plane-wave directions.  `Server` keeps `slots` workers, each owning a
context with its own HIP stream, so the device work of admitted requests
overlaps.  A free worker takes the next request in arrival order, builds its
mesh tables and asks for admission (`Admission`): a request enters when its
device footprint (bem_problem_footprint: operators, projections, Krylov
state, assembly scratch) fits beside the footprints already admitted, within
the HBM budget, and it is the oldest waiting request, or the oldest waiting
one does not fit and has been passed over fewer than `max_bypass` times (so
a large request at the head does not hold back smaller ones that fit, and
is itself admitted after at most `max_bypass` of them).  Operators and
Krylov state stay resident in HBM while the request runs; all its
directions are solved together (one matrix-core product per step for the
complex64 form).  Latency is completion time minus arrival time, split into
queueing (arrival to admission) and service (admission to completion).
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


class Admission:
    """Admission by device footprint within a byte budget.  Requests wait in
    arrival order; a request is admitted when it fits and either is the
    oldest waiting one or the oldest does not fit and has been bypassed fewer
    than `max_bypass` times.  Thread-safe; `admit` blocks until admission."""

    def __init__(self, budget, max_bypass=4):
        self.budget, self.max_bypass = budget, max_bypass
        self._cv = threading.Condition()
        self._in_use = 0
        self._waiting = []    # request ids in arrival order, not yet admitted
        self._need = {}       # footprint of the waiting requests that asked for admission
        self._bypassed = {}   # times each waiting request was passed over
        self.order = []       # admission order (ids)

    def arrive(self, rid):
        with self._cv:
            self._waiting.append(rid)
            self._bypassed[rid] = 0

    def withdraw(self, rid):
        with self._cv:
            if rid in self._waiting:
                self._waiting.remove(rid)
                self._need.pop(rid, None)
                self._cv.notify_all()

    def _may_enter(self, rid, nbytes):
        if self._in_use + nbytes > self.budget:
            return False
        head = self._waiting[0]
        if head == rid:
            return True
        # the head has not asked yet, or does not fit: pass it, within the bound
        head_need = self._need.get(head)
        head_fits = head_need is not None and self._in_use + head_need <= self.budget
        return not head_fits and self._bypassed[head] < self.max_bypass

    def admit(self, rid, nbytes):
        with self._cv:
            if nbytes > self.budget:
                self._waiting.remove(rid)
                self._cv.notify_all()
                raise A.BemError(-5, f"request needs {nbytes} bytes, above the budget {self.budget}")
            self._need[rid] = nbytes
            while not self._may_enter(rid, nbytes):
                self._cv.wait()
            i = self._waiting.index(rid)
            for older in self._waiting[:i]:
                self._bypassed[older] += 1
            self._waiting.pop(i)
            self._need.pop(rid)
            self._in_use += nbytes
            self.order.append(rid)
            self._cv.notify_all()

    def release(self, nbytes):
        with self._cv:
            self._in_use -= nbytes
            self._cv.notify_all()


class Server:
    """Worker contexts on one device, admission by footprint (`Admission`)."""

    def __init__(self, device=0, slots=4, hbm_budget_bytes=None, precision=A.C64_MIXED, tol=1e-6, maxit=500,
                 max_bypass=4):
        self.device, self.slots, self.precision, self.tol, self.maxit = device, slots, precision, tol, maxit
        if hbm_budget_bytes is None:
            free, total = torch.cuda.mem_get_info(device)
            hbm_budget_bytes = int(0.8 * free)
        self.budget = hbm_budget_bytes
        self.adm = Admission(hbm_budget_bytes, max_bypass)
        self.streams = [torch.cuda.Stream(device) for _ in range(slots)]
        self.ctx = [A.Context(device, stream=s) for s in self.streams]

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
                self.adm.admit(req.id, res.footprint)
                admitted = True
                res.t_admit = time.perf_counter()
                p.assemble_operators()
                p.assemble_projection()
                out, stats, code = p.solve(req.dirs, tol=self.tol, maxit=self.maxit, batch=len(req.dirs))
                res.traces = out.cpu().numpy()
            res.stats, res.code = stats, code
        except Exception as e:   # the request fails alone; the loop goes on
            res.error = f"{type(e).__name__}: {e}"
            self.adm.withdraw(req.id)
        finally:
            for h in (p, mi, me):
                if h is not None:
                    h.close()
            if admitted:
                ctx.trim()   # the assembly scratch counts in this request's footprint only
            res.t_done = time.perf_counter()
            if admitted:
                self.adm.release(res.footprint)

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
                self.adm.arrive(r.id)
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
        conv = [r for r in requests if results[r.id].error is None and results[r.id].code == A.OK]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        queue = np.array([r.t_admit - r.t_arrival for r in ok]) if ok else np.zeros(1)
        service = np.array([r.t_done - r.t_admit for r in ok]) if ok else np.zeros(1)
        solves = sum(len(r.dirs) for r in conv)
        pct = lambda a, q: round(1e3 * float(np.percentile(a, q)), 1)
        summary = {
            "requests": len(requests), "completed": len(ok), "converged": len(conv),
            "not_converged": sum(1 for r in ok if r.code == A.W_NOCONV),
            "errors": sum(1 for r in results.values() if r.error is not None),
            "solves": solves, "solves_unconverged": sum(len(r.dirs) for r in requests
                                                       if results[r.id].error is None) - solves,
            "makespan_s": round(makespan, 3),
            "solves_per_s": round(solves / makespan, 3), "requests_per_s": round(len(conv) / makespan, 3),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "queue_p50_ms": pct(queue, 50), "queue_p99_ms": pct(queue, 99),
            "service_p50_ms": pct(service, 50), "service_p99_ms": pct(service, 99),
            "admitted_out_of_order": sum(1 for a, b in zip(self.adm.order, sorted(self.adm.order)) if a != b),
            "slots": self.slots, "budget_bytes": self.budget,
        }
        return results, summary

    def close(self):
        for c in self.ctx:
            c.close()
