"""Continuous-batching serving loop for AMG-PCG solves on one GPU.

Requests (a 7-point diffusion operator on an N^3 grid plus a right-hand
side) arrive over time. The scheduler admits a request as soon as a slot is
free and device memory allows it, so requests that arrive while others run
are started on other slots and their GPU work overlaps:

* Slots: ``slots`` worker threads, each with its own HIP stream. The C ABI
  releases the GIL, so the slots' setups and solves run concurrently.
* Hierarchy cache: built hierarchies stay resident on the device, keyed by
  operator id; a repeated operator skips the setup (the reuse the paper
  motivates for time-dependent and nonlinear sequences). Idle entries are
  evicted least-recently-used when memory is needed.
* Admission by footprint (by default the device's memory less a headroom of
  32 GiB, 256 GiB on one MI355X): a cache miss reserves the library's footprint
  estimate for the operator (amg_estimate_footprint) plus the solve's
  vectors; a hit reserves the vectors only. A request that cannot fit even
  into an empty device is rejected; one that does not fit now waits. Later
  requests may bypass a waiting one at most ``max_bypass`` times.
* Device check: the reservations leave out what else the device holds
  (allocator caches, freed blocks kept by the library's pool, runtime
  scratch). A backend that reports its free device memory gets a second
  test before each admission: free memory, less the reservations of the
  requests in flight and a margin, must cover the request; if it does not,
  the backend's caches are released and idle hierarchies evicted before the
  request waits.
* Two requests on the same operator never run at once (a hierarchy is used
  by one thread at a time); the second waits for the first.

Latency is completion minus arrival; the summary reports p50/p99 latency,
completed solves per second, cache hits, setups, rejections and the peak of
reserved memory. The scheduler is independent of the backend: tests drive
it with a CPU backend; ``GpuBackend`` runs the HIP library.
"""

from __future__ import annotations

import dataclasses
import queue
import sys
import threading
import time
from typing import Any, Dict, List, Optional

import numpy as np

__all__ = ["Request", "Result", "Server", "GpuBackend", "summarize", "requests_from_stream"]


@dataclasses.dataclass
class Request:
    req_id: int
    t_arrival: float  # seconds from the start of the stream
    op_id: int
    N: int
    eps: tuple = (1.0, 1.0)
    rhs_seed: int = 0


@dataclasses.dataclass
class Result:
    req_id: int
    op_id: int
    N: int
    t_arrival: float
    t_admit: float = 0.0
    t_done: float = 0.0
    slot: int = -1
    cache_hit: bool = False
    status: int = 0
    iterations: int = 0
    converged: bool = False
    rel_res_true: float = 0.0
    rejected: bool = False
    reserved: int = 0  # bytes reserved while in flight
    error: str = ""  # why a request failed
    retries: int = 0  # admissions repeated after the device ran out of memory
    x: Any = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def requests_from_stream(stream: List[dict]) -> List[Request]:
    """Converts inputs.serving_requests() dicts into Requests."""
    return [Request(r["req_id"], r["t_arrival"], r["op_id"], r["N"], tuple(r["eps"]),
                    r["rhs_seed"]) for r in stream]


@dataclasses.dataclass
class _Entry:
    handle: Any
    bytes: int
    busy: bool = True
    last_used: float = 0.0


class Server:
    """Admission, slot assignment and hierarchy caching over a backend.

    The backend provides: ``make_slot(i)``, ``estimate_bytes(req)`` (setup
    footprint), ``solve_bytes(req)``, ``build(req, slot) -> (handle,
    bytes)``, ``solve(handle, req, slot) -> dict`` and ``release(handle)``.
    """

    def __init__(self, backend, slots: int = 4, budget_bytes: int = 64 << 30,
                 max_bypass: int = 8, margin_bytes: int = 4 << 30):
        if slots < 1:
            raise ValueError("slots must be positive")
        self.backend = backend
        self.nslots = slots
        self.budget = int(budget_bytes)
        self.max_bypass = max_bypass
        self.cache: Dict[int, _Entry] = {}
        self.used = 0
        self.peak_used = 0
        self.events: List[tuple] = []  # (t, kind, req_id, slot)
        self._slot_state = [backend.make_slot(i) for i in range(slots)]
        self._inbox = [queue.Queue() for _ in range(slots)]
        self._done: queue.Queue = queue.Queue()
        self._threads = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                         for i in range(slots)]
        for t in self._threads:
            t.start()
        self.stats = {"setups": 0, "hits": 0, "evictions": 0, "rejected": 0,
                      "max_concurrency": 0, "memory_waits": 0, "oom_retries": 0}
        self.max_oom_retries = 2
        self.inflight = 0  # reservations of the requests in flight
        self.margin = int(margin_bytes)
        self.device_used_peak = 0
        self._last_release = -1e9

    # -- workers -------------------------------------------------------------

    def _worker(self, i):
        while True:
            job = self._inbox[i].get()
            if job is None:
                return
            req, entry, build, t0 = job
            err = None
            out: Optional[dict] = None
            built = None
            try:
                if build:
                    built = self.backend.build(req, self._slot_state[i])
                    handle = built[0]
                else:
                    handle = entry.handle
                out = self.backend.solve(handle, req, self._slot_state[i])
            except Exception as e:  # reported, never raised on this thread
                err = e
            self._done.put((i, req, entry, built, out, err, time.perf_counter() - t0))

    def close(self):
        for q in self._inbox:
            q.put(None)
        for t in self._threads:
            t.join(timeout=30)
        for e in list(self.cache.values()):
            if e.handle is not None:
                self.backend.release(e.handle)
        self.cache.clear()

    # -- memory ----------------------------------------------------------------

    def _reserve(self, nbytes):
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        assert self.used <= self.budget, "admission exceeded the memory budget"

    def _evict_one(self) -> bool:
        idle = [(e.last_used, op) for op, e in self.cache.items() if not e.busy]
        if not idle:
            return False
        _, op = min(idle)
        e = self.cache.pop(op)
        self.backend.release(e.handle)
        self.used -= e.bytes
        self.stats["evictions"] += 1
        return True

    def _device_room(self) -> Optional[int]:
        """Bytes the device can still give to admissions: its free memory less
        the reservations of the requests in flight (whose allocations may not
        have happened yet) and a margin; None for a backend that does not
        report device memory."""
        free_fn = getattr(self.backend, "device_free_bytes", None)
        if free_fn is None:
            return None
        return int(free_fn()) - self.inflight - self.margin

    def _make_room(self, need, running) -> bool:
        """The reservation accounting leaves out what the device holds besides
        the hierarchies (allocator caches, freed pool blocks, runtime scratch).
        Checks the device's own free memory; if it is short, releases the
        backend's caches, then evicts idle hierarchies (least recently used
        first). False: wait for requests in flight to finish."""
        room = self._device_room()
        if room is None or need <= room:
            return True
        rel = getattr(self.backend, "release_cache", None)
        now = time.perf_counter()
        # at most twice a second while requests run (it may wait for the device)
        if rel is not None and (running == 0 or now - self._last_release >= 0.5):
            rel()
            self._last_release = now
        while True:
            room = self._device_room()
            if need <= room:
                return True
            if not self._evict_one():
                break
        self.stats["memory_waits"] += 1
        # nothing left to evict and nothing running: go ahead
        return running == 0

    def _evict_until(self, need) -> bool:
        idle = sorted((e.last_used, op) for op, e in self.cache.items() if not e.busy)
        for _, op in idle:
            if self.used + need <= self.budget:
                break
            e = self.cache.pop(op)
            self.backend.release(e.handle)
            self.used -= e.bytes
            self.stats["evictions"] += 1
        return self.used + need <= self.budget

    # -- main loop ---------------------------------------------------------------

    def run(self, requests: List[Request], realtime: bool = True, time_scale: float = 1.0,
            progress: int = 0):
        """Serves the stream; arrival times are replayed in real time (scaled).
        progress > 0 prints a line to stderr every `progress` completions."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        results: Dict[int, Result] = {}
        pending: List[list] = []  # [req, bypassed]
        retries: Dict[int, int] = {}  # req_id -> admissions repeated after running out of memory
        free = list(range(self.nslots))
        running = 0
        i = 0
        total = len(reqs)
        finished = 0
        t0 = time.perf_counter()
        clock = lambda: (time.perf_counter() - t0) / time_scale  # noqa: E731

        def admit():
            nonlocal running
            k = 0
            while k < len(pending) and free:
                req, bypassed = pending[k]
                entry = self.cache.get(req.op_id)
                if entry is not None and entry.busy:
                    k += 1
                    continue
                sb = self.backend.solve_bytes(req)
                need = sb if entry is not None else sb + self.backend.estimate_bytes(req)
                if need > self.budget:
                    pending.pop(k)
                    res = Result(req.req_id, req.op_id, req.N, req.t_arrival, rejected=True)
                    res.t_done = clock()
                    results[req.req_id] = res
                    self.stats["rejected"] += 1
                    continue
                if ((self.used + need > self.budget and not self._evict_until(need))
                        or not self._make_room(need, running)):
                    if k == 0 and bypassed >= self.max_bypass:
                        return  # the head has waited long enough: nobody passes it
                    k += 1
                    continue
                pending.pop(k)
                for j in range(k):  # everyone it passed was bypassed once more
                    pending[j][1] += 1
                slot = free.pop(0)
                build = entry is None
                if build:
                    entry = _Entry(None, need - sb, busy=True)
                    self.cache[req.op_id] = entry
                    self.stats["setups"] += 1
                else:
                    entry.busy = True
                    self.stats["hits"] += 1
                self._reserve(need)
                self.inflight += need
                res = Result(req.req_id, req.op_id, req.N, req.t_arrival, slot=slot,
                             cache_hit=not build)
                res.reserved = need
                res.retries = retries.get(req.req_id, 0)
                res.t_admit = clock()
                results[req.req_id] = res
                running += 1
                self.stats["max_concurrency"] = max(self.stats["max_concurrency"], running)
                self.events.append((res.t_admit, "admit", req.req_id, slot))
                self._inbox[slot].put((req, entry, build, time.perf_counter()))

        def complete(item):
            nonlocal running, finished
            slot, req, entry, built, out, err, _ = item
            res = results[req.req_id]
            res.t_done = clock()
            running -= 1
            oom = getattr(self.backend, "is_oom", None)
            if (err is not None and built is None and entry.handle is None and oom is not None
                    and oom(err) and res.retries < self.max_oom_retries):
                # the setup ran out of device memory: drop the placeholder,
                # free an idle hierarchy and queue the request again at the front
                free.append(slot)
                free.sort()
                self.used -= self.backend.solve_bytes(req)
                self.inflight -= res.reserved
                self.cache.pop(req.op_id, None)
                self.used -= entry.bytes
                self.stats["setups"] -= 1
                self.stats["oom_retries"] += 1
                self._evict_one()
                retries[req.req_id] = res.retries + 1
                del results[req.req_id]
                pending.insert(0, [req, 0])
                self.events.append((res.t_done, "retry", req.req_id, slot))
                return
            finished += 1
            if progress and finished % progress == 0:
                print("[serve] %d of %d requests done at %.1f s" % (finished, total, clock()),
                      file=sys.stderr, flush=True)
            free.append(slot)
            free.sort()
            self.used -= self.backend.solve_bytes(req)
            self.inflight -= res.reserved
            used_fn = getattr(self.backend, "device_used_bytes", None)
            if used_fn is not None:
                self.device_used_peak = max(self.device_used_peak, int(used_fn()))
            if built is not None:
                handle, nbytes = built
                entry.handle = handle
                self.used += nbytes - entry.bytes
                entry.bytes = nbytes
                self.peak_used = max(self.peak_used, self.used)
            entry.busy = False
            entry.last_used = res.t_done
            if err is not None or out is None:
                res.status = -1
                res.error = repr(err)[:200] if err is not None else "no result"
                if entry.handle is None:  # the build failed: drop the placeholder
                    self.cache.pop(req.op_id, None)
                    self.used -= entry.bytes
            else:
                res.status = out["status"]
                res.iterations = out["iterations"]
                res.converged = out["converged"]
                res.rel_res_true = out["rel_res_true"]
                res.x = out.get("x")
                if res.status != 0:
                    res.error = "status %d" % res.status
            self.events.append((res.t_done, "done", req.req_id, slot))

        while finished + self.stats["rejected"] < total:
            now = clock()
            while i < total and (not realtime or reqs[i].t_arrival <= now):
                pending.append([reqs[i], 0])
                i += 1
            while True:
                try:
                    complete(self._done.get_nowait())
                except queue.Empty:
                    break
            admit()
            if finished + self.stats["rejected"] >= total:
                break
            wait = None
            if i < total and realtime:
                wait = max(0.0, (reqs[i].t_arrival - clock()) * time_scale)
            if running == 0 and wait is None and i >= total and pending:
                raise RuntimeError("requests are pending with nothing running")
            try:
                complete(self._done.get(timeout=wait if wait is not None else 5.0))
            except queue.Empty:
                pass
        return [results[r.req_id] for r in reqs]


def summarize(results: List[Result], wall_s: Optional[float] = None, warmup: int = 0) -> dict:
    done = [r for r in results[warmup:] if not r.rejected and r.status in (0,)]
    lat = np.array([r.latency for r in done]) * 1e3 if done else np.zeros(1)
    if wall_s is None and done:
        wall_s = max(r.t_done for r in done) - min(r.t_arrival for r in done)
    return {
        "completed": len(done),
        "rejected": sum(1 for r in results if r.rejected),
        "failed": sum(1 for r in results if not r.rejected and r.status not in (0,)),
        "p50_latency_ms": float(np.percentile(lat, 50)),
        "p99_latency_ms": float(np.percentile(lat, 99)),
        "mean_latency_ms": float(lat.mean()),
        "solves_per_s": (len(done) / wall_s) if wall_s else 0.0,
        "cache_hit_rate": (sum(r.cache_hit for r in done) / len(done)) if done else 0.0,
        "all_converged": all(r.converged for r in done),
        "errors": _count([r.error for r in results if r.error]),
    }


def _count(items) -> dict:
    out: Dict[str, int] = {}
    for it in items:
        out[it] = out.get(it, 0) + 1
    return out


class GpuBackend:
    """Runs requests through the HIP library (include/amg.h) on one GPU."""

    def __init__(self, precision=None, rtol=1e-8, maxit=500, keep_x=False, device=0):
        import torch

        from . import amg

        self.torch = torch
        self.amg = amg
        self.dev = torch.device("cuda", device)
        self.precision = amg.FP32 if precision is None else precision
        self.rtol = rtol
        self.maxit = maxit
        self.keep_x = keep_x
        amg.load_library()

    # Device memory the admission budget leaves alone: the library pool's
    # reserve of freed blocks (up to 8 GiB), the torch allocator's cached
    # request arrays, the runtime's per-dispatch scratch (private segments)
    # and pool fragmentation. With 12 GiB left, a 2000-request stream filled
    # the device and a dispatch failed to get its scratch.
    HEADROOM = 32 << 30

    def default_budget(self) -> int:
        _, total = self.torch.cuda.mem_get_info(self.dev)
        return max(0, int(total) - self.HEADROOM)

    def device_free_bytes(self) -> int:
        return int(self.torch.cuda.mem_get_info(self.dev)[0])

    def device_used_bytes(self) -> int:
        free, total = self.torch.cuda.mem_get_info(self.dev)
        return int(total - free)

    def is_oom(self, err) -> bool:
        amg = self.amg
        return ((isinstance(err, amg.AmgError) and err.status == amg.Status.ERR_OOM)
                or isinstance(err, self.torch.cuda.OutOfMemoryError))

    def release_cache(self):
        # blocks the torch allocator keeps from earlier requests' operator
        # builds and vectors
        self.torch.cuda.empty_cache()

    def make_slot(self, i):
        torch = self.torch
        torch.cuda.set_device(self.dev)
        return {"stream": torch.cuda.Stream(device=self.dev), "index": i}

    def _params(self):
        return self.amg.amg_params_default(precision=self.precision)

    def estimate_bytes(self, req) -> int:
        n = req.N ** 3
        nnz = 7 * n - 6 * req.N * req.N
        csr = 4 * (n + 1) + 12 * nnz  # the operator while the setup copies it
        build = 400 * n  # torch temporaries of the operator build (stacked columns, masks)
        return self.amg.amg_estimate_footprint(n, nnz, self._params()) + csr + build

    def solve_bytes(self, req) -> int:
        return 2 * 8 * req.N ** 3

    def build(self, req, slot):
        from . import inputs

        torch = self.torch
        torch.cuda.set_device(self.dev)
        with torch.cuda.stream(slot["stream"]):
            kx, ky = req.eps
            rp, ci, va = inputs.constant_diffusion7_arrays(req.N, kx, ky, 1.0, torch,
                                                           device=self.dev)
            h = self.amg.amg_setup(rp, ci, va, precision=self.precision,
                                   stream=slot["stream"].cuda_stream)
            del rp, ci, va
        return h, h.footprint_bytes()

    def solve(self, handle, req, slot):
        torch = self.torch
        torch.cuda.set_device(self.dev)
        s = slot["stream"]
        with torch.cuda.stream(s):
            n = req.N ** 3
            g = torch.Generator(device=self.dev)
            g.manual_seed(int(req.rhs_seed))
            b = torch.rand(n, generator=g, device=self.dev, dtype=torch.float64) * 2.0 - 1.0
            x = torch.zeros_like(b)
            handle.set_stream(s)
            st, info = self.amg.amg_pcg_solve(handle, b, x, rtol=self.rtol, maxit=self.maxit,
                                              raise_on_error=False)
            out = dict(info)
            out["status"] = st
            if self.keep_x:
                out["x"] = x.cpu().numpy()
        return out

    def release(self, handle):
        handle.close()


def main(argv=None):
    import argparse
    import json

    from . import inputs

    ap = argparse.ArgumentParser(description="serve a synthetic AMG-PCG request stream")
    ap.add_argument("--rates", default="10,50,200,500")
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=None,
                    help="GiB the server may reserve (default: device memory less 32 GiB)")
    ap.add_argument("--seed", type=int, default=4)
    args = ap.parse_args(argv)
    backend = GpuBackend()
    rows = []
    for rate in [float(r) for r in args.rates.split(",")]:
        reqs = requests_from_stream(inputs.serving_requests(args.count, rate, seed=args.seed))
        budget = (int(args.budget_gb * (1 << 30)) if args.budget_gb is not None
                  else backend.default_budget())
        srv = Server(backend, slots=args.slots, budget_bytes=budget)
        t0 = time.perf_counter()
        res = srv.run(reqs, progress=250)
        wall = time.perf_counter() - t0
        summ = summarize(res, warmup=args.warmup)
        summ.update({"rate_per_s": rate, "wall_s": wall, "setups": srv.stats["setups"],
                     "evictions": srv.stats["evictions"],
                     "max_concurrency": srv.stats["max_concurrency"],
                     "memory_waits": srv.stats["memory_waits"],
                     "oom_retries": srv.stats["oom_retries"],
                     "budget_gib": budget / (1 << 30),
                     "peak_reserved_gib": srv.peak_used / (1 << 30),
                     "device_used_peak_gib": srv.device_used_peak / (1 << 30)})
        srv.close()
        rows.append(summ)
        print(json.dumps(summ), flush=True)
    return rows


if __name__ == "__main__":
    main()
