"""Serving scheduler on the CPU with fake backends: admission by footprint,
hierarchy caching and eviction, continuous batching across slots, rejection,
bounded bypass, and results that do not depend on the request mix."""

import threading
import time

import numpy as np
import pytest

from paper_2006_16147_amd import inputs
from paper_2006_16147_amd.serve import Request, Server, requests_from_stream, summarize


class SleepBackend:
    """Sleeps for the setup and the solve; declares footprints per dof."""

    def __init__(self, setup_s=0.02, solve_s=0.01, bytes_per_dof=100):
        self.setup_s = setup_s
        self.solve_s = solve_s
        self.bpd = bytes_per_dof
        self.lock = threading.Lock()
        self.active = {}  # op_id -> number of threads using it
        self.overlap_same_op = False
        self.builds = []
        self.released = []

    def make_slot(self, i):
        return {"i": i}

    def estimate_bytes(self, req):
        return self.bpd * req.N ** 3

    def solve_bytes(self, req):
        return 16 * req.N ** 3

    def _enter(self, op):
        with self.lock:
            self.active[op] = self.active.get(op, 0) + 1
            if self.active[op] > 1:
                self.overlap_same_op = True

    def _leave(self, op):
        with self.lock:
            self.active[op] -= 1

    def build(self, req, slot):
        self._enter(req.op_id)
        time.sleep(self.setup_s)
        self._leave(req.op_id)
        with self.lock:
            self.builds.append(req.op_id)
        return ("H", req.op_id), int(0.9 * self.estimate_bytes(req))

    def solve(self, handle, req, slot):
        self._enter(req.op_id)
        time.sleep(self.solve_s)
        self._leave(req.op_id)
        return {"status": 0, "iterations": 10, "converged": True, "rel_res_true": 1e-9,
                "x": np.full(3, float(req.rhs_seed))}

    def release(self, handle):
        self.released.append(handle)


def _burst(n, ops, N=10, dt=0.0):
    return [Request(i, i * dt, ops[i % len(ops)], N, (1.0, 1.0), 1000 + i) for i in range(n)]


def test_all_complete_and_latency_accounting():
    be = SleepBackend()
    srv = Server(be, slots=3, budget_bytes=10 ** 9)
    reqs = _burst(12, ops=list(range(12)), dt=0.002)
    res = srv.run(reqs)
    srv.close()
    assert len(res) == 12 and all(r.status == 0 and not r.rejected for r in res)
    for r in res:
        assert r.t_admit >= r.t_arrival - 1e-3
        assert r.t_done >= r.t_admit
        assert r.latency >= be.setup_s + be.solve_s - 1e-3
    s = summarize(res)
    assert s["completed"] == 12 and s["p99_latency_ms"] >= s["p50_latency_ms"] > 0


def test_continuous_batching_overlaps_slots():
    """Requests arriving while others run are admitted to free slots at once."""
    be = SleepBackend(setup_s=0.05, solve_s=0.02)
    srv = Server(be, slots=4, budget_bytes=10 ** 9)
    reqs = _burst(8, ops=list(range(8)), dt=0.005)
    srv.run(reqs)
    srv.close()
    assert srv.stats["max_concurrency"] == 4
    # request 1 (arriving 5 ms after request 0) is admitted before 0 finishes
    t = {(kind, rid): tt for tt, kind, rid, _ in srv.events}
    assert t[("admit", 1)] < t[("done", 0)]
    # a later request is admitted as soon as a slot frees (no batch barrier)
    assert t[("admit", 4)] < max(t[("done", j)] for j in range(4))


def test_cache_hits_and_no_concurrent_use_of_one_hierarchy():
    be = SleepBackend(setup_s=0.03, solve_s=0.02)
    srv = Server(be, slots=4, budget_bytes=10 ** 9)
    reqs = _burst(10, ops=[7, 8], dt=0.001)
    res = srv.run(reqs)
    srv.close()
    assert sorted(be.builds) == [7, 8]  # each operator built once
    assert srv.stats["hits"] == 8 and sum(r.cache_hit for r in res) == 8
    assert not be.overlap_same_op


def test_admission_by_footprint_and_lru_eviction():
    be = SleepBackend(bytes_per_dof=100)
    one = 100 * 10 ** 3 + 16 * 10 ** 3  # one N=10 hierarchy plus its vectors
    srv = Server(be, slots=4, budget_bytes=int(1.5 * one))
    reqs = _burst(6, ops=[0, 1, 2, 0, 1, 2], dt=0.0)
    res = srv.run(reqs)
    srv.close()
    assert all(r.status == 0 for r in res)
    assert srv.peak_used <= srv.budget
    assert srv.stats["max_concurrency"] == 1  # only one miss fits at a time
    assert srv.stats["evictions"] >= 2 and len(be.released) >= 2


class DeviceBackend(SleepBackend):
    """SleepBackend on a simulated device of `total` bytes: hierarchies hold
    their footprint, and every build leaves `cache_per_build` bytes in an
    allocator cache that only release_cache() gives back (memory that the
    reservations do not see)."""

    def __init__(self, total, cache_per_build, **kw):
        super().__init__(**kw)
        self.total = total
        self.cache_per_build = cache_per_build
        self.cache = 0
        self.live = {}
        self.peak = 0
        self.cache_releases = 0

    def _used(self):
        return sum(self.live.values()) + self.cache

    def device_free_bytes(self):
        with self.lock:
            return self.total - self._used()

    def device_used_bytes(self):
        with self.lock:
            return self._used()

    def release_cache(self):
        with self.lock:
            self.cache = 0
            self.cache_releases += 1

    def build(self, req, slot):
        h, nbytes = super().build(req, slot)
        with self.lock:
            self.live[h] = nbytes
            self.cache += self.cache_per_build
            self.peak = max(self.peak, self._used())
        return h, nbytes

    def release(self, handle):
        super().release(handle)
        with self.lock:
            self.live.pop(handle, None)


def test_device_check_covers_memory_the_reservations_do_not_see():
    """The budget alone would admit everything; the device's own free memory
    (hierarchies plus a growing allocator cache) forces cache releases and
    LRU evictions, and the simulated device never overflows."""
    one = 100 * 10 ** 3  # one N=10 hierarchy's estimate
    # a build holds 0.9 of its estimate plus the cache growth: within the
    # request's reservation, as the margin assumes for the real backend
    be = DeviceBackend(total=4 * one, cache_per_build=one // 8, setup_s=0.002,
                       solve_s=0.002, bytes_per_dof=100)
    srv = Server(be, slots=2, budget_bytes=10 ** 12, margin_bytes=one // 4)
    reqs = _burst(40, ops=list(range(12)), dt=0.0005)
    res = srv.run(reqs)
    srv.close()
    assert all(r.status == 0 for r in res)
    assert be.peak <= be.total
    assert be.cache_releases > 0 and srv.stats["evictions"] > 0
    assert srv.device_used_peak <= be.total


class OomOnceBackend(SleepBackend):
    """The first setup of operator 3 runs out of device memory."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.failed_once = False

    def is_oom(self, err):
        return isinstance(err, MemoryError)

    def build(self, req, slot):
        if req.op_id == 3 and not self.failed_once:
            self.failed_once = True
            raise MemoryError("device full")
        return super().build(req, slot)


def test_setup_out_of_memory_is_retried_after_an_eviction():
    be = OomOnceBackend(setup_s=0.002, solve_s=0.002)
    srv = Server(be, slots=2, budget_bytes=10 ** 9)
    reqs = _burst(8, ops=[0, 1, 2, 3], dt=0.001)
    res = srv.run(reqs)
    srv.close()
    assert all(r.status == 0 for r in res)
    assert srv.stats["oom_retries"] == 1 and srv.stats["evictions"] >= 1
    assert [r.retries for r in res if r.req_id == 3] == [1]
    assert summarize(res)["errors"] == {}
    # the eviction made room by dropping an idle hierarchy, which is built again later
    assert be.builds.count(3) == 1 and srv.stats["setups"] == len(be.builds)


def test_rejection_of_requests_larger_than_the_device():
    be = SleepBackend(bytes_per_dof=100)
    srv = Server(be, slots=2, budget_bytes=50_000)
    reqs = [Request(0, 0.0, 0, 10), Request(1, 0.0, 1, 4), Request(2, 0.0, 2, 5)]
    res = srv.run(reqs)
    srv.close()
    assert res[0].rejected and not res[1].rejected and not res[2].rejected
    assert summarize(res)["rejected"] == 1


def test_bypass_is_bounded():
    """A large request waiting for memory is passed by small ones at most
    max_bypass times, then admitted once memory frees."""
    be = SleepBackend(setup_s=0.01, solve_s=0.03, bytes_per_dof=100)
    budget = 100 * 20 ** 3 + 16 * 20 ** 3 + 1000
    srv = Server(be, slots=4, budget_bytes=budget, max_bypass=2)
    reqs = [Request(0, 0.0, 0, 12)]  # occupies memory first
    reqs.append(Request(1, 0.001, 1, 20))  # needs nearly the whole budget
    reqs += [Request(2 + i, 0.002 + 0.001 * i, 2 + i, 4) for i in range(8)]
    res = srv.run(reqs)
    srv.close()
    order = [rid for _, kind, rid, _ in srv.events if kind == "admit"]
    passed = [rid for rid in order[: order.index(1)] if rid >= 2]
    assert len(passed) <= 2
    assert all(r.status == 0 for r in res)


class OracleBackend:
    """Solves with the CPU oracle: results must not depend on the mix."""

    def __init__(self):
        import oracle

        self.oracle = oracle

    def make_slot(self, i):
        return {}

    def estimate_bytes(self, req):
        return 10 ** 6

    def solve_bytes(self, req):
        return 16 * req.N ** 3

    def build(self, req, slot):
        rp, ci, va = inputs.constant_diffusion7_arrays(req.N, req.eps[0], req.eps[1], 1.0, np)
        h = self.oracle.Hierarchy(inputs.Csr(req.N ** 3, rp, ci, va), max_coarse=20)
        return h, 10 ** 6

    def solve(self, handle, req, slot):
        b = np.random.default_rng(req.rhs_seed).uniform(-1, 1, req.N ** 3)
        x, info = handle.pcg(b, rtol=1e-8)
        return {"status": info["status"], "iterations": info["iterations"],
                "converged": info["converged"], "rel_res_true": info["rel_res_true"], "x": x}

    def release(self, handle):
        pass


def test_results_same_alone_and_in_mix(orc):
    stream = inputs.serving_requests(10, rate=400.0, seed=4, sizes=(6, 8, 10))
    reqs = requests_from_stream(stream)
    mix_srv = Server(OracleBackend(), slots=3, budget_bytes=10 ** 9)
    mix = mix_srv.run(reqs)
    mix_srv.close()
    for r, req in zip(mix, reqs):
        alone_srv = Server(OracleBackend(), slots=1, budget_bytes=10 ** 9)
        (a,) = alone_srv.run([Request(0, 0.0, req.op_id, req.N, req.eps, req.rhs_seed)])
        alone_srv.close()
        assert r.converged and a.converged
        assert r.iterations == a.iterations
        np.testing.assert_array_equal(r.x, a.x)


def test_request_stream_generator():
    s = inputs.serving_requests(300, rate=100.0, seed=4)
    t = np.array([r["t_arrival"] for r in s])
    assert np.all(np.diff(t) > 0)
    assert 2.0 < t[-1] < 4.5  # 300 arrivals at 100/s
    ops = {}
    for r in s:
        ops.setdefault(r["op_id"], (r["N"], r["eps"]))
        assert ops[r["op_id"]] == (r["N"], r["eps"])  # a reused op keeps its operator
        assert r["N"] in (32, 48, 64, 96, 128, 192)
    reuse = sum(1 for i, r in enumerate(s) if r["op_id"] < max(x["op_id"] for x in s[:i + 1]))
    assert 0.3 < reuse / len(s) < 0.7
    aniso = [o for o in ops.values() if o[1] != (1.0, 1.0)]
    assert 0.3 < len(aniso) / len(ops) < 0.7
    assert all(1e-3 <= e <= 1.0 for o in aniso for e in o[1])


@pytest.mark.parametrize("rate", [50.0])
def test_summary_fields(rate):
    be = SleepBackend(setup_s=0.002, solve_s=0.001)
    srv = Server(be, slots=2, budget_bytes=10 ** 9)
    res = srv.run(_burst(20, ops=[0, 1, 2], dt=1.0 / rate))
    srv.close()
    s = summarize(res, warmup=2)
    for key in ("p50_latency_ms", "p99_latency_ms", "solves_per_s", "cache_hit_rate"):
        assert key in s
    assert s["completed"] == 18 and s["cache_hit_rate"] > 0.5
