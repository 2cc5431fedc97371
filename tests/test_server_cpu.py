"""Serving scheduler on a virtual clock (fake backend, no GPU)."""
import numpy as np
import pytest

from paper_2605_17855_amd import scenes, server


def make_requests(times, n_scenes=2, size=(64, 64)):
    return [scenes.Request(i, i % n_scenes, size[0], size[1], np.array([4.0, 0.0, 0.0]), float(t))
            for i, t in enumerate(times)]


def run(times, pool, slots=4, keys=lambda j: 1000, est=None, prep=1e-3, rast=2e-3, scene_n=(1000, 2000), **kw):
    # reservations are placed in an arena of the pool's size, as on the device
    be = server.FakeBackend(scene_n, keys, est, prepare_s=lambda j: prep, raster_s=lambda js: rast,
                            arena_bytes=pool)
    srv = server.Server(be, pool, slots=slots, **kw)
    st = srv.run(make_requests(times, len(scene_n)))
    return st, be


def test_every_request_completes_and_pool_bound_holds():
    pool = server.job_bytes(2000, 1000, 64 * 64) * 3 + 10
    st, be = run(np.linspace(0, 0.01, 50), pool, slots=8)
    assert st.completed == 50 and st.failed == 0
    assert st.max_reserved_bytes <= pool
    assert st.max_reserved_bytes > pool // 2


def test_fifo_admission_order():
    pool = server.job_bytes(2000, 1000, 64 * 64) * 2
    st, be = run(np.linspace(0, 0.005, 30), pool, slots=4)
    admitted = [r[2] for r in be.log if r[0] == "prepare"]
    assert admitted == sorted(admitted)


def test_latency_percentiles_exact_for_idle_server():
    # arrivals far apart, one job at a time: latency = prepare + raster exactly
    st, be = run(np.arange(20) * 0.1, pool=10**9, slots=1, prep=1e-3, rast=2e-3)
    assert st.latency_p50_ms == pytest.approx(3.0, abs=1e-9)
    assert st.latency_p99_ms == pytest.approx(3.0, abs=1e-9)
    assert st.batches == 20 and st.mean_batch == 1.0


def test_retry_after_capacity_with_exact_size():
    # the estimate is low for odd requests; they come back once with the exact size
    keys = lambda j: 5000 if j.rid % 2 else 1000
    est = lambda j: 1000
    st, be = run(np.linspace(0, 0.01, 20), pool=10**9, slots=4, keys=keys, est=est)
    assert st.completed == 20
    assert st.retries == 10
    reserves = {}
    for r in be.log:
        if r[0] == "prepare":
            reserves.setdefault(r[2], []).append(r[3])
    for rid, rs in reserves.items():
        if rid % 2:
            assert len(rs) == 2 and rs[1] > rs[0]
        else:
            assert len(rs) == 1


def test_arrivals_while_busy_wait_for_memory():
    one = server.job_bytes(2000, 1000, 64 * 64)
    st, be = run(np.zeros(12), pool=2 * one, slots=16, prep=1e-3, rast=1e-3)
    assert st.completed == 12
    assert st.max_reserved_bytes <= 2 * one
    # with two reservations at a time, prepares happen in pairs
    times = sorted(r[1] for r in be.log if r[0] == "prepare")
    assert len(set(np.round(times, 9))) >= 6


def test_request_larger_than_pool_fails_without_blocking_others():
    keys = lambda j: 10**8 if j.rid == 3 else 1000
    pool = server.job_bytes(2000, 1000, 64 * 64) * 4
    st, be = run(np.linspace(0, 0.01, 10), pool=pool, slots=4, keys=keys, est=keys)
    assert st.completed == 9 and st.failed == 1


def test_continuous_batching_under_load():
    # arrivals faster than the raster: ready requests share launches
    st, be = run(np.linspace(0, 0.02, 200), pool=10**9, slots=16, prep=1e-3, rast=2e-3)
    assert st.completed == 200
    assert st.mean_batch > 2.0
    assert st.max_inflight_jobs > 4
    # every batch launched at most max_batch jobs
    assert max(len(r[2]) for r in be.log if r[0] == "raster") <= 32


def test_open_loop_latency_includes_queueing():
    # a burst of 10 at t=0 with one slot: the k-th request waits for k-1 others
    st, be = run(np.zeros(10), pool=10**9, slots=1, prep=1e-3, rast=1e-3)
    assert st.latency_p99_ms > 15.0
    assert st.completed == 10


def test_arena_first_fit_and_merge():
    a = server._Arena(1024, align=16)
    x = a.alloc(100)
    y = a.alloc(200)
    z = a.alloc(300)
    assert (x, y, z) == (0, 112, 320)
    assert a.alloc(500) is None          # 624 bytes used, 400 left at the end
    a.release(y, 200)
    assert a.alloc(50) == 112            # first fit reuses the hole
    a.release(112, 50)
    a.release(x, 100)
    a.release(z, 300)
    assert a.alloc(1024) == 0            # holes merged back into one block
    assert a.alloc(1) is None


def test_request_generator_is_open_loop_poisson():
    reqs = scenes.serving_requests(2000, rate_hz=1000.0, n_scenes=8, seed=49)
    t = np.array([r.arrival for r in reqs])
    gaps = np.diff(t)
    assert t[0] == 0.0 and np.all(gaps >= 0)
    assert np.mean(gaps) == pytest.approx(1e-3, rel=0.1)
    assert set(r.scene for r in reqs) == set(range(8))
    assert set((r.width, r.height) for r in reqs) == set(scenes.SERVE_RESOLUTIONS)


def test_estimate_above_pool_is_tried_not_rejected():
    # the estimate overshoots the pool; the exact size fits, so the request must complete
    pool = server.job_bytes(2000, 1000, 64 * 64) * 2
    st, be = run(np.linspace(0, 0.01, 6), pool=pool, slots=4, keys=lambda j: 1000, est=lambda j: 10**8)
    assert st.completed == 6 and st.failed == 0
    # each request reserves the whole pool, which holds its entries: one at a time, no retries
    assert st.retries == 0 and st.max_inflight_jobs == 1
    assert st.max_reserved_bytes == pool


def test_unaligned_pool_with_oversized_estimates_terminates():
    # a pool that is not a multiple of the arena alignment, estimates above it and exact sizes
    # above it too: every request is tried once at the pool's size, then rejected
    pool = server.job_bytes(2000, 0, 320 * 180) + 4096 + 7
    st, be = run(np.linspace(0, 0.01, 6), pool=pool, slots=4, keys=lambda j: 10**6, est=lambda j: 10**6)
    assert st.completed == 0 and st.failed == 6
    assert st.retries == 6


def test_reservation_refused_in_empty_pool_fails_the_request():
    class Refusing(server.FakeBackend):
        def try_reserve(self, job, need):
            return job.rid != 2 and super().try_reserve(job, need)
    be = Refusing((1000, 2000), lambda j: 1000, prepare_s=lambda j: 1e-3, raster_s=lambda js: 1e-3)
    st = server.Server(be, 10**9, slots=1).run(make_requests(np.linspace(0, 0.01, 5)))
    assert st.completed == 4 and st.failed == 1


def test_reservation_covers_the_library_workspace():
    # the serving reservation of a request must hold its bins and the workspace that
    # gs_workspace_bytes asks for, at the capacity the reservation implies
    import ctypes as C
    from paper_2605_17855_amd import gs
    L = gs.lib()
    for n in [1, 1000, 500_000, 1_048_576, 1_200_000, 3_000_000, 6_000_000]:
        for (w, h) in [(16, 16), (640, 360), (1920, 1080), (3840, 2160)]:
            for k in [0, 1000, 1_048_576, 1_100_000, 20_000_000]:
                for g in (1, 2, 4):
                    reserve = server.job_bytes(n, k, w * h)
                    cap = server.entry_capacity(reserve, n, w * h)
                    assert cap >= k
                    ws = int(L.gs_workspace_bytes(n, cap, C.byref(gs.camera_stub(w, h)), C.byref(gs.options(group=g))))
                    nb = int(L.gs_num_bins(C.byref(gs.camera_stub(w, h)), g))
                    parts = [8 * max(cap, 1), 4 * max(cap, 1), 2 * max(cap, 1) + 2, 8 * nb, ws]
                    assert sum((x + 255) // 256 * 256 for x in parts) <= reserve, (n, w, h, k, g)
