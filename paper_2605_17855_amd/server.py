"""Continuous-batching render server: admission by duplicated-key memory, batched raster.

Requests (scene, resolution, pose, scheduled arrival) enter a FIFO.  A request is
admitted when a slot is free and its estimated memory (duplicated entries plus
per-Gaussian scratch) fits the pool next to every reservation already held.  An
admitted request runs preprocess + bin sort on its own stream; when its entries
are ready it joins the next batched raster launch, which renders every ready
request in one persistent kernel while other requests keep preparing on their
streams.  A request whose entry count exceeds its reservation gives the memory
back and re-enters the queue head with its exact size.  Latency is completion
time minus scheduled arrival (open loop).

The scheduler only talks to a backend: `GpuBackend` drives the HIP library;
`FakeBackend` simulates durations on a virtual clock for CPU tests.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import math
import threading
import time
from typing import Dict, List, Optional

import numpy as np

# bytes per duplicated entry: key 8 + value 4 + mask 2, plus the workspace's bin key and
# the two sort double buffers (4 + 4 + 4) and the sort's per-tile digit counts
BYTES_PER_ENTRY = 27
# per-Gaussian workspace bytes: scan partials, depth keys and their double buffers, and
# each visible Gaussian's first-entry offset
BYTES_PER_GAUSSIAN = 24


@dataclasses.dataclass
class Job:
    rid: int
    scene: int
    width: int
    height: int
    position: np.ndarray
    arrival: float
    reserve: int = 0
    reserve_hint: int = 0
    slot: int = -1
    n_keys: int = -1
    retries: int = 0
    t_admit: float = math.nan
    t_ready: float = math.nan
    t_done: float = math.nan
    failed: str = ""
    payload: object = None   # backend-owned (buffers, events)


@dataclasses.dataclass
class Stats:
    completed: int
    failed: int
    retries: int
    wall_s: float
    frames_per_s: float
    latency_p50_ms: float
    latency_p99_ms: float
    latency_mean_ms: float
    max_reserved_bytes: int
    pool_bytes: int
    batches: int
    mean_batch: float
    max_inflight_jobs: int

    def as_dict(self):
        return dataclasses.asdict(self)


class Server:
    def __init__(self, backend, pool_bytes: int, slots: int = 16, max_batch: int = 32,
                 max_inflight_batches: int = 2):
        self.backend = backend
        self.pool = int(pool_bytes)
        self.slots = slots
        self.max_batch = max_batch
        self.max_inflight = max_inflight_batches

    def run(self, requests) -> Stats:
        be = self.backend
        reqs = sorted(requests, key=lambda r: r.arrival)
        jobs = [Job(r.rid, r.scene, r.width, r.height, np.asarray(r.position), r.arrival) for r in reqs]
        pending: collections.deque = collections.deque()
        ready: List[Job] = []
        inflight: Dict[object, List[Job]] = {}
        free_slots = list(range(self.slots))[::-1]
        reserved = 0
        max_reserved = 0
        nxt = 0
        done = 0
        batches = 0
        batch_sizes = 0
        max_inflight_jobs = 0
        preparing = 0
        t_start = be.now()
        while done < len(jobs):
            progressed = False
            now = be.now()
            while nxt < len(jobs) and jobs[nxt].arrival <= now - t_start:
                pending.append(jobs[nxt])
                nxt += 1
                progressed = True
            # admission: FIFO, a slot and pool room for the head of the queue
            while pending and free_slots:
                job = pending[0]
                # an estimate above the pool is tried at the pool's size; only an exact size
                # (known after a first attempt) can reject the request
                need = job.reserve_hint or min(be.estimate_bytes(job), self.pool)
                if need > self.pool:
                    pending.popleft()
                    job.failed = f"needs {need} bytes, pool is {self.pool}"
                    job.t_done = now - t_start
                    done += 1
                    progressed = True
                    continue
                if reserved + need > self.pool or not be.try_reserve(job, need):
                    if reserved == 0:
                        # nothing is held, so nothing will be released: the request can never
                        # be placed (the backend refused a reservation within the pool)
                        pending.popleft()
                        job.failed = f"backend could not reserve {need} bytes in an empty pool"
                        job.t_done = now - t_start
                        done += 1
                        progressed = True
                        continue
                    break
                pending.popleft()
                job.slot = free_slots.pop()
                job.reserve = need
                reserved += need
                max_reserved = max(max_reserved, reserved)
                job.t_admit = now - t_start
                be.start_prepare(job)
                preparing += 1
                progressed = True
            for job, n_keys, ok in be.poll_prepared():
                preparing -= 1
                progressed = True
                job.n_keys = n_keys
                if ok:
                    job.t_ready = be.now() - t_start
                    ready.append(job)
                else:
                    # entry count above the reservation: give it back, retry at the head
                    reserved -= job.reserve
                    free_slots.append(job.slot)
                    job.slot = -1
                    job.reserve = 0
                    job.reserve_hint = be.exact_bytes(job, n_keys)
                    job.retries += 1
                    pending.appendleft(job)
            while ready and len(inflight) < self.max_inflight:
                batch = ready[: self.max_batch]
                ready = ready[self.max_batch:]
                handle = be.start_raster(batch)
                inflight[handle] = batch
                batches += 1
                batch_sizes += len(batch)
                progressed = True
            max_inflight_jobs = max(max_inflight_jobs, sum(len(b) for b in inflight.values()) + preparing)
            for handle in be.poll_rasters():
                progressed = True
                t = be.now() - t_start
                for job in inflight.pop(handle):
                    job.t_done = t
                    reserved -= job.reserve
                    free_slots.append(job.slot)
                    be.release(job)
                    done += 1
            if not progressed:
                busy = bool(inflight) or preparing > 0
                next_arrival = jobs[nxt].arrival + t_start if nxt < len(jobs) else None
                be.wait(None if busy else next_arrival)
        wall = be.now() - t_start
        ok = [j for j in jobs if not j.failed]
        lat = np.array([j.t_done - j.arrival for j in ok]) * 1e3 if ok else np.zeros(1)
        first = min(j.arrival for j in jobs) if jobs else 0.0
        last = max(j.t_done for j in ok) if ok else 0.0
        span = max(last - first, 1e-9)
        return Stats(completed=len(ok), failed=len(jobs) - len(ok), retries=sum(j.retries for j in jobs),
                     wall_s=wall, frames_per_s=len(ok) / span,
                     latency_p50_ms=float(np.percentile(lat, 50)), latency_p99_ms=float(np.percentile(lat, 99)),
                     latency_mean_ms=float(lat.mean()), max_reserved_bytes=int(max_reserved), pool_bytes=self.pool,
                     batches=batches, mean_batch=batch_sizes / max(batches, 1),
                     max_inflight_jobs=max_inflight_jobs)


# ---------------------------------------------------------------------------------------
# Backends
# ---------------------------------------------------------------------------------------

# fixed bytes per request: bin ranges (8 B per 16x16 tile) come on top of this slack for
# alignment padding
FIXED_BYTES = 1 << 18


def job_bytes(n_gaussians: int, n_entries: int, pixels: int) -> int:
    return BYTES_PER_ENTRY * int(n_entries) + BYTES_PER_GAUSSIAN * int(n_gaussians) + int(pixels) // 32 + FIXED_BYTES


def entry_capacity(reserve: int, n_gaussians: int, pixels: int) -> int:
    """Entries a reservation of `reserve` bytes holds (inverse of job_bytes)."""
    return max(0, (int(reserve) - BYTES_PER_GAUSSIAN * int(n_gaussians) - int(pixels) // 32 - FIXED_BYTES)
               // BYTES_PER_ENTRY)


class FakeBackend:
    """Virtual-clock backend: scripted entry counts and durations (no GPU)."""

    def __init__(self, scene_sizes, keys_fn, est_fn=None, prepare_s=lambda j: 1e-3, raster_s=lambda js: 2e-3,
                 arena_bytes: Optional[int] = None):
        self.scene_sizes = list(scene_sizes)
        self.arena = _Arena(arena_bytes) if arena_bytes is not None else None   # as the GPU backend places them
        self.keys_fn = keys_fn            # job -> true entry count
        self.est_fn = est_fn or keys_fn   # job -> estimated entry count
        self.prepare_s = prepare_s
        self.raster_s = raster_s
        self.t = 0.0
        self.events = []                  # (time, kind, payload)
        self.seq = 0
        self.log = []

    def now(self):
        return self.t

    def estimate_bytes(self, job):
        return job_bytes(self.scene_sizes[job.scene], self.est_fn(job), job.width * job.height)

    def exact_bytes(self, job, n_keys):
        return job_bytes(self.scene_sizes[job.scene], n_keys, job.width * job.height)

    def try_reserve(self, job, need):
        if self.arena is None:
            return True
        off = self.arena.alloc(need)
        if off is None:
            return False
        job.payload = off
        return True

    def _push(self, dt, kind, payload):
        self.seq += 1
        self.events.append((self.t + dt, self.seq, kind, payload))
        self.events.sort(key=lambda e: (e[0], e[1]))

    def start_prepare(self, job):
        self.log.append(("prepare", self.t, job.rid, job.reserve))
        self._push(self.prepare_s(job), "prepared", job)

    def _due(self, kind):
        out = [e for e in self.events if e[2] == kind and e[0] <= self.t]
        self.events = [e for e in self.events if not (e[2] == kind and e[0] <= self.t)]
        return out

    def poll_prepared(self):
        res = []
        for _, _, _, job in self._due("prepared"):
            k = self.keys_fn(job)
            cap = entry_capacity(job.reserve, self.scene_sizes[job.scene], job.width * job.height)
            if k > cap:
                self.release(job)
            res.append((job, k, k <= cap))
        return res

    def start_raster(self, jobs):
        self.seq += 1
        handle = ("batch", self.seq)
        self.log.append(("raster", self.t, [j.rid for j in jobs]))
        self._push(self.raster_s(jobs), "raster", handle)
        return handle

    def poll_rasters(self):
        return [h for _, _, _, h in self._due("raster")]

    def release(self, job):
        if self.arena is not None and job.payload is not None:
            self.arena.release(job.payload, job.reserve)
            job.payload = None

    def wait(self, until):
        nxt = self.events[0][0] if self.events else None
        cands = [x for x in (nxt, until) if x is not None]
        if cands:
            self.t = max(self.t, min(cands))


class _Arena:
    """First-fit allocator of byte ranges inside one device buffer (the memory pool)."""

    def __init__(self, nbytes: int, align: int = 256):
        # sized to the pool rounded up to the alignment, so that any single reservation
        # of at most `nbytes` fits an empty arena
        self.align = align
        self.size = (int(nbytes) + align - 1) // align * align
        self.free = [(0, self.size)]

    def alloc(self, size: int) -> Optional[int]:
        size = (size + self.align - 1) // self.align * self.align
        for i, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + size, sz - size)
                return off
        return None

    def release(self, off: int, size: int):
        size = (size + self.align - 1) // self.align * self.align
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


class GpuBackend:
    """Drives the HIP library: per-slot streams for preprocess + sort, one stream for batched
    raster launches; every request's entries and workspace live in one device arena."""

    def __init__(self, device_scenes, slots: int, pool_bytes: int, opt, max_pixels: int,
                 keys_per_pixel: Dict[int, float], safety: float = 1.3, keep_results: bool = False):
        import torch
        from paper_2605_17855_amd import gs
        self.gs = gs
        self.torch = torch
        self.scenes = device_scenes
        self.opt = opt
        self.safety = safety
        self.kpp = dict(keys_per_pixel)      # per-scene calibration
        self.kpp_seen = {}                   # (scene, width, height) -> largest observed entries/pixel
        self.lock = threading.Lock()
        self.arena = _Arena(pool_bytes)
        self.arena_buf = torch.empty(self.arena.size, dtype=torch.uint8, device="cuda")
        nmax = max(s.n for s in device_scenes)
        self.slot_state = []
        for _ in range(slots):
            self.slot_state.append(dict(stream=torch.cuda.Stream(), proj=gs.Projected(nmax),
                                        image=torch.empty(3 * max_pixels, dtype=torch.float32, device="cuda")))
        self.raster_stream = torch.cuda.Stream()
        self.counters = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(8)]
        self.counter_i = 0
        self.pool = cf.ThreadPoolExecutor(max_workers=slots)
        self.futures = []
        self.raster_events = []
        self.keep_results = keep_results
        self.results = {}                    # rid -> (3, H, W) image, when keep_results
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def estimate_bytes(self, job):
        # entries per pixel fall as the resolution grows (a splat's tile count grows slower
        # than its pixel area), so observations are kept per resolution
        px = job.width * job.height
        kpp = self.kpp_seen.get((job.scene, job.width, job.height), self.kpp[job.scene])
        return job_bytes(self.scenes[job.scene].n, self.safety * kpp * px, px)

    def exact_bytes(self, job, n_keys):
        return job_bytes(self.scenes[job.scene].n, int(n_keys * 1.02) + 1024, job.width * job.height)

    def try_reserve(self, job, need):
        with self.lock:
            off = self.arena.alloc(need)
        if off is None:
            return False
        job.payload = dict(off=off)
        return True

    def _buffers(self, job, off):
        """Bins and workspace views carved from the arena at `off`."""
        gs = self.gs
        n = self.scenes[job.scene].n
        cap = entry_capacity(job.reserve, n, job.width * job.height)
        cam = self._camera(job)
        tx, ty = (job.width + 15) // 16, (job.height + 15) // 16
        g = self.opt.group
        nbins = ((tx + g - 1) // g) * ((ty + g - 1) // g)
        ws_bytes = int(gs.lib().gs_workspace_bytes(n, cap, gs.C.byref(gs.camera(cam)), gs.C.byref(self.opt)))
        buf = self.arena_buf
        o = off

        def take(nb, dtype, count):
            nonlocal o
            t = buf[o:o + nb].view(dtype)[:count]
            o += (nb + 255) // 256 * 256
            return t

        c = max(cap, 1)
        torch = self.torch
        keys = take(8 * c, torch.int64, c)
        vals = take(4 * c, torch.int32, c)
        masks = take(2 * c + 2, torch.int16, c)
        ranges = take(8 * nbins, torch.int32, 2 * nbins).view(nbins, 2)
        ws = take(ws_bytes, torch.uint8, ws_bytes)
        if o - off > job.reserve:
            raise RuntimeError("reservation layout overflow")
        return gs.Bins.from_tensors(keys, vals, masks, ranges, cap), ws, cam

    def _camera(self, job):
        from paper_2605_17855_amd import scenes
        return scenes.look_at(job.position, job.width, job.height)

    def start_prepare(self, job):
        self.futures.append(self.pool.submit(self._prepare, job))

    def _prepare(self, job):
        gs, torch = self.gs, self.torch
        st = self.slot_state[job.slot]
        bins, ws, cam = self._buffers(job, job.payload["off"])
        job.payload.update(bins=bins, ws=ws, cam=cam)
        ds = self.scenes[job.scene]
        proj = st["proj"]
        proj_n = gs.Projected.__new__(gs.Projected)
        proj_n.__dict__.update(proj.__dict__)
        proj_n.n = ds.n
        with torch.cuda.stream(st["stream"]):
            gs.gs_preprocess(ds, cam, self.opt, proj_n, ws, stream=st["stream"])
            try:
                n_keys = gs.gs_bin_sort(proj_n, cam, self.opt, bins, ws, stream=st["stream"])
            except gs.GsError as e:
                if e.status != gs.GS_ERR_CAPACITY:
                    raise
                return job, int(getattr(e, "n_keys", 0)), False
            ev = torch.cuda.Event()
            ev.record(st["stream"])
        job.payload.update(proj=proj_n, event=ev)
        return job, n_keys, True

    def poll_prepared(self):
        out = []
        keep = []
        for f in self.futures:
            if f.done():
                job, n_keys, ok = f.result()
                key = (job.scene, job.width, job.height)   # exact counts, also of failed attempts
                self.kpp_seen[key] = max(self.kpp_seen.get(key, 0.0), n_keys / (job.width * job.height))
                if not ok:
                    self.release(job)
                out.append((job, n_keys, ok))
            else:
                keep.append(f)
        self.futures = keep
        return out

    def start_raster(self, jobs):
        gs, torch = self.gs, self.torch
        rs = self.raster_stream
        items = []
        for j in jobs:
            rs.wait_event(j.payload["event"])
            img = self.slot_state[j.slot]["image"][: 3 * j.width * j.height]
            items.append((j.payload["proj"], j.payload["bins"], j.payload["cam"], img, None))
        counter = self.counters[self.counter_i % len(self.counters)]
        self.counter_i += 1
        gs.gs_rasterize_batch(items, self.opt, counter, stream=rs)
        if self.keep_results:
            with torch.cuda.stream(rs):
                for j, it in zip(jobs, items):
                    self.results[j.rid] = it[3].view(3, j.height, j.width).clone()
        ev = torch.cuda.Event()
        ev.record(rs)
        self.raster_events.append(ev)
        return ev

    def poll_rasters(self):
        out = [e for e in self.raster_events if e.query()]
        self.raster_events = [e for e in self.raster_events if e not in out]
        return out

    def release(self, job):
        if job.payload and "off" in job.payload:
            with self.lock:
                self.arena.release(job.payload["off"], job.reserve)
            job.payload = None

    def wait(self, until):
        if until is None:
            time.sleep(0)
        else:
            dt = until - self.now()
            if dt > 0:
                time.sleep(min(dt, 5e-4))

    def close(self):
        self.pool.shutdown(wait=True)
