"""Continuous-batching render server: admission by duplicated-key memory, batched raster.

Requests (scene, resolution, pose, scheduled arrival) enter a FIFO.  A request is
admitted when a slot is free and its estimated memory (duplicated entries plus
per-Gaussian scratch) fits the pool next to every reservation already held.  An
admitted request runs preprocess + bin sort on a preparation stream; when its entries
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

# bytes per duplicated entry: key 8 + value 4 + mask 2, plus the workspace's bin key and depth
# rank and the sort's two double buffers (4 + 4 + 4 + 4) and its per-tile digit counts (1 B per
# key: 256 four-byte counts per tile of at least 1,024 keys), rounded up
BYTES_PER_ENTRY = 32
# per-Gaussian workspace bytes: scan partials, depth keys and their double buffers, the depth
# sort's two value buffers, each visible Gaussian's first-entry offset in depth order, and the
# depth sort's per-tile tables (2.5 B per key: 256 digit counts and 128 weights with their
# 64-bit scans per tile of 1,024 keys), rounded up
BYTES_PER_GAUSSIAN = 32


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
    cam: object = None       # backend-owned camera struct (built when the request is attached)


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
        if hasattr(be, "attach"):
            be.attach(jobs)
        max_inflight = min(self.max_inflight, getattr(be, "max_inflight", self.max_inflight))
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
            while ready and len(inflight) < max_inflight:
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


def mask_bytes(group: int) -> int:
    """Bytes of one entry's tile-membership mask (16 bits up to 4x4 groups, 64 for 8x8)."""
    return 8 if group == 8 else 2


def job_bytes(n_gaussians: int, n_entries: int, pixels: int, group: int = 1) -> int:
    per_entry = BYTES_PER_ENTRY - 2 + mask_bytes(group)
    return per_entry * int(n_entries) + BYTES_PER_GAUSSIAN * int(n_gaussians) + int(pixels) // 32 + FIXED_BYTES


def entry_capacity(reserve: int, n_gaussians: int, pixels: int, group: int = 1) -> int:
    """Entries a reservation of `reserve` bytes holds (inverse of job_bytes)."""
    per_entry = BYTES_PER_ENTRY - 2 + mask_bytes(group)
    return max(0, (int(reserve) - BYTES_PER_GAUSSIAN * int(n_gaussians) - int(pixels) // 32 - FIXED_BYTES)
               // per_entry)


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


class _Hip:
    """The few HIP runtime calls the backend needs for its events (ctypes releases the GIL
    while a call blocks, so a waiting thread never stalls the others)."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.lib = C.CDLL("libamdhip64.so")
        for name, args in (("hipEventCreateWithFlags", [C.c_void_p, C.c_uint]),
                           ("hipEventRecord", [C.c_void_p, C.c_void_p]),
                           ("hipStreamWaitEvent", [C.c_void_p, C.c_void_p, C.c_uint]),
                           ("hipEventSynchronize", [C.c_void_p]),
                           ("hipEventDestroy", [C.c_void_p])):
            f = getattr(self.lib, name)
            f.argtypes = args
            f.restype = C.c_int

    def _ok(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed with HIP error {rc}")

    def event(self):
        ev = self.C.c_void_p()
        self._ok(self.lib.hipEventCreateWithFlags(self.C.byref(ev), 0x2), "hipEventCreateWithFlags")  # no timing
        return ev.value

    def record(self, ev, stream):
        self._ok(self.lib.hipEventRecord(ev, stream), "hipEventRecord")

    def wait_event(self, stream, ev):
        self._ok(self.lib.hipStreamWaitEvent(stream, ev, 0), "hipStreamWaitEvent")

    def synchronize(self, ev):
        self._ok(self.lib.hipEventSynchronize(ev), "hipEventSynchronize")

    def destroy(self, ev):
        self.lib.hipEventDestroy(ev)


class GpuBackend:
    """Drives the HIP library: a few preparation streams for preprocess + sort (slots map onto
    them round-robin) and one stream for batched raster launches; every request's entries and
    workspace live in one device arena.  The stream count matches the process's hardware
    queues (4 by default): more streams than queues would share queues, and in-order queues
    would then hold a request's preparation, and the host synchronization inside it, behind
    unrelated raster batches.

    Host work per request is kept small: the camera struct is built when the request is
    attached, buffers are raw pointers into the arena, and completions (a prepared request, a
    finished raster launch) arrive through a queue that wakes the scheduler instead of being
    polled."""

    def __init__(self, device_scenes, slots: int, pool_bytes: int, opt, max_pixels: int,
                 keys_per_pixel: Dict[int, float], safety: float = 1.3, keep_results: bool = False,
                 prep_streams: int = 3, max_inflight_batches: int = 4):
        import queue
        import torch
        from paper_2605_17855_amd import gs
        self.gs = gs
        self.C = gs.C
        self.L = gs.lib()
        self.torch = torch
        self.hip = _Hip()
        self.scenes = device_scenes
        self.opt = opt
        self.safety = safety
        self.kpp = dict(keys_per_pixel)      # per-scene calibration
        self.kpp_seen = {}                   # (scene, width, height) -> largest observed entries/pixel
        self.lock = threading.Lock()
        self.arena = _Arena(pool_bytes)
        self.arena_buf = torch.empty(self.arena.size, dtype=torch.uint8, device="cuda")
        self.base = self.arena_buf.data_ptr()
        nmax = max(s.n for s in device_scenes)
        self.prep_streams = [torch.cuda.Stream() for _ in range(max(1, prep_streams))]
        self.slot_state = []
        for i in range(slots):
            self.slot_state.append(dict(proj=gs.Projected(nmax),
                                        image=torch.empty(3 * max_pixels, dtype=torch.float32, device="cuda"),
                                        stream=self.prep_streams[i % len(self.prep_streams)],
                                        event=self.hip.event()))
        for st in self.slot_state:
            st["stream_h"] = st["stream"].cuda_stream
            st["image_ptr"] = st["image"].data_ptr()
        self.raster_stream = torch.cuda.Stream()
        self.raster_h = self.raster_stream.cuda_stream
        self.max_inflight = max_inflight_batches
        self.counters = torch.zeros(2 * max_inflight_batches * gs.BATCH_COUNTER_WORDS, dtype=torch.int32,
                                    device="cuda")
        self.counter_i = 0
        self.raster_events = [self.hip.event() for _ in range(2 * max_inflight_batches)]
        self.pool = cf.ThreadPoolExecutor(max_workers=slots)
        self.done = queue.Queue()            # ("prepared", job, n_keys, ok) | ("raster", handle) | ("error", e)
        self.pending = []
        self.signal = threading.Event()
        self.raster_fifo = queue.Queue()     # (handle, event) in launch order, for the waiter
        self.waiter = threading.Thread(target=self._raster_waiter, daemon=True)
        self.waiter.start()
        self.keep_results = keep_results
        self.results = {}                    # rid -> (3, H, W) image, when keep_results
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def attach(self, jobs):
        """Per-request host work that belongs to the client: the camera struct of each pose."""
        from paper_2605_17855_amd import scenes
        for job in jobs:
            job.cam = self.gs.camera(scenes.look_at(job.position, job.width, job.height))

    def estimate_bytes(self, job):
        # entries per pixel fall as the resolution grows (a splat's tile count grows slower
        # than its pixel area), so observations are kept per resolution
        px = job.width * job.height
        kpp = self.kpp_seen.get((job.scene, job.width, job.height), self.kpp[job.scene])
        return job_bytes(self.scenes[job.scene].n, self.safety * kpp * px, px, self.opt.group)

    def exact_bytes(self, job, n_keys):
        return job_bytes(self.scenes[job.scene].n, int(n_keys * 1.02) + 1024, job.width * job.height, self.opt.group)

    def try_reserve(self, job, need):
        with self.lock:
            off = self.arena.alloc(need)
        if off is None:
            return False
        job.payload = dict(off=off)
        return True

    def _buffers(self, job, off):
        """gs_bins and workspace carved from the arena at `off` (raw device pointers)."""
        gs, C = self.gs, self.C
        n = self.scenes[job.scene].n
        cap = entry_capacity(job.reserve, n, job.width * job.height, self.opt.group)
        tx, ty = (job.width + 15) // 16, (job.height + 15) // 16
        g = self.opt.group
        nbins = ((tx + g - 1) // g) * ((ty + g - 1) // g)
        ws_bytes = int(self.L.gs_workspace_bytes(n, cap, C.byref(job.cam), C.byref(self.opt)))
        o = off

        def take(nb):
            nonlocal o
            ptr = self.base + o
            o += (nb + 255) // 256 * 256
            return ptr

        c = max(cap, 1)
        b = gs.gs_bins()
        b.keys = take(8 * c)
        b.vals = take(4 * c)
        b.masks = take(mask_bytes(self.opt.group) * c + 8)
        b.capacity = cap
        b.ranges = take(8 * nbins)
        ws = take(ws_bytes)
        if o - off > job.reserve:
            raise RuntimeError("reservation layout overflow")
        return b, ws, ws_bytes

    def start_prepare(self, job):
        self.pool.submit(self._prepare, job)

    def _prepare(self, job):
        gs, C, L = self.gs, self.C, self.L
        try:
            st = self.slot_state[job.slot]
            bins, ws, ws_bytes = self._buffers(job, job.payload["off"])
            job.payload.update(bins=bins)
            ds = self.scenes[job.scene]
            proj = st["proj"].struct
            rc = L.gs_preprocess(C.byref(ds.struct), C.byref(job.cam), C.byref(self.opt), C.byref(proj), ws,
                                 ws_bytes, st["stream_h"])
            if rc != gs.GS_OK:
                raise gs.GsError(rc, L.gs_last_error().decode())
            n_keys = C.c_uint64(0)
            rc = L.gs_bin_sort(C.byref(proj), ds.n, C.byref(job.cam), C.byref(self.opt), C.byref(bins),
                               C.byref(n_keys), ws, ws_bytes, st["stream_h"])
            if rc == gs.GS_ERR_CAPACITY:
                self.done.put(("prepared", job, int(n_keys.value), False))
            elif rc != gs.GS_OK:
                raise gs.GsError(rc, L.gs_last_error().decode())
            else:
                self.hip.record(st["event"], st["stream_h"])
                self.done.put(("prepared", job, int(n_keys.value), True))
        except BaseException as e:                 # surfaced by the scheduler thread
            self.done.put(("error", e))
        self.signal.set()

    def _raster_waiter(self):
        while True:
            item = self.raster_fifo.get()
            if item is None:
                return
            handle, ev = item
            self.hip.synchronize(ev)
            self.done.put(("raster", handle))
            self.signal.set()

    def _take(self, kind):
        """Completions of one kind; the rest stay pending for the other poll."""
        import queue
        while True:
            try:
                self.pending.append(self.done.get_nowait())
            except queue.Empty:
                break
        out = [it for it in self.pending if it[0] == kind or it[0] == "error"]
        self.pending = [it for it in self.pending if not (it[0] == kind or it[0] == "error")]
        for it in out:
            if it[0] == "error":
                raise it[1]
        return out

    def poll_prepared(self):
        out = []
        for _, job, n_keys, ok in self._take("prepared"):
            key = (job.scene, job.width, job.height)   # exact counts, also of failed attempts
            self.kpp_seen[key] = max(self.kpp_seen.get(key, 0.0), n_keys / (job.width * job.height))
            if not ok:
                self.release(job)
            out.append((job, n_keys, ok))
        return out

    def start_raster(self, jobs):
        gs, C = self.gs, self.C
        arr = (gs.gs_job * len(jobs))()
        for i, j in enumerate(jobs):
            st = self.slot_state[j.slot]
            self.hip.wait_event(self.raster_h, st["event"])
            arr[i].proj = C.pointer(st["proj"].struct)
            arr[i].bins = C.pointer(j.payload["bins"])
            arr[i].cam = j.cam
            arr[i].image = st["image_ptr"]
            arr[i].aux = None
        k = self.counter_i % len(self.raster_events)
        self.counter_i += 1
        rc = self.L.gs_rasterize_batch(arr, len(jobs), C.byref(self.opt),
                                       self.counters[k * gs.BATCH_COUNTER_WORDS:].data_ptr(), self.raster_h)
        if rc != gs.GS_OK:
            raise gs.GsError(rc, self.L.gs_last_error().decode())
        if self.keep_results:
            with self.torch.cuda.stream(self.raster_stream):
                for j in jobs:
                    img = self.slot_state[j.slot]["image"][: 3 * j.width * j.height]
                    self.results[j.rid] = img.view(3, j.height, j.width).clone()
        ev = self.raster_events[k]
        self.hip.record(ev, self.raster_h)
        handle = ("batch", self.counter_i)
        self.raster_fifo.put((handle, ev))
        return handle

    def poll_rasters(self):
        return [it[1] for it in self._take("raster")]

    def release(self, job):
        if job.payload and "off" in job.payload:
            with self.lock:
                self.arena.release(job.payload["off"], job.reserve)
            job.payload = None

    def wait(self, until):
        timeout = 0.002 if until is None else max(0.0, min(until - self.now(), 0.002))
        if self.signal.wait(timeout):
            self.signal.clear()

    def close(self):
        self.pool.shutdown(wait=True)
        self.raster_fifo.put(None)
        self.waiter.join()
        self.torch.cuda.synchronize()
        for st in self.slot_state:
            self.hip.destroy(st["event"])
        for ev in self.raster_events:
            self.hip.destroy(ev)
