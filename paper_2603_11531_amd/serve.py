"""Continuous-batching render server over mgs_render_batch.

* Scenes stay resident in HBM (``SceneRegistry``).
* Requests (scene, camera, background) arrive on an open-loop clock; the server
  admits queued requests into a batch slot while the slot's limits (requests,
  Gaussians, tiles, pair capacity) and the output-image memory budget allow.
* Each slot owns a workspace, a pinned request table and a CUDA/HIP stream; with
  ``use_graphs`` the slot's launch sequence (table upload + mgs_render_batch) is
  captured once in a graph and replayed for every batch.  Two or more slots keep
  batches in flight together, so requests that arrive while others render are
  admitted as soon as a slot and memory free up.
* Latency = completion (GPU event) - arrival; reported as p50 / p99 with
  throughput.  A batch whose pairs exceeded the slot capacity is re-rendered
  request by request on the single-view path (same kernels, same images).
"""
from __future__ import annotations

import ctypes as C
import math
import time
from collections import deque
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .render import ALPHA_MAX, ALPHA_MIN, DeviceMLP, DeviceScene, Renderer

MAX_REQ = 64
N_ALIGN = 256          # a request's Gaussian range in a batch starts on a multiple of this (as in the library)


def _tiles(w, h):
    return ((w + 15) // 16) * ((h + 15) // 16)


@dataclass
class Request:
    rid: int
    scene: str
    cam: object            # mgs_data.Camera
    arrival: float         # seconds on the server clock
    bg: tuple = (0.0, 0.0, 0.0)
    image: torch.Tensor = None
    start: float = None    # GPU start of the batch (or frame) that rendered it
    done: float = None     # image ready
    path: str = ""


class SceneRegistry:
    """Resident scenes: id -> (DeviceScene, DeviceMLP or None)."""

    def __init__(self):
        self.scenes = {}

    def add(self, name, scene, mlp=None, device="cuda"):
        ds = scene if isinstance(scene, DeviceScene) else DeviceScene(scene, device)
        if ds.sh_degree != 1:
            raise ValueError("the batched renderer takes first-order SH scenes")
        dm = mlp if (mlp is None or isinstance(mlp, DeviceMLP)) else DeviceMLP(mlp, device)
        self.scenes[name] = (ds, dm)

    def __getitem__(self, k):
        return self.scenes[k]

    def resident_bytes(self):
        return sum(ds.nbytes() for ds, _ in self.scenes.values())


class BatchSlot:
    """Workspace + request table + stream for one in-flight batch."""

    def __init__(self, max_gaussians, max_tiles, capacity, device="cuda", use_graphs=True):
        self.max_gaussians, self.max_tiles, self.capacity = int(max_gaussians), int(max_tiles), int(capacity)
        self.device = torch.device(device)
        nb = C.c_size_t()
        L.check(L.lib().mgs_batch_workspace(self.max_gaussians, self.max_tiles, self.capacity, C.byref(nb)))
        self.ws = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device=self.device)
        self.req_size = C.sizeof(L.mgs_request)
        self.table_host = torch.zeros(MAX_REQ * self.req_size + 16, dtype=torch.uint8).pin_memory()
        self.table_dev = torch.zeros(MAX_REQ * self.req_size + 16, dtype=torch.uint8, device=self.device)
        self.n_pairs = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(2, dtype=torch.int32, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.start_event = torch.cuda.Event(enable_timing=True)
        self.done_event = torch.cuda.Event(enable_timing=True)
        self.requests = []
        self.graph = None
        self.use_graphs = use_graphs

    def _n_ptr(self):
        return C.c_void_p(self.table_dev.data_ptr() + MAX_REQ * self.req_size)

    def _enqueue(self):
        """Table upload + the batched render, on self.stream."""
        self.table_dev.copy_(self.table_host, non_blocking=True)
        L.check(L.lib().mgs_render_batch(
            C.c_void_p(self.table_dev.data_ptr()), self._n_ptr(), self.max_gaussians, self.max_tiles,
            self.capacity, ALPHA_MIN, ALPHA_MAX, L.ptr(self.ws), self.ws.numel() * 4, L.ptr(self.n_pairs),
            L.ptr(self.status), L.stream_ptr(self.stream)))

    def write_table(self, reqs, registry):
        arr = (L.mgs_request * MAX_REQ)()
        for k, r in enumerate(reqs):
            ds, dm = registry[r.scene]
            q = arr[k]
            q.g = ds.struct
            q.packed_mlp = dm.packed.data_ptr() if dm is not None else None
            q.cam = L.make_camera(r.cam)
            for c in range(3):
                q.bg[c] = float(r.bg[c])
            q.image = r.image.data_ptr()
        raw = bytes(arr) + np.int32(len(reqs)).tobytes()
        self.table_host[:len(raw)].copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))

    def launch(self, reqs, registry):
        self.requests = list(reqs)
        self.write_table(reqs, registry)
        with torch.cuda.stream(self.stream):
            self.start_event.record(self.stream)
            if self.use_graphs:
                if self.graph is None:
                    self._enqueue()                      # warm-up outside capture
                    self.stream.synchronize()
                    self.graph = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(self.graph, stream=self.stream):
                        self._enqueue()
                self.graph.replay()
            else:
                self._enqueue()
            self.done_event.record(self.stream)

    def ready(self):
        return self.done_event.query()

    def overflowed(self):
        return (int(self.n_pairs.cpu()[0]) & 0xFFFFFFFF) > self.capacity

    def rendered(self):
        """True when the batch plan accepted every request (status = {1, count}); a batch the
        plan refused (a request outside the slot's limits) rendered nothing."""
        ok, count = (int(v) for v in self.status.cpu())
        return ok == 1 and count == len(self.requests)


def form_batch(queue, footprint, max_batch, max_gaussians, max_tiles, capacity, image_budget, image_in_use):
    """FIFO admission: pop requests from the head of ``queue`` while the batch stays within
    the request, Gaussian, tile, estimated-pair and image-memory limits.  The first request
    of a batch is admitted on its Gaussians / tiles / memory alone (its pair estimate may
    exceed the capacity: the slot then overflows and the request is re-rendered on the
    single-view path).  Returns the admitted requests in arrival order."""
    batch, n_sum, t_sum, p_sum, b_sum = [], 0, 0, 0, 0
    while queue and len(batch) < max_batch:
        n, t, b, p = footprint(queue[0])
        if n_sum + n > max_gaussians or t_sum + t > max_tiles or image_in_use + b_sum + b > image_budget or \
                (batch and p_sum + p > capacity):
            break
        batch.append(queue.popleft())
        n_sum, t_sum, p_sum, b_sum = n_sum + n, t_sum + t, p_sum + p, b_sum + b
    return batch


class GpuBackend:
    """What the server needs from the device: batch slots, a clock, images, a single-view retry
    and the GPU time stamps of a finished slot.  A test can pass a simulated backend with the
    same methods (and a clock it controls) to exercise the scheduling on the CPU."""

    def __init__(self, device="cuda", use_graphs=True):
        self.device = torch.device(device)
        self.use_graphs = use_graphs

    def new_slot(self, max_gaussians, max_tiles, capacity):
        return BatchSlot(max_gaussians, max_tiles, capacity, self.device, self.use_graphs)

    def start(self):
        """Begin a run: the origin of now() and of slot_times()."""
        self.ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        self.ref.record()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep(self, seconds):
        time.sleep(seconds)

    def image(self, W, H):
        return torch.empty(3, H, W, dtype=torch.float32, device=self.device)

    def slot_times(self, slot):
        """(GPU start, GPU end) of a finished slot's batch, seconds from start()."""
        return self.ref.elapsed_time(slot.start_event) * 1e-3, self.ref.elapsed_time(slot.done_event) * 1e-3

    def render_alone(self, registry, r):
        ds, dm = registry[r.scene]
        R = Renderer(ds.n, r.cam.width, r.cam.height, device=self.device)
        img = R.render(ds, r.cam, dm, bg=r.bg)
        torch.cuda.synchronize()
        r.image = img.clone()

    def finish(self):
        torch.cuda.synchronize()


class Server:
    """Open-loop continuous-batching server (see the module docstring).  ``timeout_s``: a
    request still queued that long after its arrival is cancelled (``self.timed_out``) instead
    of rendered."""

    def __init__(self, registry, max_batch=16, max_gaussians=8_000_000, max_tiles=None, capacity=64_000_000,
                 n_slots=2, image_budget_bytes=2 << 30, use_graphs=True, device="cuda", timeout_s=None,
                 backend=None):
        self.reg = registry
        self.max_batch = min(int(max_batch), MAX_REQ)
        self.max_gaussians = int(max_gaussians)
        self.max_tiles = int(max_tiles if max_tiles is not None else self.max_batch * _tiles(1920, 1080))
        self.capacity = int(capacity)
        self.image_budget = int(image_budget_bytes)
        self.timeout_s = timeout_s
        self.backend = backend if backend is not None else GpuBackend(device, use_graphs)
        self.device = getattr(self.backend, "device", None)
        self.slots = [self.backend.new_slot(self.max_gaussians, self.max_tiles, self.capacity) for _ in range(n_slots)]
        self.image_bytes_in_use = 0
        self.rejected = []
        self.timed_out = []
        self.unserved = []
        self.pair_est = {}           # (scene, W, H) -> pairs of one view (from calibrate)

    def calibrate(self, resolutions, margin=1.3, radius=4.0):
        """Measure the pair count of one view per (scene, resolution) on the single-view path;
        admission then keeps the batch's estimated pairs within the slot capacity."""
        import mgs_data
        for name, (ds, dm) in self.reg.scenes.items():
            for W, H in resolutions:
                cam = mgs_data.look_at((0.0, 0.0, -radius), width=W, height=H, f=float(W))
                R = Renderer(ds.n, W, H, device=self.device)
                R.render(ds, cam, dm)
                self.pair_est[(name, W, H)] = int(R.pairs() * margin) + 1024
                del R
        torch.cuda.synchronize()

    # -- footprint ------------------------------------------------------------
    def footprint(self, r):
        """(padded Gaussians, tiles, image bytes, estimated pairs) a request needs in a batch."""
        ds, _ = self.reg[r.scene]
        n = (ds.n + N_ALIGN - 1) // N_ALIGN * N_ALIGN
        pairs = self.pair_est.get((r.scene, r.cam.width, r.cam.height), 0)
        return n, _tiles(r.cam.width, r.cam.height), 12 * r.cam.width * r.cam.height, pairs

    def admissible_alone(self, r):
        c = r.cam
        if not (c.width > 0 and c.height > 0 and c.fx > 0 and c.fy > 0 and c.near > 0):
            return False                         # the library would refuse this camera
        n, t, b, p = self.footprint(r)
        return n <= self.max_gaussians and t <= self.max_tiles and b <= self.image_budget

    # -- one run --------------------------------------------------------------
    def run(self, requests, idle_sleep=20e-6, duration=None, keep_images=True):
        """Serve ``requests`` (sorted by arrival, seconds from start); returns the served list.
        With ``duration`` no batch starts after that many seconds: requests that arrived and were
        not started are left in ``self.unserved`` (the queue at the end of an overloaded run),
        later arrivals are not offered.  ``keep_images=False`` drops each image once its request
        is complete (long replays)."""
        be = self.backend
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        served = []
        self.unserved = []
        free = list(self.slots)
        busy = []
        be.start()
        while pending or queue or busy:
            now = be.now()
            if duration is not None and now >= duration:
                self.unserved.extend(queue)
                self.unserved.extend(r for r in pending if r.arrival <= duration)
                queue.clear()
                pending.clear()
                if not busy:
                    break
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                if self.admissible_alone(r):
                    queue.append(r)
                else:
                    self.rejected.append(r)
            if self.timeout_s is not None:
                while queue and now - queue[0].arrival > self.timeout_s:     # FIFO: the oldest first
                    r = queue.popleft()
                    r.path = "timed out"
                    self.timed_out.append(r)
            progressed = False
            for slot in list(busy):
                if slot.ready():
                    busy.remove(slot)
                    free.append(slot)
                    progressed = True
                    t_start, t_done = be.slot_times(slot)
                    if slot.overflowed() or not slot.rendered():
                        # pair capacity exceeded, or the plan refused the batch: each request
                        # is rendered on the single-view path
                        for r in slot.requests:
                            r.start = be.now()
                            be.render_alone(self.reg, r)
                            r.done = be.now()
                            r.path = "single-view retry"
                    else:
                        for r in slot.requests:
                            r.start, r.done = t_start, t_done
                            r.path = "batch"
                    for r in slot.requests:
                        self.image_bytes_in_use -= 12 * r.cam.width * r.cam.height
                        if not keep_images:
                            r.image = None
                    served.extend(slot.requests)
            while free and queue:
                batch = form_batch(queue, self.footprint, self.max_batch, self.max_gaussians, self.max_tiles,
                                   self.capacity, self.image_budget, self.image_bytes_in_use)
                for r in batch:
                    r.image = be.image(r.cam.width, r.cam.height)
                    self.image_bytes_in_use += 12 * r.cam.width * r.cam.height
                if not batch:
                    break
                slot = free.pop()
                slot.launch(batch, self.reg)
                busy.append(slot)
                progressed = True
            if not progressed:
                if pending and not queue and not busy:
                    be.sleep(max(0.0, min(pending[0].arrival - now, 1e-3)))
                else:
                    be.sleep(idle_sleep)
        be.finish()
        return served

    def _render_alone(self, r):
        self.backend.render_alone(self.reg, r)


def run_plain_loop(registry, requests, device="cuda", duration=None, keep_images=True, unserved=None):
    """Baseline: one request at a time, one frame per launch sequence (single-view path), FIFO.
    ``duration`` / ``keep_images`` as for Server.run; requests that arrived before the end and
    were not started are appended to ``unserved`` (a list) when given."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    renderers = {}
    served = []
    ref = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.record()
    while pending:
        now = time.perf_counter() - t0
        if duration is not None and now >= duration:
            if unserved is not None:
                unserved.extend(r for r in pending if r.arrival <= duration)
            break
        if duration is not None and pending[0].arrival > duration:
            break                                   # no arrival left inside the window
        r = pending.popleft()
        if r.arrival > now:
            time.sleep(r.arrival - now)
        ds, dm = registry[r.scene]
        key = (r.scene, r.cam.width, r.cam.height)
        if key not in renderers:
            renderers[key] = Renderer(ds.n, r.cam.width, r.cam.height, device=device)
        R = renderers[key]
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        img = R.render(ds, r.cam, dm, bg=r.bg)      # one host sync per frame (pair count check)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        r.image = img.clone()
        ev.synchronize()
        r.start = ref.elapsed_time(ev0) * 1e-3
        r.done = ref.elapsed_time(ev) * 1e-3
        r.path = "plain"
        if not keep_images:
            r.image = None
        served.append(r)
    torch.cuda.synchronize()
    return served


def latency_stats(served, t_span=None):
    """Latency = arrival -> image ready (queueing included); service = the GPU start of the
    request's batch (or frame) -> image ready (queueing excluded)."""
    lat = np.array([r.done - r.arrival for r in served]) * 1e3
    if len(lat) == 0:
        return {}
    svc = np.array([r.done - r.start for r in served]) * 1e3
    end = max(r.done for r in served)
    start = min(r.arrival for r in served)
    span = t_span if t_span is not None else max(end - start, 1e-9)
    return {"requests": len(served), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "service_p50_ms": float(np.percentile(svc, 50)), "service_p99_ms": float(np.percentile(svc, 99)),
            "frames_per_s": len(served) / span,
            "mpix_per_s": sum(r.cam.width * r.cam.height for r in served) / span / 1e6}


def poisson_requests(scene_names, rate, count, seed, resolutions=((640, 480), (1280, 720), (1600, 1063), (1920, 1080)),
                     radius=4.0):
    """Open-loop arrivals: exponential gaps at ``rate`` req/s, random scene, pose and resolution."""
    import mgs_data
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        name = scene_names[int(rng.integers(len(scene_names)))]
        az = rng.uniform(0, 2 * math.pi)
        el = math.radians(rng.uniform(-20.0, 40.0))
        W, H = resolutions[int(rng.integers(len(resolutions)))]
        eye = (radius * math.cos(el) * math.sin(az), -radius * math.sin(el), -radius * math.cos(el) * math.cos(az))
        cam = mgs_data.look_at(eye, width=W, height=H, f=float(W))
        out.append(Request(rid=k, scene=name, cam=cam, arrival=t))
    return out
