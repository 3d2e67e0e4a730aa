"""Continuous-batching frame server for many smoke instances.

Each request asks for the next frame of one smoke instance (its density grid,
and optionally the march's bricked copy of it, stay resident on the device).
The HBM budget covers everything the server keeps on the device: the
resident grids and brick copies are charged when the scheduler starts (grids
and then brick copies are admitted smallest first; a brick copy that does not
fit is dropped and that instance's marches rebuild bricks in their per-batch
scratch; an instance whose grid does not fit is not served), and each batch's images, activations and
march scratch while it is in flight.  The scheduler admits pending requests
in arrival order as stream slots and budget free up: requests of the same
view resolution are grouped into a batch (held up to a stated deadline for
more of the same size while other batches keep the device busy), each is
marched from its own grid and camera, the batch goes through one U-Net call
and one shading launch that gives each image its own camera and light.
Batches are issued on several HIP streams, so work of requests that arrive
while others run overlaps on the device.  Every kernel computes an image
from that image's inputs only, in the same order regardless of batch
composition, so a frame is bit-identical alone and in a mix.

The device work is the library's (march, U-Net, shading); this module is
host-side scheduling, memory accounting and timing.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from . import lnm


@dataclasses.dataclass
class Instance:
    """One smoke instance: a resident density grid, its orbit camera and light."""
    key: int
    density: object  # torch float32 [n][n][n] on the device
    res: int
    sigma_scale: float = 8.0
    step_voxels: float = 4.0
    distance: float = 2.5
    fov_y_deg: float = 60.0
    deg_per_frame: float = 1.5
    start_deg: float = 0.0
    light: tuple = ((0.0, 1.0, 0.0), (1.0, 1.0, 1.0))
    seed: int = 0
    bricks: object = None  # optional bricked copy of the grid (lnm_make_bricks), resident like the grid

    def prepare(self, ctx):
        """Build the march's bricked copy of the (static) grid once, so each
        frame's march skips the relayout."""
        self.bricks = ctx.make_bricks(self.density)

    def camera(self, frame: int):
        a = math.radians(self.start_deg + self.deg_per_frame * frame)
        eye = (0.5 + self.distance * math.cos(a), 0.5, 0.5 + self.distance * math.sin(a))
        return _Cam(lnm.PERSPECTIVE, eye, (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), self.fov_y_deg, 0.8, self.res, self.res)


@dataclasses.dataclass
class _Cam:
    projection: int
    eye: tuple
    target: tuple
    up: tuple
    fov_y_deg: float
    ortho_half_extent: float
    width: int
    height: int


@dataclasses.dataclass
class Request:
    rid: int
    instance: int
    frame: int
    t_arrival: float  # seconds from the start of the run
    t_admit: float = -1.0
    t_done: float = -1.0
    batch: int = -1


class Backend:
    """Issues one batch of requests on one stream; returns a completion handle."""

    def __init__(self, ctx, net, n_streams: int = 4):
        import torch

        self.ctx, self.net = ctx, net
        # all streams at the default priority
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.keep = {}

    @staticmethod
    def resident_bytes(inst) -> int:
        """Device bytes an instance keeps resident: its grid and brick copy."""
        n = inst.density.numel() * inst.density.element_size()
        if inst.bricks is not None:
            n += inst.bricks.numel() * inst.bricks.element_size()
        return n

    def request_bytes(self, res: int) -> int:
        """Device bytes one request of this view size occupies while in flight
        (its images and its share of the batched U-Net activations)."""
        return 4 * res * res * (3 + 6 + 4) + self.net.workspace_bytes(1, res, res)

    def batch_bytes(self, reqs, instances) -> int:
        """Bytes a batch holds beyond its requests: one march scratch, reused
        by the batch's marches one after the other on its stream."""
        return max(self._march_bytes(instances[r.instance], r.frame) for r in reqs)

    def _march_bytes(self, inst, frame):
        prm = lnm.make_params(inst.step_voxels, seed=inst.seed, frame=frame)
        return self.ctx.march_workspace_bytes(inst.density, inst.sigma_scale, inst.camera(frame), prm,
                                              bricks=inst.bricks)

    def launch(self, slot: int, reqs, instances, keep_ids=()):
        import torch

        st = self.streams[slot]
        res = instances[reqs[0].instance].res
        B = len(reqs)
        with torch.cuda.stream(st):
            guide = torch.empty((B, res, res, 3), dtype=torch.float32, device="cuda")
            lm = torch.empty((B, res, res, 6), dtype=torch.float32, device="cuda")
            rgba = torch.empty((B, res, res, 4), dtype=torch.float32, device="cuda")
            ws = self.net.workspace(B, res, res)
            mws = torch.empty(self.batch_bytes(reqs, instances), dtype=torch.uint8, device="cuda")
            insts = [instances[r.instance] for r in reqs]
            # the batch's marches in one call (ragged grids, one camera and seed each)
            self.ctx.march_batch([i.density for i in insts], [i.sigma_scale for i in insts],
                                 [i.camera(r.frame) for i, r in zip(insts, reqs)],
                                 [lnm.make_params(i.step_voxels, seed=i.seed, frame=r.frame) for i, r in zip(insts, reqs)],
                                 outs=[guide[b] for b in range(B)], workspace=mws, stream=st,
                                 bricks=[i.bricks for i in insts])
            self.net.infer(guide, out=lm, workspace=ws, stream=st)
            # one shading launch for the batch, each image with its own camera and light
            self.ctx.composite_batch([i.camera(r.frame) for i, r in zip(insts, reqs)], [[i.light] for i in insts],
                                     lm, guide, out=rgba, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        for b, r in enumerate(reqs):
            if r.rid in keep_ids:
                self.keep[r.rid] = (guide[b], lm[b], rgba[b])
        return ev, (guide, lm, rgba, ws, mws)

    @staticmethod
    def done(handle) -> bool:
        return handle[0].query()


class Scheduler:
    """Admission by HBM budget and stream slots, batching by view size.

    hold_s: while at least one batch is in flight, a group of equal-size
    requests smaller than max_batch waits until its oldest request has waited
    this long (0: launch whatever is pending as soon as a slot is free); an
    idle device takes pending requests at once."""

    def __init__(self, backend, instances, budget_bytes: int, max_batch: int = 16, clock=time.perf_counter,
                 keep_ids=(), hold_s: float = 0.0):
        self.be, self.inst = backend, instances
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.clock = clock
        self.keep_ids = set(keep_ids)
        self.hold_s = float(hold_s)
        # resident data first: grids, then brick copies while they fit
        self.unserved = set()
        self.dropped_bricks = []
        resident = 0
        rb = getattr(backend, "resident_bytes", None)
        if rb is not None:
            for k in sorted(instances, key=lambda k: self._grid_bytes(instances[k])):
                g = self._grid_bytes(instances[k])
                if resident + g > self.budget:
                    self.unserved.add(k)
                else:
                    resident += g
            for k in sorted(instances, key=lambda k: self._grid_bytes(instances[k])):
                inst = instances[k]
                if k in self.unserved or getattr(inst, "bricks", None) is None:
                    continue
                extra = rb(inst) - self._grid_bytes(inst)
                if resident + extra <= self.budget:
                    resident += extra
                else:
                    inst.bricks = None
                    self.dropped_bricks.append(k)
        self.resident = resident
        self.in_use = resident
        self.peak_in_use = resident
        self.free_slots = list(range(len(getattr(backend, "streams", [0]))))
        self.inflight = []  # (slot, handle, reqs, bytes)
        self.done = []
        self.n_batches = 0
        self.rejected = []  # requests larger than the whole budget
        self.failed = []  # (request, error) of batches whose launch failed

    @staticmethod
    def _grid_bytes(inst) -> int:
        d = getattr(inst, "density", None)
        return d.numel() * d.element_size() if d is not None else 0

    def _ready(self, pending, now) -> bool:
        """Whether the oldest pending request's group should launch now."""
        if self.hold_s <= 0 or not self.inflight:
            return True
        first = pending[0]
        if now - first.t_arrival >= self.hold_s:
            return True
        res = self.inst[first.instance].res
        return sum(1 for r in pending if self.inst[r.instance].res == res) >= self.max_batch

    def _admit(self, pending, now):
        while pending and pending[0].instance in self.unserved:
            self.rejected.append(pending.popleft())
        while self.free_slots and pending and self._ready(pending, now):
            if pending[0].instance in self.unserved:
                self.rejected.append(pending.popleft())
                continue
            res = self.inst[pending[0].instance].res
            need1 = self.be.request_bytes(res)
            if hasattr(self.be, "batch_bytes"):
                need1 += self.be.batch_bytes([pending[0]], self.inst)
            if need1 > self.budget:  # can never fit, even alone
                self.rejected.append(pending.popleft())
                continue
            batch, used = [], 0
            keep = collections.deque()
            while pending and len(batch) < self.max_batch:
                r = pending.popleft()
                if self.inst[r.instance].res != res or r.instance in self.unserved:
                    keep.append(r)
                    continue
                nb = self.be.request_bytes(res)
                if self.in_use + used + nb > self.budget:
                    keep.append(r)
                    break
                batch.append(r)
                used += nb
            while keep:
                pending.appendleft(keep.pop())
            # per-batch bytes (the march scratch) must fit too; give back the
            # youngest requests of the batch until they do
            extra = self.be.batch_bytes(batch, self.inst) if batch and hasattr(self.be, "batch_bytes") else 0
            while batch and self.in_use + used + extra > self.budget:
                r = batch.pop()
                pending.appendleft(r)
                used -= self.be.request_bytes(res)
                extra = self.be.batch_bytes(batch, self.inst) if batch else 0
            if not batch:
                return
            used += extra
            slot = self.free_slots.pop()
            for r in batch:
                r.t_admit = now
                r.batch = self.n_batches
            try:
                handle = self.be.launch(slot, batch, self.inst, self.keep_ids)
            except (lnm.LnmError, MemoryError, RuntimeError) as e:
                # the batch never reached the device: release its slot and budget
                self.free_slots.append(slot)
                for r in batch:
                    self.failed.append((r, str(e)))
                self.n_batches += 1
                continue
            self.inflight.append((slot, handle, batch, used))
            self.in_use += used
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.n_batches += 1

    def _reap(self, now):
        still = []
        for slot, handle, batch, used in self.inflight:
            if self.be.done(handle):
                for r in batch:
                    r.t_done = now
                self.done.extend(batch)
                self.in_use -= used
                self.free_slots.append(slot)
            else:
                still.append((slot, handle, batch, used))
        self.inflight = still

    def run(self, requests, poll_sleep: float = 0.0):
        """Serve requests (sorted by t_arrival, seconds from start) in real time."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        pending = collections.deque()
        t0 = self.clock()
        i = 0
        while i < len(reqs) or pending or self.inflight:
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].t_arrival <= now:
                pending.append(reqs[i])
                i += 1
            self._reap(now)
            self._admit(pending, now)
            if poll_sleep:
                time.sleep(poll_sleep)
        return self.stats(self.clock() - t0)

    def stats(self, wall):
        lat = np.array([r.t_done - r.t_arrival for r in self.done]) * 1e3
        return {
            "requests": len(self.done),
            "rejected": len(self.rejected),
            "failed": len(self.failed),
            "batches": self.n_batches,
            "wall_s": wall,
            "throughput_fps": len(self.done) / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_batch": len(self.done) / max(self.n_batches, 1),
            "hold_ms": self.hold_s * 1e3,
            "resident_bytes": self.resident,
            "peak_bytes": self.peak_in_use,
            "peak_bytes_in_flight": self.peak_in_use - self.resident,
            "budget_bytes": self.budget,
            "instances_unserved": len(self.unserved),
            "brick_copies_dropped": len(self.dropped_bricks),
        }


def poisson_requests(n_instances: int, rate_hz: float, duration_s: float, seed: int = 7):
    """Aggregate Poisson arrivals; each request is the next frame of a
    uniformly chosen instance."""
    from synth.rng import substream

    s = substream(seed, "arrivals")
    n_est = int(rate_hz * duration_s * 1.5) + 16
    u = s.uniform(2 * n_est).reshape(n_est, 2)
    gaps = -np.log(1.0 - u[:, 0]) / rate_hz
    times = np.cumsum(gaps)
    frames = collections.Counter()
    out = []
    for k, (t, v) in enumerate(zip(times, u[:, 1])):
        if t > duration_s:
            break
        inst = int(v * n_instances)
        out.append(Request(k, inst, frames[inst], float(t)))
        frames[inst] += 1
    return out
