"""Continuous-batching render server on one GPU.

Render jobs (scene, camera, parameters) arrive over time.  The server keeps
the scenes resident on the device, admits an arrived job when a slot is
free and its frame buffers fit the HBM budget, and advances every admitted
job a bounded number of tiles per step, all of them in ONE persistent
kernel launch (tr_render_batch_tiles).  A job that arrives while others are
on the GPU joins at the next step; a finished job frees its slot and its
memory at once.  Frame latency is measured from arrival to the completion
of the launch that rendered the job's last tiles (GPU event timing).

Pixel values depend only on (scene, camera, params, pixel), so a job's frame
is bit-identical whether it is rendered alone or in any mix.

The admission and step-planning policies are plain functions of host state
(no device calls), testable without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import paper_0801_1500_amd as tr

SERVE_TILE_W = 8  # tile shape of the served launches (tile ranges are in these units)


@dataclasses.dataclass
class Job:
    job_id: int
    arrival: float            # seconds after the stream start
    scene: int                # index into the server's scene list
    camera: object
    params: object
    # filled in by the server
    n_tiles: int = 0
    next_tile: int = 0
    footprint: int = 0
    frame: Optional[dict] = None
    admitted: Optional[float] = None
    done: Optional[float] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


def admit(queue: Sequence[Job], n_active: int, free_bytes: int, max_slots: int,
          now: float) -> List[Job]:
    """Jobs to admit now, in arrival order: a job is admitted when it has
    arrived, a slot is free and its footprint fits the free budget; the
    queue is served in order (no job overtakes an earlier arrival that is
    waiting for memory), which bounds every job's wait."""
    out = []
    for job in queue:
        if job.arrival > now or n_active + len(out) >= max_slots:
            break
        if job.footprint > free_bytes:
            break
        out.append(job)
        free_bytes -= job.footprint
    return out


def plan_step(active: Sequence[Job], tile_budget: int) -> List[tuple]:
    """(job, tile_begin, tile_end) for one launch: the budget goes to the
    earliest-admitted jobs first, so old jobs finish first (low p99)."""
    plan = []
    left = tile_budget
    for job in sorted(active, key=lambda j: (j.arrival, j.job_id)):
        if left <= 0:
            break
        rem = job.n_tiles - job.next_tile
        if rem <= 0:
            continue
        take = min(rem, left)
        plan.append((job, job.next_tile, job.next_tile + take))
        left -= take
    return plan


@dataclasses.dataclass
class ServeStats:
    jobs: int = 0
    steps: int = 0
    launched_tiles: int = 0
    max_active: int = 0
    max_launch_jobs: int = 0
    memory_waits: int = 0      # steps at which an arrived job waited for memory
    slot_waits: int = 0
    rays: int = 0
    wall_s: float = 0.0
    latencies: List[float] = dataclasses.field(default_factory=list)

    def summary(self) -> dict:
        lat = sorted(self.latencies)
        pct = lambda q: lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)] if lat else float("nan")
        return dict(jobs=self.jobs, steps=self.steps, max_active=self.max_active,
                    max_jobs_per_launch=self.max_launch_jobs, memory_waits=self.memory_waits,
                    slot_waits=self.slot_waits, wall_s=self.wall_s,
                    latency_ms_p50=1e3 * pct(0.50), latency_ms_p99=1e3 * pct(0.99),
                    latency_ms_max=1e3 * (lat[-1] if lat else float("nan")),
                    rays=self.rays, rays_per_s=self.rays / self.wall_s if self.wall_s else 0.0)


class Server:
    """scenes: list of resident tr.Scene.  hbm_budget: bytes of frame
    buffers that may be in use at once."""

    def __init__(self, scenes: Sequence["tr.Scene"], hbm_budget: int = 64 << 30,
                 max_slots: int = 64, tile_budget: int = 24576, precision: str = "fp32_resolve",
                 outputs: Sequence[str] = ("rgb",), keep_frames: bool = False,
                 max_inflight: int = 2, stream=None):
        import torch
        if precision not in ("fp32", "fp32_resolve"):
            raise ValueError("the server renders tile ranges, which need an FP32 precision "
                             "('fp32' or 'fp32_resolve'), not %r" % (precision,))
        self.torch = torch
        self.scenes = list(scenes)
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.tile_budget = int(tile_budget)
        self.precision = precision
        self.outputs = tuple(outputs)
        self.keep_frames = keep_frames
        self.max_inflight = max(1, int(max_inflight))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.tune = {"tile_w": SERVE_TILE_W}
        self.stats_buf = torch.zeros(tr.STAT_COUNT, dtype=torch.int64, device="cuda")

    def _flags(self) -> int:
        return sum(1 << i for i, k in enumerate(("rgb", "hit_id", "ao_mask", "light_mask"))
                   if k in self.outputs) or 1

    def prepare(self, job: Job):
        if int(getattr(job.params, "aa_samples", 1)) > 1:
            # tile ranges carry one sample per pixel; an antialiased frame is
            # the ordered mean of its sample frames, rendered whole
            raise ValueError("job %d: the server renders tile ranges, which take one primary "
                             "sample per pixel; render antialiased frames with tr.render"
                             % job.job_id)
        job.n_tiles = tr.tile_count(job.camera.width, job.camera.height, SERVE_TILE_W)
        job.footprint = tr.frame_footprint(job.camera, job.params, self._flags())
        job.next_tile = 0

    def run(self, jobs: Sequence[Job], realtime: bool = True,
            on_done: Optional[Callable[[Job], None]] = None) -> ServeStats:
        torch = self.torch
        st = ServeStats(jobs=len(jobs))
        queue = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.job_id)))
        for j in queue:
            self.prepare(j)
            if j.footprint > self.budget:
                raise ValueError("job %d needs %d bytes, budget is %d" % (j.job_id, j.footprint,
                                                                          self.budget))
        active: List[Job] = []
        inflight = collections.deque()   # (event, [jobs finishing at this launch])
        used = 0
        self.stats_buf.zero_()
        torch.cuda.synchronize()
        start_ev = torch.cuda.Event(enable_timing=True)
        start_ev.record(self.stream)
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))

        def retire(block: bool):
            nonlocal used
            while inflight and (block or inflight[0][0].query()):
                ev, finishing = inflight.popleft()
                ev.synchronize()
                t_done = start_ev.elapsed_time(ev) * 1e-3
                for job in finishing:
                    job.done = t_done
                    st.latencies.append(job.done - (job.arrival if realtime else 0.0))
                    active.remove(job)
                    used -= job.footprint
                    if on_done is not None:
                        on_done(job)
                    if not self.keep_frames:
                        job.frame = None
                    elif job.frame is not None:
                        job.frame.pop("stats", None)
                block = False

        while queue or active:
            retire(block=False)
            now = clock()
            # admission
            new = admit(queue, len(active), self.budget - used, self.max_slots, now)
            if queue and queue[0].arrival <= now and not new:
                if len(active) >= self.max_slots:
                    st.slot_waits += 1
                else:
                    st.memory_waits += 1
            for job in new:
                queue.popleft()
                job.admitted = now if realtime else 0.0
                job.frame = tr.alloc_frame(job.camera, self.outputs)
                job.frame["stats"] = self.stats_buf  # one counter block per launch
                used += job.footprint
                active.append(job)
            st.max_active = max(st.max_active, len(active))
            plan = plan_step([j for j in active if j.next_tile < j.n_tiles], self.tile_budget)
            if plan and len(inflight) < self.max_inflight:
                jl = [p[0] for p in plan]
                tr.render_batch_tiles_into([self.scenes[j.scene] for j in jl],
                                           [j.camera for j in jl], [j.params for j in jl],
                                           [j.frame for j in jl], [p[1] for p in plan],
                                           [p[2] for p in plan], self.precision, self.tune,
                                           self.stream)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.stream)
                finishing = []
                for job, b, e in plan:
                    job.next_tile = e
                    st.launched_tiles += e - b
                    if e == job.n_tiles:
                        finishing.append(job)
                inflight.append((ev, finishing))
                st.steps += 1
                st.max_launch_jobs = max(st.max_launch_jobs, len(plan))
                continue
            if inflight:
                if not plan or len(inflight) >= self.max_inflight:
                    retire(block=True)
                continue
            if queue:
                # idle GPU: wait for the next arrival
                wait = queue[0].arrival - clock()
                if wait > 0:
                    time.sleep(min(wait, 0.002))
        retire(block=True)
        torch.cuda.synchronize()
        st.wall_s = time.perf_counter() - t0
        counts = dict(zip(tr.STAT_NAMES, self.stats_buf.cpu().tolist()))
        st.rays = counts["pixels"] + counts["ao_rays"]
        return st

