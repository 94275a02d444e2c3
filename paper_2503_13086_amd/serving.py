"""Serving loop of progressive training (Sec. IV-B to IV-D) on one GPU.

Images arrive over time.  Each arrival registers its image, appends its new
Gaussians to a field that stays resident in device memory (capacity doubles when
it runs out; Adam moments and per-Gaussian step counters grow with it) and
becomes a job of T_I iterations: Eq. 3-4 weights from the overlap graph, Eq. 5
shares for the local half, an even spread over the other images for the
semi-global half (gs_sched_weights, gs_sched_plan).  Every iteration trains one
image with its Eq. 6-8 learning rate (gs_sched_lr, trained-iteration counts kept
per image).

The loss of an iteration is Eq. 10: w_l1 L1 + w_dssim (1 - SSIM) + w_load L_load
(Eq. 9 on the soft per-pixel count; the paper's weights are 0.47, 0.12, 0.41).

Continuous batching: the engine keeps up to `max_slots` jobs in flight.  Each
engine step takes the next iteration of every active job and runs them as one
batched multi-view step (one gs_preprocess / gs_bin_sort / gs_render_fwd /
gs_loss / gs_render_bwd over all the step's views, then one gs_adam_step whose
per-Gaussian rate is the mean of the rates of the views that see the Gaussian).
An arrival is admitted as soon as a slot is free and its memory estimate fits the
HBM budget; jobs that arrive while others run join the next step.  With
max_slots = 1 the engine is the plain loop: one job at a time, one view per step.

A step renders and differentiates each of its views exactly as a step with that
view alone would on the same field: images and losses are the same bit for bit
and the gradient is the sum of the single-view gradients (up to the order of fp32
atomic additions).

Checkpoint and resume: Engine.save(path) writes the field (parameters, Adam
moments, step counters, capacity), the registered images (cameras, targets,
overlap matrix, trained-iteration counts), the jobs with their plans and
progress, the planning generator's state and the clock to one safetensors file;
Engine.load(path) rebuilds the engine, and run() on the same arrival stream
continues where the saved one stopped (arrivals already registered are skipped,
unfinished jobs resume).  With the ordered backward and a plain loop the resumed
run ends with the same bits as an uninterrupted one.
"""
from __future__ import annotations

import json
import time
from collections import deque
from dataclasses import dataclass, field as dc_field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import gs_sched_weights, gs_sched_plan, gs_sched_lr
from .pipeline import Rasterizer, DEFAULT_LR, n_params


class Field:
    """Resident Gaussian field in the parameter layout of include/gs.h, with Adam
    state, gradient buffer and per-Gaussian step counters of the same capacity."""

    def __init__(self, params: np.ndarray, sh_degree: int, device=0, capacity: int = 0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.sh_degree = sh_degree
        self.n_p = n_params(sh_degree)
        if params.shape[0] != self.n_p:
            raise ValueError(f"expected {self.n_p} parameter rows, got {params.shape[0]}")
        self.n = 0
        self.cap = 0
        self.params = self.m = self.v = self.grad = self.step = None
        self.growths = 0
        self._alloc(max(capacity, params.shape[1], 1))
        self.append(params)

    def _alloc(self, cap: int):
        z = lambda: torch.zeros((self.n_p, cap), dtype=torch.float32, device=self.device)
        new = dict(params=z(), m=z(), v=z(), grad=z(), step=torch.zeros(cap, dtype=torch.int32, device=self.device))
        if self.n:
            for k in ("params", "m", "v", "grad"):
                new[k][:, : self.n].copy_(getattr(self, k)[:, : self.n])
            new["step"][: self.n].copy_(self.step[: self.n])
        for k, t in new.items():
            setattr(self, k, t)
        if self.cap:
            self.growths += 1
        self.cap = cap

    def reserve(self, n_total: int):
        if n_total > self.cap:
            self._alloc(max(2 * self.cap, n_total))

    def append(self, block):
        """Append Gaussians (a [n_p, k] array or device tensor); their Adam moments
        and step counters start at zero."""
        blk = torch.as_tensor(block, dtype=torch.float32).to(self.device)
        if blk.dim() != 2 or blk.shape[0] != self.n_p:
            raise ValueError("block must be [n_params, k]")
        k = blk.shape[1]
        self.reserve(self.n + k)
        a, b = self.n, self.n + k
        self.params[:, a:b].copy_(blk)
        self.m[:, a:b].zero_()
        self.v[:, a:b].zero_()
        self.step[a:b].zero_()
        self.n = b

    def bytes_at(self, n_total: int) -> int:
        cap = self.cap if n_total <= self.cap else max(2 * self.cap, n_total)
        return cap * (4 * 4 * self.n_p + 4)

    def snapshot(self):
        return {k: getattr(self, k)[..., : self.n].clone() for k in ("params", "m", "v", "step")}, self.n

    def restore(self, snap):
        data, n = snap
        self.n = n
        for k, t in data.items():
            getattr(self, k)[..., :n].copy_(t)


@dataclass
class Job:
    image: int
    plan: List[int]
    arrival: float
    admitted: float = 0.0
    done: Optional[float] = None
    next: int = 0
    local_share: Optional[np.ndarray] = None

    @property
    def finished(self) -> bool:
        return self.next >= len(self.plan)


@dataclass
class ServeStats:
    latencies: List[float] = dc_field(default_factory=list)
    makespan: float = 0.0
    steps: int = 0
    iterations: int = 0
    pixels: int = 0
    max_batch: int = 0
    peak_bytes: int = 0
    field_growths: int = 0
    final_n: int = 0

    def summary(self) -> dict:
        lat = np.asarray(self.latencies, np.float64)
        return {"jobs": int(lat.size),
                "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
                "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
                "makespan_s": self.makespan, "steps": self.steps, "iterations": self.iterations,
                "mpix_s": self.pixels / self.makespan / 1e6 if self.makespan > 0 else None,
                "max_batch": self.max_batch, "peak_bytes": self.peak_bytes, "field_growths": self.field_growths,
                "final_gaussians": self.final_n}


class Engine:
    """Continuous-batching trainer over a resident, growing field."""

    def __init__(self, fld: Field, *, max_slots: int = 8, hbm_budget: Optional[int] = None, t_i: int = 200,
                 n_m: int = 10, eta0: float = 1.6e-4, etaf: float = 1.6e-6, t_a: float = 200.0, w_l1: float = 0.8,
                 w_dssim: float = 0.2, w_load: float = 0.0, lr_group: Sequence[float] = DEFAULT_LR,
                 group_mask: int = 1, seed: int = 0, rasterizer=None, autotuner=None):
        if not 1 <= max_slots <= 64:
            raise ValueError("max_slots must be in 1..64 (views per batched launch)")
        self.field = fld
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.t_i, self.n_m = t_i, n_m
        self.eta0, self.etaf, self.t_a = eta0, etaf, t_a
        self.w_l1, self.w_dssim, self.w_load = w_l1, w_dssim, w_load
        self.lr_group = tuple(float(x) for x in lr_group)
        self.group_mask = group_mask
        self.rng = np.random.default_rng(seed)
        self.rz = rasterizer if rasterizer is not None else Rasterizer(fld.device.index or 0)
        # tile edge per step shape (autotune.Autotuner: timed once per field-size bucket,
        # SH degree and multiset of view sizes), or the rasterizer's edge when None
        self.autotuner = autotuner
        self.cams: List[dict] = []
        self.targets: List[torch.Tensor] = []
        self.M = np.zeros((0, 0), np.float64)
        self.trained: List[int] = []
        self.pairs_per_view = None
        self._img = self._dl = None
        self._loss = torch.zeros(64, dtype=torch.float64, device=fld.device)
        self._load = torch.zeros(64, dtype=torch.float64, device=fld.device)
        self.stats = ServeStats()
        self.jobs: List[Job] = []
        self.elapsed = 0.0          # seconds of run() so far (arrival times are measured on this clock)
        self._hyper = dict(max_slots=max_slots, hbm_budget=hbm_budget, t_i=t_i, n_m=n_m, eta0=eta0, etaf=etaf,
                           t_a=t_a, w_l1=w_l1, w_dssim=w_dssim, w_load=w_load, lr_group=list(self.lr_group),
                           group_mask=group_mask)

    # ---- checkpoint / resume ----
    def save(self, path: str) -> None:
        """Write the engine's state to `path` (safetensors; the scalar state as JSON
        metadata).  Call between run() calls (no step in flight)."""
        from safetensors.torch import save_file
        self._sync()
        fld = self.field
        n = fld.n
        t = {"field.params": fld.params[:, :n], "field.m": fld.m[:, :n], "field.v": fld.v[:, :n],
             "field.step": fld.step[:n], "engine.M": torch.as_tensor(self.M)}
        for i, tg in enumerate(self.targets):
            t[f"engine.target.{i}"] = tg
        t = {k: v.detach().to("cpu").contiguous() for k, v in t.items()}
        jobs = [dict(image=j.image, plan=j.plan, arrival=j.arrival, admitted=j.admitted, done=j.done, next=j.next,
                     local_share=None if j.local_share is None else np.asarray(j.local_share).tolist())
                for j in self.jobs]
        cams = [{k: np.asarray(v).tolist() for k, v in c.items()} for c in self.cams]
        meta = dict(format=1, sh_degree=fld.sh_degree, n=n, cap=fld.cap, growths=fld.growths, hyper=self._hyper,
                    cams=cams, trained=[int(x) for x in self.trained], jobs=jobs, elapsed=self.elapsed,
                    pairs_per_view=self.pairs_per_view, rng=self.rng.bit_generator.state,
                    stats=dict(self.stats.__dict__))
        save_file(t, path, metadata={"engine": json.dumps(meta)})

    @classmethod
    def load(cls, path: str, device=0, rasterizer=None, autotuner=None) -> "Engine":
        """An engine in the state Engine.save wrote (the field on `device`)."""
        from safetensors import safe_open
        from safetensors.torch import load_file
        with safe_open(path, framework="pt") as f:
            meta = json.loads(f.metadata()["engine"])
        if meta.get("format") != 1:
            raise ValueError(f"{path}: unknown checkpoint format {meta.get('format')}")
        t = load_file(path)
        fld = Field(t["field.params"].numpy(), meta["sh_degree"], device=device, capacity=meta["cap"])
        fld.m[:, :fld.n].copy_(t["field.m"])
        fld.v[:, :fld.n].copy_(t["field.v"])
        fld.step[:fld.n].copy_(t["field.step"])
        fld.growths = meta["growths"]
        h = dict(meta["hyper"])
        eng = cls(fld, rasterizer=rasterizer, autotuner=autotuner, **h)
        eng.M = t["engine.M"].numpy().astype(np.float64)
        eng.cams = [{k: (np.asarray(v, np.float32) if isinstance(v, list) else np.float32(v) if isinstance(v, float)
                         else v) for k, v in c.items()} for c in meta["cams"]]
        eng.targets = [t[f"engine.target.{i}"].to(fld.device) for i in range(len(eng.cams))]
        eng.trained = [int(x) for x in meta["trained"]]
        eng.jobs = [Job(image=j["image"], plan=[int(x) for x in j["plan"]], arrival=j["arrival"],
                        admitted=j["admitted"], done=j["done"], next=j["next"],
                        local_share=None if j["local_share"] is None else np.asarray(j["local_share"]))
                    for j in meta["jobs"]]
        eng.elapsed = meta["elapsed"]
        eng.pairs_per_view = meta["pairs_per_view"]
        eng.rng.bit_generator.state = meta["rng"]
        for k, v in meta["stats"].items():
            setattr(eng.stats, k, v)
        return eng

    def close(self):
        self.rz.close()

    def _sync(self):
        if self.field.device.type == "cuda":
            torch.cuda.synchronize(self.field.device)

    # ---- registration and admission ----
    def register(self, cam: dict, target: torch.Tensor, overlap_row: Sequence[float], block, arrival: float = 0.0,
                 now: float = 0.0) -> Job:
        """Add an image (overlap_row: its overlap degree with each earlier image),
        append its Gaussians and plan its T_I iterations."""
        i = len(self.cams)
        ov = np.asarray(overlap_row, np.float64).reshape(-1)
        if ov.size != i:
            raise ValueError(f"overlap row of image {i} must have {i} entries")
        M = np.zeros((i + 1, i + 1), np.float64)
        M[:i, :i] = self.M
        M[i, :i] = ov
        M[:i, i] = ov
        self.M = M
        self.field.append(block)
        self.cams.append(dict(cam))
        self.targets.append(torch.as_tensor(target, dtype=torch.float32).reshape(-1).to(self.field.device))
        self.trained.append(0)
        w, _ = gs_sched_weights(self.M, i)
        plan, share = gs_sched_plan(w, self.n_m, self.t_i, self.rng.random(i + 1))
        job = Job(image=i, plan=[int(x) for x in plan], arrival=arrival, admitted=now, local_share=share)
        self.jobs.append(job)
        return job

    def _view_bytes(self, n: int, pixels: int) -> int:
        """Context and image memory of one view of a step: 142 B per Gaussian
        (record, depth, tiles touched, rect, sort keys and values, scan, kept
        counts and emission info, 2D gradient, histograms, split-work lists), 16 B
        per pair (tile ids and record ids, ping-pong), the buffers' 25 %
        over-allocation and 320 KiB of fixed buffers (status and split counters,
        the split lists' floors, small scratch); 100 B per pixel (per-pixel forward
        state, soft count and its gradient, SSIM statistics, image and dL/dimage)."""
        pairs = self.pairs_per_view if self.pairs_per_view is not None else 16 * n
        ctx = int((142 * n + 16 * pairs) * 5 // 4) + 327680
        return ctx + 100 * pixels

    def _resident_bytes(self, n_total: int, extra_targets: int) -> int:
        tgt = sum(t.numel() * 4 for t in self.targets) + extra_targets
        return self.field.bytes_at(n_total) + tgt

    def fits(self, active: List[Job], cam: dict, k_new: int) -> bool:
        """HBM admission: resident field and targets after the append, plus the
        larger of the context memory held now and the working set of a step with
        every active job and the newcomer, within the budget."""
        if self.budget is None:
            return True
        n_total = self.field.n + k_new
        px_new = cam["width"] * cam["height"]
        work = self._view_bytes(n_total, px_new)
        for j in active:
            c = self.cams[j.plan[j.next]] if not j.finished else self.cams[j.image]
            work += self._view_bytes(n_total, c["width"] * c["height"])
        held = self.rz.memory_bytes()
        return self._resident_bytes(n_total, 12 * px_new) + max(work, held) <= self.budget

    def footprint(self) -> int:
        return self._resident_bytes(self.field.n, 0) + self.rz.memory_bytes() + \
            (0 if self._img is None else 2 * self._img.numel() * 4)

    # ---- one batched iteration ----
    def step(self, jobs: List[Job], record: bool = False):
        views = [j.plan[j.next] for j in jobs]
        cams = [self.cams[v] for v in views]
        _, lr = gs_sched_lr(np.asarray(self.trained, np.int64), self.M, self.eta0, self.etaf, self.t_a)
        scales = [float(lr[v]) / self.lr_group[0] for v in views]
        rz, fld = self.rz, self.field
        rz.set_views(cams)
        P3 = 3 * rz.P
        if self._img is None or self._img.numel() < P3:
            self._img = torch.empty(P3, dtype=torch.float32, device=fld.device)
            self._dl = torch.empty(P3, dtype=torch.float32, device=fld.device)
        color, dl = self._img[:P3], self._dl[:P3]
        target = torch.cat([self.targets[v] for v in views]) if len(views) > 1 else self.targets[views[0]]
        if self.autotuner is not None:
            self.autotuner.choose(rz, fld.params, fld.n, fld.sh_degree, cams, target, self.w_l1, self.w_dssim)
        rz.preprocess(fld.params, fld.n, fld.sh_degree)
        K = rz.bin_sort()
        rz.render_fwd(color)
        loss = self._loss[: len(views)]
        rz.loss(color, target, self.w_l1, self.w_dssim, loss, dl)
        if self.w_load != 0.0:
            load = self._load[: len(views)]
            rz.load_balance(self.w_load, load)
            loss = loss + load
        out = None
        if record:
            rz.render_bwd(dl, fld.grad)
            out = {"views": views, "color": [x.clone() for x in rz.image_views(color)], "loss": loss.clone(),
                   "grad": fld.grad[:, : fld.n].clone(), "pairs": K}
            rz.adam_step(fld.grad, fld.m, fld.v, fld.step, self.lr_group, scales, self.group_mask)
        else:   # the same update with the gradient applied as it is formed
            rz.render_bwd_adam(dl, fld.m, fld.v, fld.step, self.lr_group, scales, self.group_mask)
        for j, v in zip(jobs, views):
            self.trained[v] += 1
            j.next += 1
        per_view = K / len(views)
        self.pairs_per_view = per_view if self.pairs_per_view is None else max(per_view, 0.9 * self.pairs_per_view)
        st = self.stats
        st.steps += 1
        st.iterations += len(views)
        st.pixels += rz.P
        st.max_batch = max(st.max_batch, len(views))
        st.peak_bytes = max(st.peak_bytes, self.footprint())
        return out

    # ---- the loop ----
    def run(self, arrivals, targets: Sequence[torch.Tensor], time_scale: float = 1.0,
            on_job_done=None, max_steps: Optional[int] = None) -> ServeStats:
        """Serve a stream.  arrivals: objects with .time (s), .cam, .overlap (with
        the earlier images), .block (new Gaussians); targets: the images as device
        tensors, in arrival order.  Arrival times are multiplied by time_scale and
        measured on the engine's clock (from the start of its first run); a job's
        latency runs from its arrival to the end of the step that completes its
        last iteration.  on_job_done(job) is called as each job completes.  Arrivals
        the engine has already registered are skipped and its unfinished jobs
        continue (a loaded checkpoint resumes).  max_steps: return after this many
        engine steps of this call (then save() and a later run() carry on)."""
        pending = deque(range(len(self.cams), len(arrivals)))
        active: List[Job] = [j for j in self.jobs if not j.finished]
        st = self.stats
        t0 = time.perf_counter() - self.elapsed
        steps0 = st.steps
        while pending or active:
            if max_steps is not None and st.steps - steps0 >= max_steps:
                break
            now = time.perf_counter() - t0
            while pending and len(active) < self.max_slots:
                a = arrivals[pending[0]]
                at = a.time * time_scale
                if at > now or not self.fits(active, a.cam, a.block.shape[1]):
                    break
                pending.popleft()
                active.append(self.register(a.cam, targets[len(self.cams)], a.overlap, a.block, at, now))
            if not active:
                a = arrivals[pending[0]]
                wait = a.time * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                    continue
                raise MemoryError(f"arrival {len(self.cams)} does not fit the HBM budget of {self.budget} B "
                                  "even with no job in flight")
            self.step(active)
            fin = [j for j in active if j.finished]
            if fin:
                self._sync()
                t = time.perf_counter() - t0
                for j in fin:
                    j.done = t
                    st.latencies.append(t - j.arrival)
                    active.remove(j)
                    if on_job_done is not None:
                        on_job_done(j)
        self._sync()
        self.elapsed = time.perf_counter() - t0
        st.makespan = self.elapsed
        st.field_growths = self.field.growths
        st.final_n = self.field.n
        return st
