"""Continuous-batching search server.

Requests (image stacks of uneven image count, frame size and velocity grid)
arrive while others run.  The scheduler

  * admits requests in arrival order while their device footprint fits the
    HBM budget (a request larger than the whole budget fails at once);
  * prepares each admitted request on the device (inputs, likelihood planes,
    candidate and result buffers) as soon as it is admitted;
  * launches prepared requests in arrival order, packing consecutive ones
    into ONE batched search (kb_search_batch: one persistent launch over the
    tiles of all those stacks) while the batch's work stays within
    `batch_work` trajectory-image evaluations (a larger request runs alone,
    so small stacks never wait for a large one that shares their launch),
    each followed by its stacks' final top-k, and keeps up to `max_inflight`
    batches queued on the device so it never idles between them;
  * resolves each request's future when its results are ready and frees its
    memory, which admits the next requests.

A request's result is the same as running it alone (the batched search runs
the single-stack arithmetic per tile).  All device work sits behind an
executor, so the scheduling logic is tested on the CPU with a fake one.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future
from typing import Any, Callable, Optional


@dataclasses.dataclass
class Request:
    """One search problem.  `make` builds the device inputs (img, var, mask) when
    the request is admitted; t, vel, psf are host arrays; k results per pixel
    are kept (k_cand >= k candidates are searched)."""
    rid: int
    shape: tuple            # (n_img, h, w)
    t: Any
    vel: Any
    psf: Any
    k: int
    make: Callable[[], tuple]
    k_cand: Optional[int] = None
    arrival: float = 0.0    # set by submit() unless given


@dataclasses.dataclass
class Done:
    """What a request's future resolves to."""
    rid: int
    result: Any             # executor-specific (device tensors for the GPU executor)
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, executor, budget_bytes: int, max_batch: int = 64,
                 max_inflight: int = 2, poll_s: float = 2e-4, batch_work: float = 2e10):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.batch_work = batch_work
        self.max_inflight = max_inflight
        self.poll_s = poll_s
        self._lock = threading.Condition()
        self._pending = collections.deque()     # (req, future)
        self._ready = []                        # prepared, not launched: (req, fut, handle, t_adm)
        self._inflight = collections.deque()    # (token, [(req, fut, handle, t_adm)])
        self._in_use = 0
        self._peak = 0
        self._stop = False
        self._thread = None
        self.batches = []                       # sizes of launched batches

    # -- client side ---------------------------------------------------------
    def submit(self, req: Request) -> Future:
        fut = Future()
        if not req.arrival:
            req.arrival = time.perf_counter()
        if self.ex.footprint(req) > self.budget:
            fut.set_exception(MemoryError(
                f"request {req.rid} needs {self.ex.footprint(req)} bytes, budget {self.budget}"))
            return fut
        with self._lock:
            self._pending.append((req, fut))
            self._lock.notify()
        return fut

    @property
    def bytes_in_use(self) -> int:
        return self._in_use

    @property
    def peak_bytes(self) -> int:
        return self._peak

    # -- scheduler -----------------------------------------------------------
    def start(self):
        self._thread = threading.Thread(target=self._loop, name="kbmi-serve", daemon=True)
        self._thread.start()
        return self

    def stop(self):
        with self._lock:
            self._stop = True
            self._lock.notify()
        if self._thread is not None:
            self._thread.join()

    def idle(self) -> bool:
        with self._lock:
            return not (self._pending or self._ready or self._inflight)

    def _admit(self):
        """Admit pending requests in order while they fit the budget."""
        admitted = []
        with self._lock:
            while self._pending:
                req, fut = self._pending[0]
                need = self.ex.footprint(req)
                if self._in_use + need > self.budget:
                    break
                self._pending.popleft()
                self._in_use += need
                self._peak = max(self._peak, self._in_use)
                admitted.append((req, fut, need))
        for req, fut, need in admitted:
            t_adm = time.perf_counter()
            try:
                handle = self.ex.prepare(req)
            except Exception as e:               # isolate a failing request
                self._release_bytes(need)
                fut.set_exception(e)
                continue
            self._ready.append((req, fut, handle, t_adm))

    def _release_bytes(self, n):
        with self._lock:
            self._in_use -= n
            self._lock.notify()

    @staticmethod
    def work(req: Request) -> int:
        """Trajectory-image evaluations of a request: N * H * W * V."""
        n, h, w = req.shape
        return int(n) * int(h) * int(w) * len(req.vel)

    def _next_batch(self):
        take, total = 0, 0
        while take < len(self._ready) and take < self.max_batch:
            wk = self.work(self._ready[take][0])
            if take and total + wk > self.batch_work:
                break
            take, total = take + 1, total + wk
        batch, self._ready = self._ready[:take], self._ready[take:]
        return batch

    def _launch(self):
        while self._ready and len(self._inflight) < self.max_inflight:
            batch = self._next_batch()
            try:
                token = self.ex.launch([h for _, _, h, _ in batch])
            except Exception as e:
                # A batch that cannot be launched fails its members only.
                for req, fut, h, _ in batch:
                    self.ex.release(h)
                    self._release_bytes(self.ex.footprint(req))
                    fut.set_exception(e)
                continue
            self.batches.append(len(batch))
            self._inflight.append((token, batch))

    def _complete(self) -> bool:
        progressed = False
        while self._inflight and self.ex.done(self._inflight[0][0]):
            token, batch = self._inflight.popleft()
            t_done = time.perf_counter()
            for req, fut, h, t_adm in batch:
                try:
                    res = self.ex.result(h)
                except Exception as e:
                    fut.set_exception(e)
                else:
                    fut.set_result(Done(req.rid, res, req.arrival, t_adm, t_done))
                self.ex.release(h)
                self._release_bytes(self.ex.footprint(req))
            progressed = True
        return progressed

    def _loop(self):
        while True:
            with self._lock:
                if self._stop and not (self._pending or self._ready or self._inflight):
                    return
            self._admit()
            self._launch()
            if not self._complete():
                with self._lock:
                    if not (self._pending or self._ready or self._inflight) and not self._stop:
                        self._lock.wait(0.05)
                if self._inflight:
                    time.sleep(self.poll_s)


# ---------------------------------------------------------------------------
# Device executor.
# ---------------------------------------------------------------------------

def in_place(k, k_cand, lp=None) -> bool:
    """Whether kb_topk orders the candidate lists in place (plain planes and
    every candidate kept), so a request needs no separate result buffers."""
    return lp is None and k_cand == k


def footprint_bytes(n_img, h, w, n_vel, k, k_cand, lp=None) -> int:
    """Device bytes one request holds while admitted: inputs (img, var, mask),
    float32 planes (+ the 16-bit copy), candidates, results (unless ordered in
    place), workspace."""
    px = h * w
    inputs = n_img * px * 9
    planes = n_img * px * (8 + (4 if lp else 0))
    cand = px * k_cand * 14
    out = 0 if in_place(k, k_cand, lp) else px * k * 14
    # The request's kb_search / kb_topk workspace and its share of a batch's
    # workspace: a 16-byte gather-table entry per (velocity, image slot), the
    # visiting order, the 16-bit scales and counters, each 256-byte rounded,
    # plus the batch's job descriptor.
    r256 = lambda b: (b + 255) // 256 * 256
    stride = (n_img + 15) // 16 * 16
    one = r256(stride * n_vel * 16) + r256(4 * n_vel) + r256(stride * 8) + 256
    ws = 2 * one + 4096
    return inputs + planes + cand + out + ws


class GpuExecutor:
    """Runs requests with libkbmi on one HIP device.  Inputs and planes are
    prepared on a stream of their own; each batch goes to a search stream and
    waits there for its requests' preparation; results stay on the device.
    A batch of at least LARGE_TIE trajectory-image evaluations fills the GPU
    many times over on its own: such batches share the first search stream,
    so two of them never interleave their tiles on the same CUs (their
    working sets evict each other from the L2: 25 x 4096^2 x 4000 FP16
    requests, two outstanding, took 1.13 s each, against 0.77 s alone).
    Smaller batches go round-robin to the other streams, never behind a
    large one."""

    LARGE_TIE = 2.5e11

    def __init__(self, device="cuda:0", lp=None, streams=2):
        import torch
        from . import lib
        self.torch, self.lib = torch, lib
        self.dev = torch.device(device)
        self.lp = lp
        self.prep_stream = torch.cuda.Stream(device=self.dev)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self._next = 0

    def footprint(self, req: Request) -> int:
        n, h, w = req.shape
        kc = req.k_cand or req.k
        return footprint_bytes(n, h, w, len(req.vel), req.k, kc, self.lp)

    def prepare(self, req: Request):
        torch, lib = self.torch, self.lib
        s = self.prep_stream
        with torch.cuda.stream(s):
            img, var, mask = req.make()
            n, h, w = img.shape
            kc = req.k_cand or req.k
            if self.lp is None:
                planes = lib.make_psi_phi(img, var, mask, req.psf)
                src, sc = planes, None
            else:
                planes, src, sc = lib.make_psi_phi(img, var, mask, req.psf, lp=self.lp)
            cand = lib.alloc_candidates(h, w, kc, self.dev)
            # Plain planes with every candidate kept: kb_topk orders the
            # lists in place, so the results are the candidate arrays.
            out = (cand if in_place(req.k, kc, self.lp)
                   else lib.alloc_candidates(h, w, req.k, self.dev))
            ws = lib.alloc_workspace(n, h, w, len(req.vel), self.dev)
            ev = torch.cuda.Event()
            ev.record(s)
        return dict(req=req, img=img, var=var, mask=mask, planes=planes, src=src, scale=sc,
                    cand=cand, out=out, ws=ws, prepared=ev, stream=s)

    def launch(self, handles):
        torch, lib = self.torch, self.lib
        tie = sum(hd["img"].numel() * len(hd["req"].vel) for hd in handles)
        if tie >= self.LARGE_TIE or len(self.streams) == 1:
            s = self.streams[0]
        else:
            s = self.streams[1 + self._next % (len(self.streams) - 1)]
            self._next += 1
        groups = collections.defaultdict(list)      # one batched launch per k_cand
        for hd in handles:
            groups[hd["cand"][0].shape[-1]].append(hd)
        with torch.cuda.stream(s):
            for hd in handles:
                s.wait_event(hd["prepared"])
            for kc, hs in groups.items():
                if len(hs) == 1:
                    # A stack alone: the single-stack search (same per-tile
                    # arithmetic, so the same results) in its fastest order.
                    hd = hs[0]
                    lib.search(hd["src"], hd["req"].t, hd["req"].vel, kc, out=hd["cand"],
                               workspace=hd["ws"], stream=s, lp_scale=hd["scale"])
                else:
                    jobs = [dict(planes=hd["src"], t=hd["req"].t, vel=hd["req"].vel,
                                 out=hd["cand"], lp_scale=hd["scale"]) for hd in hs]
                    lib.search_batch(jobs, kc, stream=s)
                for hd in hs:
                    n = hd["img"].shape[0]
                    rescore = None if self.lp is None else (hd["planes"], hd["req"].t,
                                                            hd["req"].vel, hd["ws"])
                    lib.topk(hd["cand"], hd["req"].k, n, out=hd["out"], stream=s,
                             rescore=rescore)
            ev = torch.cuda.Event()
            ev.record(s)
        for hd in handles:
            hd["stream"] = s
        return ev

    def done(self, token) -> bool:
        return token.query()

    def result(self, handle):
        return handle["out"]

    def release(self, handle):
        # Tensors return to torch's caching allocator once unreferenced; make
        # the allocator aware of the stream that used them (a request whose
        # batch never launched only ran on the preparation stream).
        s = handle["stream"]
        for key in ("img", "var", "mask", "planes", "src", "scale", "ws"):
            t = handle.get(key)
            if t is not None:
                t.record_stream(s)
        for t in (*handle["cand"], *handle["out"]):
            t.record_stream(s)
        handle.clear()
