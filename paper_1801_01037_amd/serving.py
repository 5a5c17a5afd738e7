"""Continuous-batching serving loop over the C ABI.

Requests (a gate list, a qubit count and a dtype) arrive over time. The
server keeps admitted states resident in device memory and advances all of
them together:

  * admission: arrived requests are admitted in arrival order while their
    state (2^n amplitudes of 8 or 16 bytes) fits the device-memory budget;
    an admitted request gets a state on its dtype's stream and a plan (its
    circuit fused into tile passes, uploaded once);
  * step: every active circuit of a dtype advances by up to `chunk` passes
    in one batched launch sequence (sv_batch_run); complex64 and complex128
    batches run on their own streams and overlap on the device, and each
    dtype starts its next step as soon as its own step has finished;
  * while steps run, newly arrived requests are admitted and planned on the
    host, and they join their dtype's next step; finished circuits leave and
    free their memory.

Latency of a request = completion time - arrival time (host clock). The
scheduler is plain Python; every amplitude update runs in libsv's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

import paper_1801_01037_amd as sv


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    n: int
    dtype: int
    gates: np.ndarray
    # filled in by the server
    t_admit: float = -1.0
    t_done: float = -1.0
    state: object = None
    plan: int = 0
    passes: int = 0
    next_pass: int = 0
    result: np.ndarray | None = None
    norm: float = float("nan")

    @property
    def nbytes(self) -> int:
        return (1 << self.n) * (8 if self.dtype == sv.SV_C64 else 16)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Server:
    """Continuous-batching executor of circuits on one GPU."""

    def __init__(self, budget_bytes: int | None = None, reserve_bytes: int = 16 << 30,
                 chunk: int = 8, keep_results: bool = False, batch_config=None,
                 persist_tiles: int = 0, solo_tiles: int = 2048):
        import torch
        self.torch = torch
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = max(0, free - reserve_bytes)
        self.budget = budget_bytes
        self.chunk = chunk
        self.keep_results = keep_results
        self.streams = {dt: torch.cuda.Stream() for dt in (sv.SV_C64, sv.SV_C128)}
        self.batches = {dt: sv.sv_batch_create(dt, s.cuda_stream) for dt, s in self.streams.items()}
        if batch_config:
            for dt, (bpc, tpt) in batch_config.items():
                sv.sv_batch_config(self.batches[dt], bpc, tpt)
        # Paths of each step's batch besides the levels: small circuits whole in
        # the persistent launch (off by default: no gain measured here), large
        # ones (2048 tiles per pass and more) pass by pass on a third stream
        # (+12 % saturated throughput, p99 -11 % on the default workload).
        for b in self.batches.values():
            sv.sv_batch_persist(b, persist_tiles)
            sv.sv_batch_solo(b, solo_tiles)
        self.in_use = 0

    def close(self):
        for b in self.batches.values():
            sv.sv_batch_destroy(b)
        self.batches = {}

    # -- admission ----------------------------------------------------------
    def _admit(self, r: Request, now: float):
        st = sv.StateVector(r.n, r.dtype, stream=self.streams[r.dtype])
        r.state = st
        r.plan = sv.sv_plan_create(st.handle, r.gates)
        r.passes = sv.sv_plan_passes(r.plan)
        r.t_admit = now
        self.in_use += r.nbytes

    def _release(self, r: Request):
        if self.keep_results:
            r.result = r.state.numpy()
        r.norm = r.state.norm()
        sv.sv_plan_destroy(r.plan)
        r.plan = 0
        r.state.close()
        r.state = None
        self.in_use -= r.nbytes

    # -- the loop -----------------------------------------------------------
    def run(self, requests: list[Request]) -> dict:
        torch = self.torch
        for r in requests:
            if r.nbytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.nbytes} bytes, over the budget")
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque[Request] = collections.deque()
        active = {sv.SV_C64: [], sv.SV_C128: []}
        done: list[Request] = []
        steps = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731

        def admit_arrived():
            now = clock()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting and self.in_use + waiting[0].nbytes <= self.budget:
                r = waiting.popleft()
                self._admit(r, clock())
                active[r.dtype].append(r)

        # Each dtype steps on its own stream, independently: when a dtype's
        # step has finished on the device, its circuits are retired and its
        # next step is launched at once (with the requests admitted
        # meanwhile), whether or not the other dtype's step is still running.
        inflight = {sv.SV_C64: None, sv.SV_C128: None}   # (event, circuits, pass counts)

        def retire(dt):
            ev, rs, count = inflight[dt]
            inflight[dt] = None
            finished = set()
            for r, c in zip(rs, count):
                r.next_pass += c
                if r.next_pass >= r.passes:
                    r.t_done = clock()
                    self._release(r)
                    done.append(r)
                    finished.add(id(r))
            active[dt] = [r for r in active[dt] if id(r) not in finished]

        def launch(dt):
            rs = list(active[dt])
            plans = [r.plan for r in rs]
            first = [r.next_pass for r in rs]
            count = [min(self.chunk, r.passes - r.next_pass) for r in rs]
            self.streams[dt].wait_stream(torch.cuda.current_stream())
            sv.sv_batch_run(self.batches[dt], plans, first, count)
            ev = torch.cuda.Event()
            ev.record(self.streams[dt])
            inflight[dt] = (ev, rs, count)

        dtypes = (sv.SV_C64, sv.SV_C128)
        while pending or waiting or any(active.values()) or any(inflight.values()):
            admit_arrived()
            progressed = False
            for dt in dtypes:
                if inflight[dt] is not None:
                    if not inflight[dt][0].query():
                        continue
                    retire(dt)
                    progressed = True
                if active[dt]:
                    launch(dt)
                    steps += 1
                    progressed = True
            if progressed:
                continue
            if not any(inflight.values()):
                # nothing on the device: wait for the next arrival
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - clock()))
                continue
            # Steps in flight: admit arrivals meanwhile, check again shortly.
            time.sleep(2e-4)
        elapsed = clock()
        lat = np.array([r.latency for r in done])
        gates = int(sum(len(r.gates) for r in done))
        return {
            "requests": len(done),
            "elapsed_s": elapsed,
            "steps": steps,
            "throughput_rps": len(done) / elapsed if elapsed > 0 else 0.0,
            "gates_per_s": gates / elapsed if elapsed > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
        }


def poisson_requests(rate: float, count: int, seed: int, n_lo: int = 12, n_hi: int = 28,
                     d_lo: int = 10, d_hi: int = 100) -> list[Request]:
    """Seeded Poisson stream: n ~ U{n_lo..n_hi}, depth ~ U{d_lo..d_hi}, dtype
    complex64 or complex128 with probability one half, layered random circuits."""
    import qcircuits as qc
    arrivals = qc.poisson_arrivals(rate, count, qc.derive_seed(seed, 1 << 20))
    specs = qc.batch_specs(seed, count, n_lo, n_hi, d_lo, d_hi)
    out = []
    for i, ((n, d, gseed), t) in enumerate(zip(specs, arrivals)):
        dt = sv.SV_C64 if (gseed >> 7) & 1 else sv.SV_C128
        out.append(Request(i, float(t), n, dt, qc.layer_circuit(n, d, gseed)))
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serving sweep over Poisson arrival rates")
    ap.add_argument("--rates", default="5,20,100,500,5000")
    ap.add_argument("--arrivals", type=int, default=200)
    ap.add_argument("--n-lo", type=int, default=12)
    ap.add_argument("--n-hi", type=int, default=28)
    ap.add_argument("--chunk", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    for rate in [float(x) for x in a.rates.split(",")]:
        reqs = poisson_requests(rate, a.arrivals, a.seed, a.n_lo, a.n_hi)
        srv = Server(chunk=a.chunk)
        try:
            stats = srv.run(reqs)
        finally:
            srv.close()
        stats["offered_rps"] = rate
        print(json.dumps(stats), flush=True)


if __name__ == "__main__":
    main()
