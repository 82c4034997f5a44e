"""Serving-loop driver: replays a request trace through the native server.

The real-time loop (arrivals, admission by the HBM budget, continuous
batching on several HIP streams, completion polling) runs in the library
(cprng_server_replay); this module only prepares the trace and summarises the
completions.
"""
import time

import numpy as np

from . import _lib as L
from . import workloads


class Server:
    """One server over a V0 Generator (which must outlive it)."""

    def __init__(self, gen, n_gpu_streams: int = 2, budget_bytes: int = 64 << 30, max_batch: int = 1024):
        self.gen = gen
        self.s = L.cprng_server_create(gen.h, n_gpu_streams, budget_bytes, max_batch)

    def close(self):
        if getattr(self, "s", None):
            L.cprng_server_destroy(self.s)
            self.s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, client: int, length: int, tag: int, t_submit_ns: int = 0):
        L.cprng_server_submit(self.s, client, length, tag, t_submit_ns)

    def poll(self, max_done: int = 256):
        return L.cprng_server_poll(self.s, max_done)

    def release(self, out: int):
        L.cprng_server_release(self.s, out)

    def stats(self):
        return L.cprng_server_stats(self.s)

    def replay(self, arrival_ns, client, length, release_results: bool = True):
        arrival_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        client = np.ascontiguousarray(client, dtype=np.uint32)
        length = np.ascontiguousarray(length, dtype=np.uint64)
        return L.cprng_server_replay(self.s, arrival_ns, client, length, release_results)


def summarize(res, count: int, wall_s: float):
    lat = np.array([(res[i].t_done_ns - res[i].t_submit_ns) for i in range(count)], dtype=np.float64) / 1e6
    qwait = np.array([(res[i].t_admit_ns - res[i].t_submit_ns) for i in range(count)], dtype=np.float64) / 1e6
    numbers = float(sum(res[i].length for i in range(count)))
    status = {int(res[i].status) for i in range(count)}
    return {
        "requests": count,
        "numbers": int(numbers),
        "wall_s": round(wall_s, 3),
        "gnumbers_per_s": round(numbers / wall_s / 1e9, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "max": round(float(lat.max()), 4), "mean": round(float(lat.mean()), 4)},
        "admission_wait_ms": {"p50": round(float(np.percentile(qwait, 50)), 4),
                              "p99": round(float(np.percentile(qwait, 99)), 4)},
        "statuses": sorted(status),
    }


def bench_line(args):
    """JSON line of the serving workload: Poisson arrivals at 2,000 req/s for
    `args.duration` s, sizes log-uniform 1 KiB..256 MiB, 10,000 clients, 64 GiB
    result budget; each result is released as soon as it completes."""
    import torch
    from .generator import Generator

    arrival, client, length = workloads.serving_trace(duration_s=args.duration)
    gen = Generator(10000, "v0", seed=4)
    srv = Server(gen, n_gpu_streams=2, budget_bytes=64 << 30)
    try:
        # warm-up: a few requests so the first kernels and tables are built
        srv.replay(np.zeros(8, np.uint64), np.arange(8, dtype=np.uint32),
                   np.full(8, 1 << 20, np.uint64), True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.replay(arrival, client, length, True)
        wall = time.perf_counter() - t0
        summary = summarize(res, len(arrival), wall)
    finally:
        srv.close()
        gen.close()
    return {
        "metric": "serving: aggregate Gnumbers/s with p50/p99 request latency",
        "value": summary["gnumbers_per_s"],
        "unit": "Gnumbers/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u32",
        "data": "synthetic",
        "latency_ms": summary["latency_ms"],
        "admission_wait_ms": summary["admission_wait_ms"],
        "config": {"workload": f"serving: Poisson 2000 req/s for {args.duration:g} s, sizes log-uniform "
                               "1 KiB..256 MiB of uint32, 10000 resident client streams (V0, seed 4), "
                               "64 GiB result budget, 2 HIP streams",
                   "requests": summary["requests"], "numbers": summary["numbers"], "wall_s": summary["wall_s"]},
        "statuses": summary["statuses"],
    }
