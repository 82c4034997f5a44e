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

    def replay(self, arrival_ns, client, length, release_results: bool = True, keep=None):
        """Real-time replay of a trace in the library.  keep (optional, bool per
        request): results to keep while every other one is released as soon as
        it completes."""
        arrival_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        client = np.ascontiguousarray(client, dtype=np.uint32)
        length = np.ascontiguousarray(length, dtype=np.uint64)
        if keep is not None:
            keep = np.ascontiguousarray(keep, dtype=np.uint8)
            return L.cprng_server_replay_keep(self.s, arrival_ns, client, length, keep)
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


_HIP = None


def copy_result(c) -> np.ndarray:
    """Host copy (uint32 numpy) of a completion's device result (hipMemcpy)."""
    import ctypes
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    n = int(c.length)
    host = np.empty(n, dtype=np.uint32)
    rc = _HIP.hipMemcpy(host.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(c.out), n * 4, 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy of a result failed ({rc})")
    return host


def run_trace(duration_s: float, check_clients: int = 0, oracle_check=None):
    """Replay the serving workload (Poisson 2,000 req/s for duration_s s, sizes
    log-uniform 1 KiB..256 MiB, 10,000 clients, 64 GiB budget, 2 HIP streams);
    every result is released as soon as it completes, except those of
    `check_clients` sampled clients, which are kept and handed to
    oracle_check(client, [host copies of its results in arrival order]) after
    the run (a checker the caller supplies)."""
    import torch
    from .generator import Generator

    arrival, client, length = workloads.serving_trace(duration_s=duration_s)
    gen = Generator(10000, "v0", seed=4)
    srv = Server(gen, n_gpu_streams=2, budget_bytes=64 << 30)
    checked = 0
    try:
        # warm-up: a few requests so the first kernels and tables are built;
        # the streams are put back afterwards, so the trace starts from the seed
        start = gen.get_state()
        srv.replay(np.zeros(8, np.uint64), np.arange(8, dtype=np.uint32), np.full(8, 1 << 20, np.uint64), True)
        torch.cuda.synchronize()
        gen.set_state(start)
        picks = np.unique(client)[:: max(1, np.unique(client).size // max(1, check_clients))][:check_clients] \
            if check_clients else np.zeros(0, np.uint32)
        keep = np.isin(client, picks)
        t0 = time.perf_counter()
        res = srv.replay(arrival, client, length, keep=keep)
        wall = time.perf_counter() - t0
        summary = summarize(res, len(arrival), wall)
        if oracle_check is not None:
            for c in picks.tolist():
                idx = np.nonzero(client == c)[0]
                oracle_check(int(c), [copy_result(res[i]) for i in idx])
                checked += 1
        for i in np.nonzero(keep)[0]:
            srv.release(res[i].out)
    finally:
        srv.close()
        gen.close()
    summary["clients_checked"] = checked
    summary["duration_s"] = duration_s
    return summary


def bench_line(args):
    """JSON line of the serving workload alone (`args.duration` s of arrivals)."""
    summary = run_trace(args.duration)
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
