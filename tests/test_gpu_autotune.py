"""GPU tests of the autotuner and its JSON cache, through the C ABI.

Each case runs in two child processes that share one $CPRNG_TUNE_CACHE file:
the first tunes (cprng_autotune / cprng_autotune_ragged), the second is a fresh
process whose fresh handles must find the tuned entries in that file.  In both,
the configuration each call will use is read back (cprng_resolved_tuning*),
and the outputs of the call are compared bit for bit with the oracle
generating the same streams from the seed: tuning leaves the streams where
they were, and every configuration the tuner may pick produces the same words.

Shapes: V0 stream-major (1,024 x 256); V2 (Algorithm 4) interleaved (4,096
streams x 64: four tiles of 1,024); batched uneven V1 (Listing 1, 48 streams
with runs of up to 4e4 outputs: several chunks each), V2 (three groups of 32)
and V0 (40 streams).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, os, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import torch
from oracle import oracle as O
from paper_1112_5239_amd import generator as G

mode = sys.argv[1]
tune = mode == "tune"
res = {}

def check_rows(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{what}: first mismatch at {bad[0].tolist()}"

# V0 stream-major
g = G.Generator(1024, "v0", seed=0)
if tune:
    g.autotune(256)
res["gen_v0"] = g.resolved_tuning(256)
got = G.as_u32(g.generate(256))
want, _ = O.generate(0, O.seed(0, 0, 0, 1024), 256)
check_rows(got, want, "v0 stream-major")
g.close()

# V2 interleaved (4 tiles of 1,024 streams)
g = G.Generator(4096, "v2", seed=1, interleaved=True)
if tune:
    g.autotune(64)
res["gen_v2_ilv"] = g.resolved_tuning(64)
got = G.as_u32(g.generate(64))
st = O.seed(2, 1, 0, 4096)
want, _ = O.generate(2, st, 64, comb=O.comb_tables(32))
check_rows(got.T.copy(), want, "v2 interleaved")
got2 = G.as_u32(g.generate(64))                       # continuation
want2, _ = O.generate(2, st, 64, comb=O.comb_tables(32))
check_rows(got2.T.copy(), want2, "v2 interleaved, second call")
g.close()

def ragged(name, ov, ns, lengths, sigma, group=0):
    g = G.Generator(ns, name, seed=sigma, group=group)
    total = int(lengths.sum())
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    if tune:
        g.autotune_ragged(lengths, out=out)
    cfg = g.resolved_tuning_ragged(lengths)
    got = G.as_u32(g.generate_ragged(lengths, out=out))
    st = O.seed(ov, sigma, 0, ns)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    if group:
        combs = O.comb_tables(group)
        for gi in range(ns // group):
            rows = slice(gi * group, (gi + 1) * group)
            sub = st[rows].copy()
            L = int(lengths[gi * group])
            want, _ = O.generate(ov, sub, L, comb=combs)
            st[rows] = sub
            for j in range(group):
                s = gi * group + j
                check_rows(got[offs[s]:offs[s] + L], want[j], f"{name} group {gi} stream {j}")
    else:
        for s in range(ns):
            sub = st[s:s + 1].copy()
            L = int(lengths[s])
            want, _ = O.generate(ov, sub, L)
            st[s:s + 1] = sub
            check_rows(got[offs[s]:offs[s] + L], want[0], f"{name} stream {s}")
    assert np.array_equal(g.get_state(), st), f"{name}: end states differ"
    g.close()
    return cfg

rng = np.random.default_rng(7)
res["ragged_v1"] = ragged("v1", 1, 48, rng.integers(0, 40000, size=48).astype(np.uint64), 2)
gl = np.array([30000, 0, 7001], dtype=np.uint64)
res["ragged_v2"] = ragged("v2", 2, 96, np.repeat(gl, 32), 2, group=32)
res["ragged_v0"] = ragged("v0", 0, 40, rng.integers(0, 50000, size=40).astype(np.uint64), 2)
print("RESULT " + json.dumps(res), flush=True)
'''


def _child(mode, cache):
    env = dict(os.environ, CPRNG_TUNE_CACHE=cache)
    print(f"[autotune] child: {mode}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, mode, ROOT], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, f"{mode} child failed:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_autotune_cache_round_trip_and_parity(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    cache = str(tmp_path / "tune.json")
    tuned = _child("tune", cache)
    for k, v in tuned.items():
        assert v["source"] == "autotuned", f"{k}: the tuned entry is not used ({v})"
    with open(cache) as f:
        table = json.load(f)                       # the file is valid JSON
    keys = list(table)
    assert any("/gen/v0/ns2^10/n2^8" in k for k in keys), keys
    assert any("/gen/v2/ilv/ns2^12/n2^6" in k for k in keys), keys
    assert sum("/ragged/v" in k for k in keys) == 3, keys
    for entry in table.values():
        assert set(entry) == {"block", "unroll", "store", "chunk", "waves", "slots", "exchange"}
    # a fresh process reads the file and uses the same configurations
    used = _child("use", cache)
    assert used == tuned
    # the interleaved pick is an interleaved kernel: the per-lane dword
    # kernel (the default at this stream count), the tiles or the quad lanes
    assert tuned["gen_v2_ilv"]["store"] in (5, 9, 10, 11, 12)
    assert tuned["ragged_v1"]["streams_per_lane"] in (1, 2, 4)
    assert tuned["ragged_v1"]["unroll"] in (32, 64, 128)
