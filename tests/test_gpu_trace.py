"""MBW_TRACE=1: one JSON line per SMEM launch and per mbw_seed call on stderr, consistent with the
call's result (checked in a child process, since the flag is read once per process).  The launch
lines also show the persistent grid: sized by the work by default (a small batch gets one block per
compute unit), at the occupancy limit with blocks_per_cu = -1."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
import synth, paper_2606_15357_amd as mbw
ref = synth.workload_reference("small_1mbp")
idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
reads = synth.reads_uniform_len(ref, 2000, 50, 400, seed=81)
ctx = mbw.Context(idx)
out = ctx.seed(reads.seq, reads.lengths)
print(out.n_seeds, out.n_pos, out.n_smem_launches, flush=True)
sys.stderr.write("--- occupancy limit\n"); sys.stderr.flush()
ctx.seed(reads.seq, reads.lengths, blocks_per_cu=-1)
""" % ROOT


def test_trace_lines():
    env = dict(os.environ, MBW_TRACE="1")
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    n_seeds, n_pos, launches = (int(x) for x in r.stdout.split())
    first, second = r.stderr.split("--- occupancy limit")
    recs = [json.loads(ln) for ln in first.splitlines() if ln.startswith('{"mbw"')]
    occ = [json.loads(ln) for ln in second.splitlines() if ln.startswith('{"mbw": "smem_launch"')]
    smem = [x for x in recs if x["mbw"] == "smem_launch"]
    seed = [x for x in recs if x["mbw"] == "seed"]
    assert len(seed) == 1 and len(smem) == launches >= 2
    assert seed[0]["seeds"] == n_seeds and seed[0]["positions"] == n_pos
    assert {x["round"] for x in smem} == {1, 2} and all(x["ms"] > 0 for x in smem)
    assert abs(sum(x["ms"] for x in smem) - seed[0]["ms_smem"]) < 1e-2 * max(1.0, seed[0]["ms_smem"])
    # 2,000 reads: far below one block per CU's worth of queries in either round, so every launch
    # has one block per CU; the occupancy limit is a larger multiple of the CU count
    n_cu = smem[0]["blocks"]
    assert all(x["blocks"] == n_cu for x in smem)
    assert len(occ) == len(smem) and all(x["blocks"] > n_cu and x["blocks"] % n_cu == 0 for x in occ)
