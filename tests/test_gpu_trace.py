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
sys.stderr.write("--- deferred\n"); sys.stderr.flush()
out = ctx.seed(reads.seq, reads.lengths, unique_defer=1)
print(out.n_seeds, out.n_pos, out.n_smem_launches, flush=True)
""" % ROOT


def test_trace_lines():
    env = dict(os.environ, MBW_TRACE="1")
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.split("\n")
    n_seeds, n_pos, launches = (int(x) for x in lines[0].split())
    d_seeds, d_pos, d_launches = (int(x) for x in lines[1].split())
    first, rest = r.stderr.split("--- occupancy limit")
    second, third = rest.split("--- deferred")
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
    assert {x["kind"] for x in smem + occ} == {"smem"}
    # deferred unique matches: round 1 of the staged bin alternates the SMEM kernel (kind "defer")
    # and the continuation kernel ("unique"), starting and ending with the former unless the last
    # continuation pass leaves no read; the unstaged bin and round 2 stay "smem"
    dl = [json.loads(ln) for ln in third.splitlines() if ln.startswith('{"mbw": "smem_launch"')]
    assert (d_seeds, d_pos) == (n_seeds, n_pos) and len(dl) == d_launches
    kinds = [x["kind"] for x in dl if x["round"] == 1 and x["staged"]]
    assert kinds[0] == "defer" and "unique" in kinds and kinds.count("defer") >= 2
    assert all(a != b for a, b in zip(kinds, kinds[1:]))
    assert all(x["kind"] == "smem" for x in dl if x["round"] == 2 or not x["staged"])
