"""Index lifetime: contexts and servers keep the index they were created on.  Freeing the index
while a context or a server with queued requests is alive defers the release: the context still
seeds correctly, the server's queued requests still come back equal to the oracle's, and the index
is released when the last user is freed or closed."""
import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle

mbw = pytest.importorskip("paper_2606_15357_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    ref = synth.workload_reference("small_1mbp")
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    return ref, ox


def test_context_keeps_its_index(small):
    ref, ox = small
    reads = synth.reads_fixed(ref, 3000, 150, False, seed=91)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    ctx = mbw.Context(idx)
    idx.free()                                  # deferred: the context still uses it
    s, p = ctx.seed(reads.seq, reads.lengths).download()
    compare_with_oracle(s, p, ox.seed(reads.seq, reads.offsets))
    ctx.free()                                  # the last user: the index is released here


def test_server_keeps_its_index_with_queued_work(small):
    ref, ox = small
    reqs = [synth.reads_fixed(ref, 800 + 50 * q, 150, False, seed=100 + q) for q in range(24)]
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    srv = mbw.Server(idx, n_workers=2, max_batch_reads=4000, max_batch_bases=800_000)
    ts = [srv.submit(r.seq, r.lengths) for r in reqs]
    idx.free()                                  # while requests are queued and running
    for r, t in zip(reqs, ts):
        s, p, _ = srv.wait(t)
        compare_with_oracle(s, p, ox.seed(r.seq, r.offsets))
    # more work after the free
    t = srv.submit(reqs[0].seq, reqs[0].lengths)
    s, p, _ = srv.wait(t)
    compare_with_oracle(s, p, ox.seed(reqs[0].seq, reqs[0].offsets))
    srv.close()                                 # the last user: the index is released here
