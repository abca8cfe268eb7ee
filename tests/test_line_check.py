"""The CPU checker of resident occurrence lines (mbw_helpers.check_line_table) on lines encoded
here from the oracle's BWT by the documented layout, with the device copies replaced by host
reads: it accepts a correct table and rejects each planted mistake (a flipped plane bit, a wrong
header, sub-checkpoint or superblock entry, a bit set past n), so that its pass at 3.1 Gbp on
the GPU means something."""
import ctypes

import numpy as np
import pytest

import mbw_helpers
import oracle


def encode(ox, sh):
    """Lines (bytes) and superblock table of the oracle's BWT, by the documented layout."""
    b = ox.bwt().astype(np.int64)
    codes = np.where(b == 0, 0, b - 1)                  # $ stored as A
    n = codes.size
    nl = (n + 383) // 384
    pad = np.zeros(nl * 384, np.int64)
    pad[:n] = codes
    valid = np.zeros(nl * 384, bool)
    valid[:n] = True
    rows = pad.reshape(nl, 6, 64)
    ok = valid.reshape(nl, 6, 64)
    w = np.uint64(1) << np.arange(64, dtype=np.uint64)
    lo = ((rows & 1).astype(np.uint64) * w).sum(axis=2, dtype=np.uint64)
    hi = ((rows >> 1).astype(np.uint64) * w).sum(axis=2, dtype=np.uint64)
    cnt = np.stack([((rows == c) & ok).sum(axis=2) for c in range(4)], axis=2)   # nl x 6 x 4
    per_line = cnt.sum(axis=1)                                                    # nl x 4
    u32 = np.zeros((nl, 32), np.uint32)
    u64 = u32.view(np.uint64)
    nsb = ((nl - 1) >> sh) + 1
    sbt = np.zeros((nsb, 8), np.uint64)
    before = np.concatenate([np.zeros((1, 4), np.int64), np.cumsum(per_line, axis=0)])
    for L in range(nl):
        s0 = (L >> sh) << sh
        u32[L, 0:3] = before[L, :3] - before[s0, :3]
        sub = np.cumsum(cnt[L, :, :3], axis=0)
        for bb in range(1, 6):
            word = int(sub[bb - 1, 0]) | int(sub[bb - 1, 1]) << 9 | int(sub[bb - 1, 2]) << 18
            if bb == 1:
                u32[L, 3] = word
            else:
                u32[L, 4 + bb - 2] = word
        u64[L, 4::2] = lo[L]
        u64[L, 5::2] = hi[L]
    for sb in range(nsb):
        t = before[sb << sh]
        sbt[sb, :4] = t
        for c in range(4):
            sbt[sb, 4 + c] = t[c + 1:].sum()
    return u32, sbt, n


class HostIndex:
    def __init__(self, u32, sbt, n, C, sh):
        self.u32, self.sbt = np.ascontiguousarray(u32), np.ascontiguousarray(sbt)
        self._info = dict(n=n, n_lines=u32.shape[0], sb_lines_log2=sh, n_superblocks=sbt.shape[0],
                          C=[int(x) for x in C[:5]])

    def info(self):
        return self._info

    def device_arrays(self):
        return self.u32.ctypes.data, 0, 0

    def superblock_table(self):
        return self.sbt.ctypes.data


@pytest.fixture
def host_reads(monkeypatch):
    def read(ptr, nbytes):
        return np.frombuffer((ctypes.c_char * int(nbytes)).from_address(int(ptr)), np.uint8).copy()
    monkeypatch.setattr(mbw_helpers, "device_to_host", read)


@pytest.fixture(scope="module")
def table():
    rng = np.random.default_rng(11)
    R = rng.integers(0, 4, 3000).astype(np.uint8)
    ox = oracle.OracleIndex(R)
    return encode(ox, 2), ox.C()


def test_accepts_a_correct_table(host_reads, table):
    (u32, sbt, n), C = table
    assert u32.shape[0] > 4 * 3 and sbt.shape[0] >= 4      # several superblocks of 4 lines
    mbw_helpers.check_line_table(HostIndex(u32, sbt, n, C, 2), log=lambda *a: None)


@pytest.mark.parametrize("mistake", ["plane_bit", "header", "subcheckpoint", "superblock", "suffix_sum", "past_n"])
def test_rejects_planted_mistakes(host_reads, table, mistake):
    (u32, sbt, n), C = table
    u32, sbt = u32.copy(), sbt.copy()
    u64 = u32.view(np.uint64)
    L = 7
    if mistake == "plane_bit":
        u64[L, 4 + 2 * 3] ^= np.uint64(1) << np.uint64(17)
    elif mistake == "header":
        u32[L, 1] += 1
    elif mistake == "subcheckpoint":
        u32[L, 5] += 1 << 9
    elif mistake == "superblock":
        sbt[2, 3] += 1
    elif mistake == "suffix_sum":
        sbt[1, 4] += 1
    elif mistake == "past_n":
        last = u32.shape[0] - 1
        r = n - last * 384                      # rows of the last line
        assert r < 384
        blk, bit = r // 64, r % 64
        u64[last, 4 + 2 * blk] |= np.uint64(1) << np.uint64(bit)
    with pytest.raises(AssertionError):
        mbw_helpers.check_line_table(HostIndex(u32, sbt, n, C, 2), log=lambda *a: None)
