"""Brute-force statements of the definitions (tiny inputs only), used to pin the oracle.

Everything here works on Python strings over '$ACGT' ('$' sorts before 'A' in ASCII, matching the
paper's order $ < A < C < G < T) and recomputes each quantity by direct enumeration: no suffix
array search, no FM-index, nothing shared with the oracle's code.
"""
from __future__ import annotations

COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def revcomp(p: str) -> str:
    return "".join(COMP.get(ch, ch) for ch in reversed(p))


def text_of(ref: str) -> str:
    """T = R . revcomp(R) . $"""
    return ref + revcomp(ref) + "$"


def bs_text_of(ref: str) -> str:
    conv = ref.replace("C", "T") + ref.replace("G", "A")
    return conv + revcomp(conv) + "$"


def suffix_array(T: str):
    return sorted(range(len(T)), key=lambda i: T[i:])


def bwt(T: str, SA):
    return "".join(T[i - 1] if i > 0 else "$" for i in SA)


def occ(T: str, P: str) -> int:
    """occ(P) = |{i : T[i, i+|P|) = P}| by scanning every start."""
    m = len(P)
    return sum(1 for i in range(len(T) - m + 1) if T[i:i + m] == P)


def lo(T: str, P: str) -> int:
    """lo(P) = |{i : T[i, n) < P}| by comparing every suffix."""
    return sum(1 for i in range(len(T)) if T[i:] < P)


def ds_interval(T: str, P: str):
    return lo(T, P), lo(T, revcomp(P)), occ(T, P)


def smems(T: str, P: str, l: int, c: int):
    """All (l,c)-SMEMs of P: enumerate every (l,c)-match [i,j) (length >= l, occ >= c) and keep
    those contained in no other match.  Returns sorted [(i, j, (lo, lo_rc, occ))]."""
    m = len(P)
    matches = []
    for i in range(m):
        for j in range(i + l, m + 1):
            sub = P[i:j]
            if "N" in sub:
                continue
            if occ(T, sub) >= c:
                matches.append((i, j))
    out = []
    for (i, j) in matches:
        if not any((a <= i and j <= b) and (a, b) != (i, j) for (a, b) in matches):
            out.append((i, j, ds_interval(T, P[i:j])))
    return sorted(out)


def positions(T: str, P: str):
    m = len(P)
    return sorted(i for i in range(len(T) - m + 1) if T[i:i + m] == P)


def seeds_two_rounds(T: str, P: str, l: int = 19, c: int = 1, reseed_len: int = 38, reseed_occ: int = 10):
    """Two seeding rounds: round-1 SMEMs, then for each with length >= reseed_len and occ <=
    reseed_occ the (floor(len/2), occ+1)-SMEMs of that substring; union without duplicates."""
    r1 = smems(T, P, l, c)
    out = {(i, j): iv for (i, j, iv) in r1}
    for (i, j, iv) in r1:
        if j - i >= reseed_len and iv[2] <= reseed_occ:
            for (a, b, iv2) in smems(T, P[i:j], (j - i) // 2, iv[2] + 1):
                out[(i + a, i + b)] = iv2
    return sorted((i, j, iv) for (i, j), iv in out.items())
