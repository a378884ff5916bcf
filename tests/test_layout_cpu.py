"""CPU check of the GPU state layout and neighbour indexing.

Mirrors, step by step, the index arithmetic of the layer kernels (segment
decoding, tile offsets, low-bit rank tables) and verifies on small N and
every tile width that (1) the (layer, segment, lane) -> position map is a
bijection onto [0, 2^N) and equals the colexicographic rank inside each
layer, and (2) every neighbour index the kernel forms points at the true
Hamming neighbour (m xor 2^u) in layer n -+ 1, and stays inside the vector.
"""
import math

import pytest


def C(n, k):
    return math.comb(n, k) if 0 <= k <= n else 0


def tile_off(b, Tb, q):
    off, i, k = 0, 0, 0
    while Tb:
        if Tb & 1:
            i += 1
            off += C(b + k, q + i)
        Tb >>= 1
        k += 1
    return off


def layer_args(N, b, n):
    H = N - b
    qlo, qhi = max(0, n - H), min(b, n)
    seg = []
    acc = 0
    for q in range(qlo, qhi + 1):
        seg.append(acc)
        acc += C(H, n - q)
    seg.append(acc)
    return qlo, qhi, seg, acc


def decode(N, b, n, g, qlo, qhi, seg):
    H = N - b
    qi = 0
    while qlo + qi < qhi and g >= seg[qi + 1]:
        qi += 1
    q = qlo + qi
    r = g - seg[qi]
    h = n - q
    Tb, top = 0, H
    for i in range(h, 0, -1):
        c = top - 1
        while C(c, i) > r:
            c -= 1
        Tb |= 1 << c
        r -= C(c, i)
        top = c
    return q, Tb


def colex_rank(m):
    r, i = 0, 0
    p = 0
    while m:
        if m & 1:
            i += 1
            r += C(p, i)
        m >>= 1
        p += 1
    return r


@pytest.mark.parametrize("N,b", [(1, 1), (2, 1), (3, 2), (5, 5), (6, 3), (7, 4), (8, 1), (9, 5), (10, 10),
                                 (11, 4), (12, 6), (13, 7), (14, 10), (12, 12)])
def test_layout_and_neighbours(N, b):
    H = N - b
    lo_unrank = []
    lo_rank = [0] * (1 << b)
    lo_qstart = []
    for q in range(b + 1):
        lo_qstart.append(len(lo_unrank))
        r = 0
        for L in range(1 << b):
            if bin(L).count("1") == q:
                lo_unrank.append(L)
                lo_rank[L] = r
                r += 1
    layer_off = [0]
    for n in range(N + 1):
        layer_off.append(layer_off[-1] + C(N, n))
    pos_of = {}
    for n in range(N + 1):
        qlo, qhi, seg, groups = layer_args(N, b, n)
        for g in range(groups):
            q, Tb = decode(N, b, n, g, qlo, qhi, seg)
            assert bin(Tb).count("1") == n - q and Tb < (1 << H)
            self_off = layer_off[n] + tile_off(b, Tb, q)
            for t in range(C(b, q)):
                L = lo_unrank[lo_qstart[q] + t]
                m = (Tb << b) | L
                pos = self_off + t
                assert pos == layer_off[n] + colex_rank(m)
                assert m not in pos_of
                pos_of[m] = pos
    assert sorted(pos_of.values()) == list(range(1 << N))
    # neighbour indices exactly as the layer kernel forms them
    for m, pos in pos_of.items():
        n = bin(m).count("1")
        Tb, L = m >> b, m & ((1 << b) - 1)
        q = bin(L).count("1")
        t = pos - layer_off[n] - tile_off(b, Tb, q)
        for k in range(H):
            bit = 1 << k
            if Tb & bit:
                idx = layer_off[n - 1] + tile_off(b, Tb ^ bit, q) + t
                assert idx == pos_of[m ^ (bit << b)]
            elif n < N:
                idx = layer_off[n + 1] + tile_off(b, Tb | bit, q) + t
                assert idx == pos_of[m | (bit << b)]
        offDlo = layer_off[n - 1] + tile_off(b, Tb, q - 1) if q >= 1 else 0
        offUlo = layer_off[n + 1] + tile_off(b, Tb, q + 1) if (q < b and n < N) else 0
        for l in range(b):
            bit = 1 << l
            busy = bool(L & bit)
            idx = (offDlo if busy else offUlo) + lo_rank[L ^ bit]
            assert 0 <= idx < (1 << N)
            assert idx == pos_of[m ^ bit]
