"""CPU check of the schedule of the batched band march (the flattened D2Q9 march of the
batched step): lanes walk the case's stored order in chunks of B that start on multiples
of 64 nodes; phi and psi go to an LDS ring at padded positions v = (r + 1)(nx + 2) + x + 1
(column -1 of a row formed in the chunk that holds the row's first node, column nx read
from column 0);
iteration i writes chunk i and then updates chunk i - lag.

The lag and ring-size rules below are the ones the library applies when it sets a
batch's launch shape.  Replaying the schedule node by node shows, for every width and
band, that (1) each stencil input an update reads holds the right node's value at the
time of the read (the lag suffices and nothing newer has wrapped onto it), and (2) no
ring slot written in iteration i + 1 is read in iteration i, so one barrier per
iteration suffices.
"""
import pytest


def flat_lag(nx, B):
    need = (nx + 1 + B - 1) // B
    return 1 if need <= 1 else (3 if need <= 3 else 0)


def flat_ring_cap(nx, B, lag):
    span = (lag + 2) * B
    need = span + 2 * (span // nx + 1) + 2 * nx + 3
    cap = 1
    while cap <= need:
        cap <<= 1
    return cap


D2Q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def replay(nx, y0, y1, B):
    lag = flat_lag(nx, B)
    assert lag > 0
    cap = flat_ring_cap(nx, B, lag)
    P = nx + 2
    e_begin, e_end = (y0 - 1) * nx, (y1 + 1) * nx
    e_first = e_begin - (e_begin % 64)          # Python's % is a floor modulus
    nchunk = -(-(e_end - e_first) // B)
    ring = {}

    def node(e):
        return e // nx, e % nx                  # row (may be -1) and column

    def writes(i):
        out = []
        if i >= nchunk:
            return out
        for lane in range(B):
            e = e_first + i * B + lane
            if not (e_begin <= e < e_end):
                continue
            r, x = node(e)
            v = (r + 1) * P + x + 1
            out.append((v, (r, x)))
            if x == 0:                           # column -1: image of column nx - 1
                out.append((v - 1, (r, -1)))
        return out

    def reads(i):
        out = []
        k = i - lag
        if k < 0 or k >= nchunk:
            return out
        for lane in range(B):
            e = e_first + k * B + lane
            if not (e_begin <= e < e_end):
                continue
            r, x = node(e)
            if not (y0 <= r < y1):
                continue
            vu = (r + 1) * P + x + 1
            for cx, cy in D2Q9:
                s = vu + cx + P * cy
                xn = x + cx
                if cx > 0 and x == nx - 1:
                    s -= nx
                    xn = 0
                out.append((s, (r + cy, xn)))
        return out

    nupd = 0
    for i in range(nchunk + lag):
        for v, lab in writes(i):
            ring[v % cap] = lab
        rd = reads(i)
        for s, lab in rd:
            assert ring.get(s % cap) == lab, (nx, y0, y1, B, i, s, lab, ring.get(s % cap))
        nupd += len(rd) // 9
        later = {v % cap for v, _ in writes(i + 1)}
        assert not later & {s % cap for s, _ in rd}, (nx, y0, y1, B, i)
    assert nupd == (y1 - y0) * nx                # every node of the band updated once
    return lag, cap


@pytest.mark.parametrize("B", [256, 512, 1024])
@pytest.mark.parametrize("nx", [1, 2, 3, 5, 17, 63, 64, 65, 127, 200, 255, 256, 257, 383, 500, 511, 512, 767, 1023])
def test_band_schedule_reads_the_right_nodes(nx, B):
    if flat_lag(nx, B) == 0:
        pytest.skip("rows too wide for the band march with this many lanes")
    for y0, y1 in ((0, 9), (3, 7), (0, 1), (8, 9), (2, 3)):
        replay(nx, y0, y1, B)


def test_band_ring_sizes_of_the_common_shapes():
    """The lag and ring sizes the batched step uses for the widths of the 512-case batch
    (64..512): one chunk of lag with 1024 lanes, and a ring of 4096 entries up to
    width 511 (8192 beyond: 64 KiB of LDS in FP32)."""
    for nx in (64, 100, 257, 500):
        assert flat_lag(nx, 1024) == 1 and flat_ring_cap(nx, 1024, 1) == 4096
    assert flat_ring_cap(512, 1024, 1) == 8192
    assert flat_lag(511, 512) == 1 and flat_lag(512, 512) == 3
    assert flat_ring_cap(200, 512, 1) == 2048 and flat_ring_cap(511, 512, 1) == 4096
