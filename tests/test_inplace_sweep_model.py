"""Model (CPU) of the hydro strip sweep written over its input.

A segment [j0, j1) of a line walks chunks of C cells: its prologue reads
cells j0-2 .. j0; each chunk first reads cell p+1 for its cells p (p <= j1),
then, after barriers, updates cell p-1 (p > j0), reading that cell just
before writing it.  Segments run in any order relative to each other.  A
read is at risk when another segment writes the cell, or when the segment
itself wrote it earlier.  The in-place kernel sends a read of cell x to the
copy saved before the sweep exactly when x lies outside [j0, j1) and a
transmissive end does not clamp it onto the segment's own cells; the copy
holds, for every boundary b = s * seg, the cells b-2 .. b+1 (boundary
applied).  The tests check that every at-risk read goes to the copy, and
that the copy slot it takes holds the cell it asks for."""
import itertools

import pytest

PERIODIC, TRANSMISSIVE = 0, 1


def wrap(x, n, bc):
    if bc == PERIODIC:
        return x % n
    return min(max(x, 0), n - 1)


def segment_accesses(j0, j1, C):
    """(kind, cell) of one segment in program order; cells unwrapped."""
    acc = [("r", j0 - 2), ("r", j0 - 1), ("r", j0)]
    c0 = j0
    while c0 <= j1:
        ps = [p for p in range(c0, c0 + C) if p <= j1]
        acc += [("r", p + 1) for p in ps]
        for p in ps:
            if p > j0:
                acc += [("r", p - 1), ("w", p - 1)]
        c0 += C
    return acc


def halo_slot(x, j0, j1, seg, nsg):
    """The kernel's (boundary, slot) for a redirected read of cell x."""
    s0 = j0 // seg
    if x < j0:
        return s0, x - (j0 - 2)
    return (0 if s0 + 1 == nsg else s0 + 1), 2 + (x - j1)


def check(n, seg, C, bc):
    nsg = (n + seg - 1) // seg
    segs = [(s * seg, min(s * seg + seg, n)) for s in range(nsg)]
    writer = {}
    for s, (j0, j1) in enumerate(segs):
        for kind, x in segment_accesses(j0, j1, C):
            if kind == "w":
                assert 0 <= x < n and writer.setdefault(x, s) == s, "each cell has one writer"
    assert sorted(writer) == list(range(n))
    for s, (j0, j1) in enumerate(segs):
        written = set()
        for kind, x in segment_accesses(j0, j1, C):
            w = wrap(x, n, bc)
            if kind == "w":
                written.add(w)
                continue
            at_risk = writer[w] != s or w in written
            redirected = (x < j0 or x >= j1) and (bc == PERIODIC or not j0 <= w < j1)
            if at_risk:
                assert redirected, (n, seg, C, bc, s, x)
            if redirected:
                sb, c = halo_slot(x, j0, j1, seg, nsg)
                assert 0 <= sb < nsg and 0 <= c < 4, (n, seg, s, x, sb, c)
                assert wrap(sb * seg - 2 + c, n, bc) == w, (n, seg, s, x, sb, c)


@pytest.mark.parametrize("bc", [PERIODIC, TRANSMISSIVE])
def test_every_at_risk_read_comes_from_the_saved_copy(bc):
    for n, seg, C in itertools.product([1, 2, 3, 5, 8, 17, 64, 100, 191, 383], [1, 2, 3, 7, 15, 63, 191, 400],
                                       [1, 4, 64]):
        check(n, min(seg, n) if seg > n else seg, C, bc)


def test_the_model_sees_the_hazards():
    """Without the copy, a periodic line split into segments has reads of
    cells other segments write, and one segment wrapping onto itself reads
    its own first cells after writing them."""
    def hazards(n, seg, C, bc):
        nsg = (n + seg - 1) // seg
        segs = [(s * seg, min(s * seg + seg, n)) for s in range(nsg)]
        writer = {x: s for s, (j0, j1) in enumerate(segs) for x in range(j0, j1)}
        out = []
        for s, (j0, j1) in enumerate(segs):
            written = set()
            for kind, x in segment_accesses(j0, j1, C):
                w = wrap(x, n, bc)
                if kind == "w":
                    written.add(w)
                elif writer[w] != s or w in written:
                    out.append((s, x))
        return out
    assert hazards(64, 16, 4, PERIODIC)
    assert (0, 64) in hazards(64, 64, 4, PERIODIC)          # one segment: cell 0 read again after its update
    assert hazards(64, 64, 4, TRANSMISSIVE) == []           # clamped ends read own cells before writing them
    assert (0, 2) in hazards(2, 1, 1, TRANSMISSIVE)         # a clamp onto the next segment's cell
