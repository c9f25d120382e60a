"""The LDS-ring schedule of the strip sweeps (the hydro sweeps' default
kernels), checked on the CPU: a model of every ring-slot access per stage
and wave of one segment, with the kernel's barriers, must order every pair
of accesses to one slot by different waves where one of them writes.  The
rings hold C + 2 cells (slot = (cell - j0 + 2) mod (C + 2)); lane group q
of a chunk at c0 owns the cell p = c0 + q of its W lines, and q runs on
wave q W / 64 (W = 64 lines: one wave per q; W = 1: 64 values of q per
wave, in program order).  The model follows the kernel's
stages: prologue (three primitive states and the conserved state of j0,
then the first plus face by wave 0), then per chunk: (1) the primitive and
conserved state of p + 1, (2) slopes and
trace of p from p - 1, p, p + 1 and its plus face, (3) the left state
(plus face of p - 1) and then, with no barrier between, the flux at
p - 1/2 into that slot, (4) the update of p - 1 from the fluxes in the
slots of p - 1 and p - 2 and the conserved state of p - 1 from its slot
of the conserved-state ring (a third ring of C + 2 slots)."""
import itertools

import pytest


def schedule(C, W, j0, j1, prologue_barrier=True):
    """Accesses (epoch, wave, ring, slot, is_write) of one segment [j0, j1)."""
    RW = C + 2
    slot = lambda cell: (cell - j0 + 2) % RW
    wave = lambda q: q * W // 64
    acc, ep = [], 0

    def barrier():
        nonlocal ep
        ep += 1

    for k in range(3):                     # prologue: cells j0-2 .. j0
        acc.append((ep, wave(k % C), "w", slot(j0 - 2 + k), True))
        if k == 2:                         # the conserved state of cell j0
            acc.append((ep, wave(k % C), "u", slot(j0), True))
    barrier()
    for c in (j0 - 2, j0 - 1, j0):
        acc.append((ep, 0, "w", slot(c), False))
    acc.append((ep, 0, "f", slot(j0 - 1), True))
    if prologue_barrier:
        barrier()
    for c0 in range(j0, j1 + 1, C):
        waves = [(q, c0 + q) for q in range(C) if c0 + q <= j1]
        for q, p in waves:
            acc.append((ep, wave(q), "w", slot(p + 1), True))
            acc.append((ep, wave(q), "u", slot(p + 1), True))
        barrier()
        for q, p in waves:
            for c in (p - 1, p, p + 1):
                acc.append((ep, wave(q), "w", slot(c), False))
            acc.append((ep, wave(q), "f", slot(p), True))
        barrier()
        for q, p in waves:
            acc.append((ep, wave(q), "f", slot(p - 1), False))
        for q, p in waves:
            acc.append((ep, wave(q), "f", slot(p - 1), True))
        barrier()
        for q, p in waves:
            if p > j0:
                acc.append((ep, wave(q), "f", slot(p - 1), False))
                acc.append((ep, wave(q), "f", slot(p - 2), False))
                acc.append((ep, wave(q), "u", slot(p - 1), False))
        # no barrier before the next chunk's stage 1
    return acc


def races(acc):
    out = []
    by_key = {}
    for a in acc:
        by_key.setdefault((a[0], a[2], a[3]), []).append(a)
    for group in by_key.values():
        for a, b in itertools.combinations(group, 2):
            if a[1] != b[1] and (a[4] or b[4]):
                out.append((a, b))
    return out


# the kernels' shapes: y strips of 64 lines x 2, 4 or 8 rows and of 32 x 8,
# 16 x 16 and 8 x 32 (a wave on 2, 4 or 8 rows of its tile); x strips of one
# line x 64, 128 or 256 cells, and of 4 lines x 64 cells (the x items of the
# one-launch batch step: a wave holds 16 cells of each of the 4 lines) and
# of 2 lines x 32 cells in one wave
SHAPES = [(2, 64), (4, 64), (8, 64), (8, 32), (16, 16), (32, 8), (64, 1), (128, 1), (256, 1), (64, 4), (32, 2)]


@pytest.mark.parametrize("C,W", SHAPES)
@pytest.mark.parametrize("seg", [1, 3, 7, 15, 16, 19, 63, 127, 191, 255])
def test_strip_schedule_has_no_lds_race(C, W, seg):
    assert races(schedule(C, W, 10, 10 + seg)) == []


@pytest.mark.parametrize("C,W", [(2, 64), (4, 64), (8, 64), (8, 32), (16, 16), (32, 8), (128, 1), (256, 1)])
def test_without_the_prologue_barrier_multiwave_strips_race(C, W):
    # the first chunk's cell j0 + C takes the slot of cell j0 - 2, which
    # wave 0 reads in the prologue
    r = races(schedule(C, W, 0, 300, prologue_barrier=False))
    assert r and all(a[2] == b[2] == "w" for a, b in r)


def test_one_wave_strips_need_no_prologue_barrier():
    # a one-wave x strip runs its accesses in program order
    assert races(schedule(64, 1, 0, 191, prologue_barrier=False)) == []
