"""The work queues of the one-launch batch step, checked on the CPU with a
model of their protocol.  Before the step the grids are dealt to the XCDs
(rank by cells, largest first, ties by index; snake order over the ranks).
Per XCD one atomic cursor hands out the x items of that XCD's grids (bands
of 4 rows x 191-cell segments) before its y items (64 columns x seg rows);
a workgroup only draws from its own XCD (the hardware deals workgroups
round robin) and takes nothing on an XCD index not below the XCD count; a
finished x item adds one to its grid's counter; a y item polls its grid's
counter, at most `limit` times, until it holds the grid's x item count,
and gives up (status bit 0, its work skipped) otherwise; the last
workgroup out sets status bit 1 if an XCD's items were not all taken.

The model runs P workgroups as discrete events with random item durations
and checks, for any P: the deal balances the cells; the decode of the item
index (grid, band, segment / tile) on each XCD covers every cell of every
grid once; every item of a grid runs on its XCD; every y item starts after
all x items of its grid finished; no y item waits longer than the longest
x item (the x items it awaits are held by running workgroups); nothing
gives up with the kernel's poll limit; with the test mode (awaited count
+ 1) every y item gives up and every workgroup still exits; with fewer
workgroups than XCDs, status bit 1 reports the XCDs that ran none."""
import heapq
import random

import pytest

from paper_1710_08774_amd import inputs

XSEG, XROWS, NXCD = 191, 4, 8


def x_items(nx, ny):
    return -(-ny // XROWS) * -(-nx // XSEG)


def y_items(nx, ny, seg):
    return -(-nx // 64) * -(-ny // seg)


def deal(sizes, nxcd):
    """XCD of every grid: snake order over the ranks by cells."""
    out = []
    for g, (nx, ny) in enumerate(sizes):
        c = nx * ny
        r = sum(1 for h, (a, b) in enumerate(sizes) if a * b > c or (a * b == c and h < g))
        p = r % (2 * nxcd)
        out.append(p if p < nxcd else 2 * nxcd - 1 - p)
    return out


def decode(sizes, segs, xcd, k, it):
    """(kind, grid, cells) of item `it` of XCD k, as the kernel derives it:
    a cursor over the per-grid counts of the grids dealt to k, then
    band/segment (x) or tile (y)."""
    mine = [g for g in range(len(sizes)) if xcd[g] == k]
    nxi = sum(x_items(*sizes[g]) for g in mine)
    kind, local = ("x", it) if it < nxi else ("y", it - nxi)
    for g in mine:
        nx, ny = sizes[g]
        n = x_items(nx, ny) if kind == "x" else y_items(nx, ny, segs[g])
        if local < n:
            break
        local -= n
    else:
        raise AssertionError("item past the end")
    if kind == "x":
        nsg = -(-nx // XSEG)
        j, i0 = (local // nsg) * XROWS, (local % nsg) * XSEG
        cells = {(i, jj) for jj in range(j, min(j + XROWS, ny)) for i in range(i0, min(i0 + XSEG, nx))}
    else:
        ntx = -(-nx // 64)
        i0, j0 = (local % ntx) * 64, (local // ntx) * segs[g]
        cells = {(i, j) for j in range(j0, min(j0 + segs[g], ny)) for i in range(i0, min(i0 + 64, nx))}
    return kind, g, cells


def totals(sizes, segs, xcd, k):
    mine = [g for g in range(len(sizes)) if xcd[g] == k]
    return sum(x_items(*sizes[g]) for g in mine) + sum(y_items(*sizes[g], segs[g]) for g in mine)


def simulate(sizes, segs, P, seed, nxcd=NXCD, limit=10**9, extra=0, poll=1.0, hw_xcds=NXCD):
    """Event simulation; workgroup w runs on XCD w mod hw_xcds.  Returns the
    per-item log {(k, it): [start, end, kind, grid, gave_up, poll_start,
    polls, xcd of the workgroup]} and the status."""
    rng = random.Random(seed)
    xcd = deal(sizes, nxcd)
    tot = [totals(sizes, segs, xcd, k) for k in range(nxcd)]
    nxi = [sum(x_items(*sizes[g]) for g in range(len(sizes)) if xcd[g] == k) for k in range(nxcd)]
    need = [x_items(nx, ny) for nx, ny in sizes]
    cnt = [0] * len(sizes)
    cursor = [0] * nxcd
    status = 0
    log = {}
    ev, order = [], 0

    def push(t, w, act, key=None):
        nonlocal order
        heapq.heappush(ev, (t, order, w, act, key))
        order += 1

    for w in range(P):
        push(rng.random() * 3, w, "take")
    exited = 0
    while ev:
        t, _, w, act, key = heapq.heappop(ev)
        k = w % hw_xcds
        if act == "take":
            if k >= nxcd:
                exited += 1
                continue
            it, cursor[k] = cursor[k], cursor[k] + 1
            if it >= tot[k]:
                exited += 1
                continue
            kind, g, _ = decode(sizes, segs, xcd, k, it)
            key = (k, it)
            if kind == "x":
                log[key] = [t, None, "x", g, False, t, 0, k]
                push(t + rng.uniform(5, 40), w, "xdone", key)
            else:
                log[key] = [t, None, "y", g, False, t, 0, k]
                push(t, w, "poll", key)
        elif act == "xdone":
            cnt[log[key][3]] += 1
            log[key][1] = t
            push(t, w, "take")
        elif act == "poll":
            rec = log[key]
            g = rec[3]
            if cnt[g] >= need[g] + extra:
                rec[0] = t
                push(t + rng.uniform(5, 40), w, "ydone", key)
            elif rec[6] >= limit:
                status |= 1
                rec[4] = True
                rec[1] = t
                push(t, w, "take")
            else:
                rec[6] += 1
                push(t + poll, w, "poll", key)
        elif act == "ydone":
            log[key][1] = t
            push(t, w, "take")
    assert exited == P, "a workgroup did not exit"
    for k in range(nxcd):
        if cursor[k] < tot[k]:
            status |= 2
    return log, status, xcd, tot


SIZES = [(64, 64), (1, 1), (300, 5), (191, 4), (192, 3), (5, 300), (1024, 37), (65, 129), (383, 8),
         (200, 200), (17, 33), (700, 2), (2, 700), (128, 128), (96, 80), (1, 64), (64, 1), (500, 11)]
SEGS = [15, 15, 3, 1, 7, 15, 63, 15, 2, 31, 15, 7, 15, 15, 3, 15, 15, 15]


def test_deal_balances_the_batched_workload():
    sizes = inputs.batch_sizes(512)
    xcd = deal(sizes, NXCD)
    per = [sum(nx * ny for (nx, ny), k in zip(sizes, xcd) if k == q) for q in range(NXCD)]
    assert (max(per) - min(per)) / (sum(per) / NXCD) < 0.01       # 0.8%
    assert sorted(set(xcd)) == list(range(NXCD))
    # one XCD: everything on it
    assert set(deal(sizes[:20], 1)) == {0}


def test_item_decode_covers_every_cell_once_on_its_xcd():
    xcd = deal(SIZES, NXCD)
    seen = {(kind, g): set() for kind in "xy" for g in range(len(SIZES))}
    for k in range(NXCD):
        for it in range(totals(SIZES, SEGS, xcd, k)):
            kind, g, cells = decode(SIZES, SEGS, xcd, k, it)
            assert xcd[g] == k and cells, (kind, g, it)
            assert not (seen[(kind, g)] & cells)
            seen[(kind, g)] |= cells
    for g, (nx, ny) in enumerate(SIZES):
        every = {(i, j) for i in range(nx) for j in range(ny)}
        assert seen[("x", g)] == every and seen[("y", g)] == every


@pytest.mark.parametrize("P", [8, 9, 16, 64, 1024])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_y_items_wait_only_for_running_x_items(P, seed):
    log, status, xcd, tot = simulate(SIZES, SEGS, P, seed)
    assert status == 0 and len(log) == sum(tot)
    xend, longest_x = {}, 0.0
    for rec in log.values():
        assert rec[7] == xcd[rec[3]]                          # every item on its grid's XCD
        if rec[2] == "x":
            xend[rec[3]] = max(xend.get(rec[3], 0.0), rec[1])
            longest_x = max(longest_x, rec[1] - rec[0])
    for rec in log.values():
        if rec[2] == "y":
            assert not rec[4]
            assert rec[0] >= xend[rec[3]]                     # after every x item of its grid
            assert rec[0] - rec[5] <= longest_x + 1.0         # waited at most one x item (+ a poll)


def test_one_workgroup_per_xcd_never_waits():
    log, status, _, _ = simulate(SIZES, SEGS, NXCD, 3)
    assert status == 0
    assert all(rec[6] == 0 for rec in log.values() if rec[2] == "y")


def test_fewer_xcds_than_the_hardware_has():
    """A device with fewer XCDs than workgroup XCD indices: workgroups on
    the extra indices take nothing, the rest do every item."""
    log, status, _, tot = simulate(SIZES, SEGS, 64, 4, nxcd=3)
    assert status == 0 and len(log) == sum(tot)


@pytest.mark.parametrize("P", [8, 64])
def test_give_up_mode_sets_status_and_drains(P):
    """awaited count + 1 (the test mode): every y item gives up after its
    polls, and every workgroup still takes its final ticket and exits."""
    log, status, _, _ = simulate(SIZES, SEGS, P, 7, limit=64, extra=1)
    assert status & 1
    ys = [rec for rec in log.values() if rec[2] == "y"]
    assert ys and all(rec[4] and rec[6] == 64 for rec in ys)


def test_an_xcd_without_workgroups_is_reported():
    log, status, xcd, tot = simulate(SIZES, SEGS, 5, 1)       # XCDs 5..7 run no workgroup
    assert status == 2
    assert all(rec[7] < 5 for rec in log.values())
