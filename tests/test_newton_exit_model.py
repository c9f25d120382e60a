"""Model of the Riemann solver's early stop (CPU): a wave of lanes each
iterates its own map N from its own p0; after a step K >= 5 the wave stops
when every lane has p_K == p_{K-m} for some m <= 6 (from p_{K-m} on that
lane's iterates repeat with period m), and every lane must get exactly its
n-th iterate.  The maps below are arbitrary functions on
a small set, so every pattern (fixed points, 2-cycles, longer cycles,
transients of any length) occurs, and the result is compared with plain
iteration."""
import itertools
import math
import random


def plain(N, p, n):
    for _ in range(n):
        p = N(p)
    return p


HIST = 6         # earlier iterates each new one is compared with (NEWTON_HIST)
TEST_FROM = 5    # first step after which the wave tests (NEWTON_TEST_FROM)


def early_wave(maps, p0s, n):
    """The device loop's logic for one wave: every lane steps until, after a
    step k in [TEST_FROM, n), every lane's newest iterate equals one of its
    last HIST; then each lane picks its n-th iterate from its cycle."""
    hs = [[p] for p in p0s]
    for k in range(1, n + 1):
        for N, h in zip(maps, hs):
            h.append(N(h[k - 1]))
        if TEST_FROM <= k < n:
            if all(any(h[k] == h[k - m] for m in range(1, min(HIST, k) + 1)) for h in hs):
                out = []
                for h in hs:
                    r = h[k]
                    for m in range(min(HIST, k), 0, -1):
                        if h[k] == h[k - m]:
                            r = h[k - m + (n - k) % m]
                    out.append(r)
                return out, k
    return [h[n] for h in hs], n


def early(N, p, n):
    return early_wave([N], [p], n)[0][0]


def test_every_map_on_four_points():
    pts = [1.0, 2.0, 3.0, 4.0]
    for images in itertools.product(pts, repeat=len(pts)):
        table = dict(zip(pts, images))
        for p0 in pts:
            for n in range(0, 12):
                assert early(table.__getitem__, p0, n) == plain(table.__getitem__, p0, n), (images, p0, n)


def test_random_maps_with_long_transients():
    rng = random.Random(1710)
    for _ in range(2000):
        m = rng.randint(1, 30)
        pts = [float(k + 1) for k in range(m)]
        table = {p: rng.choice(pts) for p in pts}
        p0 = rng.choice(pts)
        for n in (0, 1, 2, 3, 7, 10, 11, 40):
            assert early(table.__getitem__, p0, n) == plain(table.__getitem__, p0, n)


def test_newton_on_a_float_root_stops_early():
    """Newton for x^2 = 2 in binary64 reaches a repeat well before 10 steps."""
    N = lambda p: p - (p * p - 2.0) / (2.0 * p)
    assert early(N, 1.0, 10) == plain(N, 1.0, 10)
    steps = 0
    h = [1.0]
    while h[-1] not in h[-7:-1]:
        h.append(N(h[-1]))
        steps += 1
    assert steps < 10


def test_waves_of_random_maps():
    rng = random.Random(7741)
    for _ in range(300):
        lanes = rng.randint(1, 64)
        maps, p0s = [], []
        for _ in range(lanes):
            m = rng.randint(1, 12)
            pts = [float(k + 1) for k in range(m)]
            table = {p: rng.choice(pts) for p in pts}
            maps.append(table.__getitem__)
            p0s.append(rng.choice(pts))
        for n in (10, 6, 12):
            got, _ = early_wave(maps, p0s, n)
            assert got == [plain(N, p, n) for N, p in zip(maps, p0s)]
