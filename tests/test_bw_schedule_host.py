"""Host-side checks of the window schedule of the brickwork and circuit passes
(fq_host_bw_schedule, no GPU): every gate is applied once, inside its window,
after every earlier gate on a shared bit (the gates of U in the order of
Eq. (U) and Eq. (unitary)); the number of windows is the minimum that a
brute-force search over the applied-gate sets finds; and the fused first and
last windows start high enough for whole 128-byte lines."""

import ctypes
from collections import deque

import numpy as np
import pytest

MAX_GATES_PER_WINDOW = 8


def _schedule(n, wb, gates, line_bits):
    from paper_2102_05054_amd import _lib
    G = len(gates)
    cap = max(G, 1)
    IntArr = ctypes.c_int * cap
    q = IntArr(*[g[0] for g in gates])
    w = IntArr(*[g[1] for g in gates])
    nwin = ctypes.c_int(-1)
    wb_, wf, wc, order = IntArr(), IntArr(), IntArr(), IntArr()
    st = _lib.lib().fq_host_bw_schedule(n, wb, G, q, w, line_bits, ctypes.byref(nwin), wb_, wf, wc, order)
    assert st == 0, _lib.lib().floquet_last_error()
    wins = [(wb_[j], wf[j], wc[j]) for j in range(nwin.value)]
    return wins, [order[k] for k in range(G)]


def _overlap(a, b):
    return a[0] < b[0] + b[1] and b[0] < a[0] + a[1]


def _check_valid(n, wb, gates, wins, order):
    G = len(gates)
    assert sorted(order) == list(range(G))  # every gate exactly once
    pos = {}
    for j, (b, first, count) in enumerate(wins):
        assert 0 <= b and b + wb <= n
        assert 1 <= count <= MAX_GATES_PER_WINDOW
        for k in range(first, first + count):
            g = order[k]
            q, w = gates[g]
            assert b <= q and q + w <= b + wb  # inside its window
            pos[g] = (j, k)
    assert sum(c for _, _, c in wins) == G
    for j in range(G):
        for i in range(j):
            if _overlap(gates[i], gates[j]):
                assert pos[i] < pos[j]  # acting order on shared bits kept


def _fewest_windows(n, wb, gates):
    """Brute force: breadth-first over the sets of applied gates; a window at
    bit b applies, in acting order, each remaining gate inside it whose
    earlier gates on shared bits are done (at most eight per window)."""
    G = len(gates)
    full = (1 << G) - 1

    def step(done, b):
        taken = 0
        for j in range(G):
            if taken == MAX_GATES_PER_WINDOW:
                break
            q, w = gates[j]
            if done >> j & 1 or q < b or q + w > b + wb:
                continue
            if any(not (done >> i & 1) and _overlap(gates[i], gates[j]) for i in range(j)):
                continue
            done |= 1 << j
            taken += 1
        return done

    dist = {0: 0}
    queue = deque([0])
    while queue:
        s = queue.popleft()
        if s == full:
            return dist[s]
        for b in range(n - wb + 1):
            t = step(s, b)
            if t != s and t not in dist:
                dist[t] = dist[s] + 1
                queue.append(t)
    raise AssertionError("unreachable")


# The two blocks of the complex64 brickwork pass at L = 24 (cut at site 12:
# the right block on tile bits 0..12, the left block on a 2-bit chunk plus
# sites 1..11) and of the complex128 pass at L = 20 (tile bits 0..10; a 2-bit
# chunk plus sites 1..9): (tile bits, gates, fewest windows).
BLOCKS = {
    "L24 right": (13, [(11, 2), (9, 2), (7, 2), (5, 2), (3, 2), (1, 2), (0, 1),
                       (10, 2), (8, 2), (6, 2), (4, 2), (2, 2), (0, 2)], 4),
    "L24 left": (14, [(13, 1), (11, 2), (9, 2), (7, 2), (5, 2), (3, 2),
                      (12, 2), (10, 2), (8, 2), (6, 2), (4, 2), (2, 2)], 4),
    "L20 right c128": (11, [(9, 2), (7, 2), (5, 2), (3, 2), (1, 2), (0, 1),
                            (8, 2), (6, 2), (4, 2), (2, 2), (0, 2)], 4),
    "L20 left c128": (12, [(11, 1), (9, 2), (7, 2), (5, 2), (3, 2),
                           (10, 2), (8, 2), (6, 2), (4, 2), (2, 2)], 3),
}


@pytest.mark.parametrize("name", sorted(BLOCKS))
def test_brickwork_blocks_fewest_windows(name):
    n, gates, expect = BLOCKS[name]
    wins, order = _schedule(n, 4, gates, 3)
    _check_valid(n, 4, gates, wins, order)
    assert len(wins) == expect == _fewest_windows(n, 4, gates)
    # the fused first and last windows read whole 128-byte lines of complex128
    assert wins[0][0] >= 3 and wins[-1][0] >= 3


@pytest.mark.parametrize("seed", range(12))
def test_random_circuits_fewest_windows(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 9))
    wb = int(rng.integers(2, 5))
    G = int(rng.integers(1, 11))
    gates = []
    for _ in range(G):
        w = int(rng.integers(1, 3))
        gates.append((int(rng.integers(0, n - w + 1)), w))
    wins, order = _schedule(n, wb, gates, 4)
    _check_valid(n, wb, gates, wins, order)
    assert len(wins) == _fewest_windows(n, wb, gates)


def test_long_program_keeps_a_valid_greedy_schedule():
    # beyond 64 gates the greedy placement: still every gate once and in order
    rng = np.random.default_rng(7)
    n = 12
    gates = [(int(q), 2) for q in rng.integers(0, n - 1, size=90)]
    wins, order = _schedule(n, 4, gates, 3)
    _check_valid(n, 4, gates, wins, order)


def test_schedule_rejects_bad_gates():
    from paper_2102_05054_amd import _lib
    IntArr = ctypes.c_int * 2
    nwin = ctypes.c_int()
    outs = [IntArr() for _ in range(4)]
    lib = _lib.lib()
    # a gate past the tile's last bit, then a width of 3
    for q, w in (((5, 0), (2, 2)), ((0, 1), (3, 1))):
        st = lib.fq_host_bw_schedule(6, 4, 2, IntArr(*q), IntArr(*w), 3, ctypes.byref(nwin), *outs)
        assert st != 0
    assert lib.fq_host_bw_schedule(6, 7, 0, None, None, 3, ctypes.byref(nwin), None, None, None, None) != 0
    assert lib.fq_host_bw_schedule(6, 4, 0, None, None, 3, ctypes.byref(nwin), None, None, None, None) == 0
    assert nwin.value == 0
