"""The solve server's scheduler (arena allocator, residency, admission) on a
simulated device: the host-only build of the same C++ code the server runs,
driven by a discrete-event simulation of requests with durations."""
import ctypes
import heapq
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# GPSPCA_SCHED_LIB: a separately built copy (the sanitizer test's instrumented build)
LIB = os.environ.get("GPSPCA_SCHED_LIB") or os.path.join(ROOT, "paper_1312_6182_amd",
                                                         "libgpspca_sched.so")

U64, SZ, I, P = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p
MAXU = (1 << 64) - 1


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        from paper_1312_6182_amd import build
        build.build_sched()
    lib = ctypes.CDLL(LIB)
    sig = {
        "sched_create": (P, [SZ, I]), "sched_destroy": (None, [P]),
        "sched_add_matrix": (None, [P, U64, SZ]), "sched_remove_matrix": (I, [P, U64]),
        "sched_fits_alone": (I, [P, U64, SZ]), "sched_enqueue": (None, [P, U64, U64, SZ]),
        "sched_admit": (I, [P, ctypes.POINTER(U64), ctypes.POINTER(U64), ctypes.POINTER(U64),
                            ctypes.POINTER(U64), ctypes.POINTER(I), ctypes.POINTER(U64), I,
                            ctypes.POINTER(I)]),
        "sched_finish": (None, [P, U64, U64]), "sched_waiting": (SZ, [P]),
        "sched_free_bytes": (SZ, [P]), "sched_arena_bytes": (SZ, [P]),
        "sched_resident_bytes": (SZ, [P]), "sched_evictions": (U64, [P]),
        "sched_matrix_state": (ctypes.c_int64, [P, U64]),
        "sched_used_blocks": (I, [P, ctypes.POINTER(U64), I]),
        "arena_create": (P, [SZ]), "arena_destroy": (None, [P]), "arena_alloc": (U64, [P, SZ]),
        "arena_release": (I, [P, U64]), "arena_free_bytes": (SZ, [P]),
        "arena_largest_free": (SZ, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def used_blocks(L, s):
    buf = (U64 * 8192)()
    k = L.sched_used_blocks(s, buf, 4096)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(k)]


def check_layout(L, s):
    blocks = sorted(used_blocks(L, s))
    size = L.sched_arena_bytes(s)
    for (o1, l1), (o2, _) in zip(blocks, blocks[1:]):
        assert o1 + l1 <= o2
    if blocks:
        assert blocks[-1][0] + blocks[-1][1] <= size
    assert L.sched_free_bytes(s) + sum(b[1] for b in blocks) == size


def admit(L, s):
    req, mat, wso, mo = U64(), U64(), U64(), U64()
    up, ne = I(), I()
    ev = (U64 * 256)()
    ok = L.sched_admit(s, ctypes.byref(req), ctypes.byref(mat), ctypes.byref(wso), ctypes.byref(mo),
                       ctypes.byref(up), ev, 256, ctypes.byref(ne))
    evicted = [ev[i] for i in range(ne.value)]
    if not ok:
        return None, evicted
    return dict(req=req.value, matrix=mat.value, ws_off=wso.value, m_off=mo.value,
                upload=bool(up.value)), evicted


def simulate(L, arena, mats, reqs, slots, max_bypass=8):
    """reqs: list of (arrival, matrix, ws_bytes, duration).  Returns per-request
    (admit time, finish time, upload flag) and the scheduler's eviction count."""
    s = L.sched_create(arena, max_bypass)
    for mid, b in mats.items():
        L.sched_add_matrix(s, mid, b)
    order = sorted(range(len(reqs)), key=lambda r: (reqs[r][0], r))
    ai = 0
    t = 0.0
    running = []   # heap of (end, req, matrix, ws_off)
    log = {}
    while ai < len(order) or running or L.sched_waiting(s):
        nxt = []
        if ai < len(order):
            nxt.append(reqs[order[ai]][0])
        if running:
            nxt.append(running[0][0])
        assert nxt, "waiting requests that can never be admitted"
        t = min(nxt)
        while running and running[0][0] <= t:
            _, r, mid, wso = heapq.heappop(running)
            L.sched_finish(s, mid, wso)
        while ai < len(order) and reqs[order[ai]][0] <= t:
            r = order[ai]
            assert L.sched_fits_alone(s, reqs[r][1], reqs[r][2])
            L.sched_enqueue(s, r, reqs[r][1], reqs[r][2])
            ai += 1
        while len(running) < slots:
            a, evicted = admit(L, s)
            busy = {x[2] for x in running}
            assert not (set(evicted) & busy), "evicted a matrix in use"
            if a is None:
                break
            assert a["matrix"] not in evicted
            assert L.sched_matrix_state(s, a["matrix"]) & 1
            check_layout(L, s)
            r = a["req"]
            log[r] = (t, t + reqs[r][3], a["upload"])
            heapq.heappush(running, (t + reqs[r][3], r, a["matrix"], a["ws_off"]))
    ev = L.sched_evictions(s)
    free = L.sched_free_bytes(s) + L.sched_resident_bytes(s)
    size = L.sched_arena_bytes(s)
    L.sched_destroy(s)
    assert free == size  # everything but resident matrices returned
    return log, ev


def test_arena_random_alloc_free_coalesces(L):
    rng = np.random.default_rng(0)
    size = 1 << 24
    a = L.arena_create(size)
    live = {}
    for step in range(4000):
        if live and (rng.random() < 0.45 or len(live) > 60):
            off = list(live)[rng.integers(len(live))]
            assert L.arena_release(a, off) == 1
            del live[off]
        else:
            b = int(rng.integers(1, 1 << 19))
            off = L.arena_alloc(a, b)
            if off == MAXU:
                assert L.arena_largest_free(a) < (b + 255) // 256 * 256
                continue
            assert off % 256 == 0
            for o, ln in live.items():
                assert off + b <= o or o + ln <= off
            live[off] = b
        assert L.arena_free_bytes(a) <= size
    for off in list(live):
        assert L.arena_release(a, off) == 1
    assert L.arena_free_bytes(a) == size and L.arena_largest_free(a) == size
    assert L.arena_release(a, 12345) == 0
    L.arena_destroy(a)


def test_repeat_requests_upload_once(L):
    mats = {1: 10 << 20}
    reqs = [(0.0, 1, 1 << 20, 1.0), (0.5, 1, 1 << 20, 1.0), (5.0, 1, 1 << 20, 1.0)]
    log, ev = simulate(L, 64 << 20, mats, reqs, slots=4)
    assert [log[r][2] for r in range(3)] == [True, False, False]
    assert log[1][0] == 0.5          # admitted at arrival, overlapping request 0
    assert ev == 0


def test_lru_eviction_of_idle_matrices(L):
    # room for two matrices and a workspace: the third matrix evicts the least
    # recently used idle one
    mats = {1: 20 << 20, 2: 20 << 20, 3: 20 << 20}
    reqs = [(0.0, 1, 1 << 20, 1.0), (2.0, 2, 1 << 20, 1.0), (4.0, 1, 1 << 20, 1.0),
            (6.0, 3, 1 << 20, 1.0), (8.0, 1, 1 << 20, 1.0)]
    log, ev = simulate(L, 45 << 20, mats, reqs, slots=2)
    assert [log[r][2] for r in range(5)] == [True, True, False, True, False]
    assert ev == 1  # matrix 2 (least recently used) made room for 3; matrix 1 stayed


def test_matrix_in_use_is_never_evicted(L):
    mats = {1: 30 << 20, 2: 30 << 20}
    reqs = [(0.0, 1, 1 << 20, 10.0), (1.0, 2, 1 << 20, 1.0)]
    log, ev = simulate(L, 40 << 20, mats, reqs, slots=2)
    assert log[1][0] == 10.0      # waits for request 0 to finish
    assert ev == 1


def test_bypass_is_bounded(L):
    # a large request at the head cannot fit while small ones keep arriving;
    # after max_bypass small admissions nothing passes it
    mats = {1: 8 << 20, 2: 40 << 20}
    reqs = [(0.0, 1, 8 << 20, 2.0), (0.1, 2, 8 << 20, 1.0)]
    reqs += [(0.2 + 0.01 * i, 1, 8 << 20, 2.0) for i in range(20)]
    log, _ = simulate(L, 64 << 20, mats, reqs, slots=4, max_bypass=3)
    big = log[1][0]
    passed = [r for r in range(2, 22) if log[r][0] < big]
    assert len(passed) <= 3
    assert all(log[r][0] >= big for r in range(2, 22) if r not in passed)


def test_no_eviction_when_it_cannot_help(L):
    s = L.sched_create(100 << 20, 8)
    L.sched_add_matrix(s, 1, 30 << 20)
    L.sched_add_matrix(s, 2, 30 << 20)
    L.sched_add_matrix(s, 3, 60 << 20)
    L.sched_enqueue(s, 10, 1, 1 << 20)
    a, _ = admit(L, s)
    L.sched_enqueue(s, 11, 2, 1 << 20)
    b, _ = admit(L, s)
    L.sched_finish(s, 1, a["ws_off"])       # matrix 1 idle, matrix 2 busy
    L.sched_enqueue(s, 12, 3, 20 << 20)     # needs 80 MB: impossible while 2 is busy
    c, evicted = admit(L, s)
    assert c is None and evicted == []
    assert L.sched_matrix_state(s, 1) & 1   # matrix 1 still resident
    assert not L.sched_fits_alone(s, 3, 50 << 20)
    L.sched_destroy(s)


def test_mixed_workload_completes_within_the_arena(L):
    rng = np.random.default_rng(7)
    mats = {}
    reqs = []
    t = 0.0
    for r in range(400):
        if mats and rng.random() < 0.5:
            mid = int(rng.choice(list(mats)))
        else:
            mid = len(mats) + 1
            mats[mid] = int(np.exp(rng.uniform(np.log(1 << 20), np.log(900 << 20))))
        t += rng.exponential(0.02)
        reqs.append((t, mid, int(rng.integers(1 << 16, 64 << 20)), float(rng.exponential(0.1))))
    log, ev = simulate(L, 2 << 30, mats, reqs, slots=6)
    assert len(log) == len(reqs)
    assert ev > 0
    uploads = sum(1 for v in log.values() if v[2])
    assert len(mats) <= uploads < len(reqs)
