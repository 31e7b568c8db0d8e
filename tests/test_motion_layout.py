"""Host-side checks of the motion search's task and LDS layout (no GPU).

The library reports, through ct_motion_layout_query, the LDS layout and the
task list its kernel uses for each search range (the same host/device
functions the kernel calls). These tests check that the tasks cover each of
the (2w + 1)^2 candidates exactly once, that every LDS word a candidate reads
lies inside its copy's written rows, and that the split last pass gives each
of its tasks one lane pair.
"""
import ctypes
import os

import numpy as np
import pytest

BLOCK, PAIRS, MAX_W = 16, 8, 16


@pytest.fixture(scope="module")
def lib():
    from paper_1510_00561_amd import ct
    if not os.path.exists(ct.LIB_PATH):
        from paper_1510_00561_amd import build
        build.build()
    lib = ct._lib()
    lib.ct_motion_layout_query.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int32]
    lib.ct_motion_layout_query.restype = ctypes.c_int
    return lib


def query(lib, w):
    lay = np.zeros(6, np.int32)
    n = lib.ct_motion_layout_query(w, lay.ctypes.data, None, None, 0)
    assert n > 0
    rows = np.zeros(n, np.int32)
    sa = np.zeros(n, np.int32)
    assert lib.ct_motion_layout_query(w, lay.ctypes.data, rows.ctypes.data, sa.ctypes.data, n) == n
    return lay, list(zip(rows.tolist(), sa.tolist()))


@pytest.mark.parametrize("w", range(1, MAX_W + 1))
def test_tasks_cover_every_candidate_once(lib, w):
    _, tasks = query(lib, w)
    seen = []
    for row, sa in tasks:
        seen.append((row, sa))
        if sa + 2 <= 2 * w:
            seen.append((row, sa + 2))
    want = [(r, c) for r in range(2 * w + 1) for c in range(2 * w + 1)]
    assert sorted(seen) == want


@pytest.mark.parametrize("w", range(1, MAX_W + 1))
def test_window_reads_stay_inside(lib, w):
    lay, tasks = query(lib, w)
    rp, odd_off, cur_off, per_wave = (int(v) for v in lay[:4])
    S = BLOCK + 2 * w
    assert per_wave == cur_off + PAIRS * BLOCK
    assert per_wave % 4 == 0 and cur_off % 4 == 0          # 16-byte aligned block rows
    assert odd_off >= S * rp and cur_off >= odd_off + S * rp  # copies do not overlap
    written = S // 2 + 1                                     # pairs per row, pad included
    assert written <= rp
    for row, sa in tasks:
        k0 = sa >> 1
        # rows row .. row + 15 of the window, pairs k0 .. k0 + 8 (second candidate)
        assert row + BLOCK - 1 < S
        assert k0 + PAIRS < written


@pytest.mark.parametrize("w", range(1, MAX_W + 1))
def test_split_pass_lane_pairs(lib, w):
    lay, tasks = query(lib, w)
    nt = len(tasks)
    nfull, tail = divmod(nt, 64)
    assert bool(lay[5]) == (0 < tail <= 32)
    if lay[5]:
        # lanes 2i and 2i + 1 take the two halves of task 64 nfull + i: each
        # of the tail tasks gets exactly one lane pair, and the pairs fit a wave
        owners = {}
        for lane in range(64):
            i = min(lane >> 1, tail - 1)
            if (lane >> 1) < tail:
                owners.setdefault(64 * nfull + i, []).append((lane, lane & 1))
        assert sorted(owners) == list(range(64 * nfull, nt))
        assert all(sorted(h for _, h in v) == [0, 1] for v in owners.values())


def test_query_rejects_bad_ranges(lib):
    lay = np.zeros(6, np.int32)
    assert lib.ct_motion_layout_query(0, lay.ctypes.data, None, None, 0) == -1
    assert lib.ct_motion_layout_query(17, lay.ctypes.data, None, None, 0) == -1
