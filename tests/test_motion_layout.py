"""Host-side checks of the motion search's task and LDS layout (no GPU).

The kernel hands each lane tasks of two candidates (dy, sc) and (dy, sc + 2)
with sc = dx + w and sc mod 4 in {0, 1}, tpr tasks per window row, and lays
out the window as even- and odd-column pair copies followed by the block.
These tests restate that arithmetic for every supported search range and
check that the tasks cover each of the (2w + 1)^2 candidates exactly once,
that the split last pass stays within one lane pair per task, and that every
LDS word a candidate reads lies inside its copy's written rows.
"""
import pytest

BLOCK, PAIRS, MAX_W = 16, 8, 16


def layout(w):
    S = BLOCK + 2 * w
    tuned = w == 8
    rp = S // 2 + 1 + (4 if tuned else 0)
    odd_off = S * rp + (1 if tuned else 0)
    cur_off = (odd_off + S * rp + 3) & ~3
    return S, rp, odd_off, cur_off, cur_off + PAIRS * BLOCK


def tasks(w):
    side = 2 * w + 1
    tpr = 2 * (side // 4) + min(side % 4, 2)
    out = []
    for t in range(side * tpr):
        row, u = divmod(t, tpr)
        sa = 4 * (u >> 1) + (u & 1)
        out.append((row, sa))
    return out


@pytest.mark.parametrize("w", range(1, MAX_W + 1))
def test_tasks_cover_every_candidate_once(w):
    seen = []
    for row, sa in tasks(w):
        seen.append((row, sa))
        if sa + 2 <= 2 * w:
            seen.append((row, sa + 2))
    want = [(r, c) for r in range(2 * w + 1) for c in range(2 * w + 1)]
    assert sorted(seen) == want


@pytest.mark.parametrize("w", range(1, MAX_W + 1))
def test_window_reads_stay_inside(w):
    S, rp, odd_off, cur_off, per_wave = layout(w)
    assert per_wave % 4 == 0 and cur_off % 4 == 0          # 16-byte aligned block rows
    assert odd_off >= S * rp and cur_off >= odd_off + S * rp  # copies do not overlap
    written = S // 2 + 1                                     # pairs per row, pad included
    assert written <= rp
    for row, sa in tasks(w):
        k0 = sa >> 1
        # rows row .. row + 15 of the window, pairs k0 .. k0 + 8 (second candidate)
        assert row + BLOCK - 1 < S
        assert k0 + PAIRS < written


@pytest.mark.parametrize("w", range(1, MAX_W + 1))
def test_split_pass_shape(w):
    nt = len(tasks(w))
    nfull, tail = divmod(nt, 64)
    if 0 < tail <= 32:
        # lanes 2i, 2i + 1 hold the halves of task 64 * nfull + i
        assert 2 * tail <= 64
    else:
        # every task runs whole: ceil(nt / 64) passes
        assert (nt + 63) // 64 * 64 >= nt
