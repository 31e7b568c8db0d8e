"""Pins of the layout: section 3.3 (resolutions per level, coarse-to-fine stream), section 2.1 (2^l subbands)."""
import json
import os

import pytest

from oracle import geometry as geo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_vga_two_levels_resolutions():
    with open(os.path.join(GOLDEN, "vga_pyramid.json")) as f:
        ref = json.load(f)
    W, H = ref["frame_wh"]
    R, C = geo.padded_size(H, W, ref["levels"], [4] * ref["levels"])
    got = [[C >> j, R >> j] for j in range(ref["levels"] + 1)]
    assert got == ref["resolutions_wh"]


@pytest.mark.parametrize("H,W,J,dirs,ncoef,R,C", [
    (256, 256, 2, [8, 4], 86016, 256, 256),
    (480, 640, 3, [16, 8, 4], 408000, 480, 640),
    (1080, 1920, 4, [32, 16, 8, 8], 2782560, 1088, 1920),
    (720, 1280, 3, [16, 8, 4], 1224000, 720, 1280),
    (240, 320, 4, [16, 8, 8, 8], None, 256, 320),
    (720, 1280, 4, [16, 8, 8, 8], None, 736, 1280),
])
def test_sizes_and_redundancy(H, W, J, dirs, ncoef, R, C):
    assert geo.padded_size(H, W, J, dirs) == (R, C)
    n = geo.ncoef(H, W, J, dirs)
    rho = 4.0 ** -J + sum(4.0 ** -i for i in range(J))
    assert n == round(rho * R * C)
    if ncoef is not None:
        assert n == ncoef


def test_subband_counts_and_contiguity():
    J, dirs = 4, [32, 16, 8, 8]
    table = geo.subband_table(1080, 1920, J, dirs)
    assert len(table) == 1 + sum(dirs)
    off = 0
    for sb in table:
        assert sb.offset == off
        off += sb.size
    # coarse to fine after the lowpass
    levels = [sb.level for sb in table[1:]]
    assert levels == sorted(levels, reverse=True)
    for j in range(1, J + 1):
        ks = [sb.k for sb in table if sb.level == j]
        assert ks == list(range(dirs[j - 1]))
        # critically sampled: subbands of a level tile the level image
        R, C = geo.padded_size(1080, 1920, J, dirs)
        Rj, Cj = geo.level_size(R, C, j)
        assert sum(sb.size for sb in table if sb.level == j) == Rj * Cj
        # every level pixel belongs to exactly one subband lattice coset
        covered = set()
        for sb in table:
            if sb.level != j:
                continue
            key = (sb.o1 % sb.s1, sb.o2 % sb.s2, sb.s1, sb.s2)
            assert key not in covered
            covered.add(key)


def test_cosets_partition_the_level_image():
    for l in range(2, 7):
        leaves = geo.tree_levels(l)[l]
        N = 1 << (l + 1)
        hit = {}
        for n in leaves:
            for i in range(N // n.D[0]):
                for k in range(N // n.D[1]):
                    p = ((n.o[0] + n.D[0] * i) % N, (n.o[1] + n.D[1] * k) % N)
                    assert p not in hit
                    hit[p] = (n.cone, n.a)
        assert len(hit) == N * N


@pytest.mark.parametrize("bad", [
    dict(height=256, width=256, levels=0, dirs=[]),
    dict(height=256, width=256, levels=2, dirs=[8]),
    dict(height=256, width=256, levels=2, dirs=[6, 4]),
    dict(height=256, width=256, levels=2, dirs=[128, 4]),
    dict(height=256, width=256, levels=2, dirs=[2, 4]),
    dict(height=8, width=256, levels=2, dirs=[32, 4]),
])
def test_validation_rejects(bad):
    with pytest.raises(ValueError):
        geo.validate(**bad)
