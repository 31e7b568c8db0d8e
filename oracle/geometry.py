"""Geometry of the contourlet decomposition: padding, level sizes, DFB tree, layout.

Paper anchors:
  * section 3.3: each LP level halves the resolution (two levels of a 640x480
    frame give 640x480, 320x240 and 160x120) and the result is the coarsest
    lowpass plus the directional subbands of every scale;
  * section 2.1: the DFB at level l yields 2^l wedge-shaped subbands.

Readings (the paper is silent on these):
  * Boundary. Convolutions are periodic (the paper computes them with FFTs,
    section 3.10). Every stage acts on an R x C torus. R and C are the frame
    size rounded up to a multiple of 2^e, with
        e = max(J, max_j (j + l_j - 2)),   j = 1 (finest) .. J.
    The extra rows and columns repeat the frame mirrored about its last
    sample: x[H + i] = x[H - 1 - i]. The inverse crops them off.
  * DFB tree (each node is a two-channel quincunx fan filter bank, see dfb.py):
      - tree level 1 splits Z^2 with basis v1 = (1,0), v2 = (0,1). The even
        child (n1 + n2 even) is the vertical cone |w1| > |w2|. The odd child,
        on the coset (1,0), is the horizontal cone.
      - tree level 2 splits the vertical cone with v1 = (1,1), v2 = (-1,1),
        and the horizontal cone with v1 = (1,1), v2 = (1,-1). All four
        children land on cosets of 2Z^2.
      - tree level t >= 3, m = t - 2. A vertical channel with parameter a
        lives on o + diag(2, 2^m) Z^2. It is split with v1 = (2a, -2^m),
        v2 = (2a + 2, -2^m). The even child gets a' = 2a + 1 at offset o,
        the odd child a' = 2a at offset o + v1. Horizontal channels are the
        coordinate swap: v1 = (-2^m, 2a), v2 = (-2^m, 2a + 2).
      - every offset is reduced into [0, D1) x [0, D2) for the channel's
        lattice diag(D1, D2) Z^2, and the even sub-coset of a node is the one
        that contains its offset (the labelling of the two children depends
        on the representative, so it has to be fixed).
      - a vertical channel with parameter a covers the slopes w2/w1 in
        (a, a+1) / 2^(t-2); a horizontal one covers w1/w2 in the same range.
  * Subband order k: by wedge angle atan2(w1, w2), increasing over
    (-45, 135) degrees. Horizontal cone first (ascending a), then vertical
    cone (descending a).
  * Packed layout per plane: the lowpass, then levels j = J..1 (coarse to
    fine, so that a receiver can drop the finer scales, section 3.3), each
    level's subbands in k order. Horizontal-cone subbands are stored row
    major as their natural (R_j / 2^(l-1)) x (C_j / 2) array. Vertical-cone
    subbands, natural shape (R_j / 2) x (C_j / 2^(l-1)), are stored
    transposed, i.e. row major as (C_j / 2^(l-1)) x (R_j / 2).
"""
from dataclasses import dataclass, field

MAX_LEVELS = 6


def log2_exact(n):
    """log2 of a positive power of two; raises ValueError otherwise."""
    if n <= 0 or n & (n - 1):
        raise ValueError(f"{n} is not a positive power of two")
    return n.bit_length() - 1


def validate(height, width, levels, dirs):
    """Check a geometry; raises ValueError with the reason."""
    if not 1 <= levels <= MAX_LEVELS:
        raise ValueError("levels must be in 1..6")
    if len(dirs) != levels:
        raise ValueError("one direction count per level is required")
    for d in dirs:
        if d < 4 or d > 64 or d & (d - 1):
            raise ValueError("direction counts must be powers of two in [4, 64]")
    e = pad_exponent(levels, dirs)
    if height < (1 << e) or width < (1 << e):
        raise ValueError(f"frame smaller than 2^{e} in one dimension")


def pad_exponent(levels, dirs):
    """e = max(J, max_j (j + l_j - 2)) with j = 1 the finest level."""
    e = levels
    for j, d in enumerate(dirs, start=1):
        e = max(e, j + log2_exact(d) - 2)
    return e


def padded_size(height, width, levels, dirs):
    """(R, C): the torus size, each side rounded up to a multiple of 2^e."""
    step = 1 << pad_exponent(levels, dirs)
    return (-(-height // step) * step, -(-width // step) * step)


def level_size(R, C, j):
    """Size of the level-j bandpass image (j = 1 is the full torus)."""
    return R >> (j - 1), C >> (j - 1)


@dataclass
class Node:
    """One channel of the DFB tree, on the lattice coset o + diag(D) Z^2.

    For tree levels 1 and 2 the lattice is not diagonal; `basis` then holds
    the generator columns of the channel's lattice and D is None.
    """
    cone: str              # 'root', 'V' or 'H'
    a: int                 # wedge parameter (slopes in (a, a+1) / 2^(t-2))
    o: tuple               # offset in level coordinates (row, col)
    D: tuple = None        # diagonal lattice (rows step, cols step) if diagonal
    basis: tuple = None    # lattice generators as two column vectors
    children: list = field(default_factory=list)


def split_basis(node, t):
    """(v1, v2) used to split `node` at tree level t (1-based)."""
    if t == 1:
        return (1, 0), (0, 1)
    if t == 2:
        return ((1, 1), (-1, 1)) if node.cone == 'V' else ((1, 1), (1, -1))
    m = t - 2
    a = node.a
    if node.cone == 'V':
        return (2 * a, -(1 << m)), (2 * a + 2, -(1 << m))
    return (-(1 << m), 2 * a), (-(1 << m), 2 * a + 2)


def _reduce(o, D):
    return (o[0] % D[0], o[1] % D[1])


def tree_levels(l):
    """List of node lists, one per tree level 0..l, each in subband order.

    Level 0 is the root; level l holds the 2^l final subbands in k order.
    """
    root = Node('root', 0, (0, 0), D=(1, 1), basis=((1, 0), (0, 1)))
    levels = [[root]]
    # tree level 1: vertical = even child on the quincunx lattice
    v = Node('V', 0, (0, 0), basis=((1, 1), (-1, 1)))
    h = Node('H', 0, (1, 0), basis=((1, 1), (1, -1)))
    levels.append([h, v])
    if l == 1:
        return levels
    # tree level 2: four cosets of 2Z^2
    nodes2 = [
        Node('H', -1, (0, 1), D=(2, 2)),
        Node('H', 0, (1, 0), D=(2, 2)),
        Node('V', 0, (0, 0), D=(2, 2)),
        Node('V', -1, (1, 1), D=(2, 2)),
    ]
    levels.append(nodes2)
    for t in range(3, l + 1):
        m = t - 2
        nxt_h, nxt_v = [], []
        for node in levels[-1]:
            v1, _ = split_basis(node, t)
            if node.cone == 'V':
                D = (2, 1 << (m + 1))
            else:
                D = (1 << (m + 1), 2)
            even = Node(node.cone, 2 * node.a + 1, _reduce(node.o, D), D=D)
            odd = Node(node.cone, 2 * node.a,
                       _reduce((node.o[0] + v1[0], node.o[1] + v1[1]), D), D=D)
            (nxt_v if node.cone == 'V' else nxt_h).extend([even, odd])
        nxt_h.sort(key=lambda n: n.a)
        nxt_v.sort(key=lambda n: -n.a)
        levels.append(nxt_h + nxt_v)
    return levels


@dataclass
class Subband:
    level: int            # LP level j (1 = finest); J + 1 marks the lowpass
    k: int                # subband index within its level (-1 for the lowpass)
    rows: int             # natural number of rows
    cols: int             # natural number of columns
    offset: int           # offset of the first element in the packed plane
    o1: int               # lattice offset (row) in level-j bandpass coordinates
    o2: int               # lattice offset (col)
    s1: int               # lattice step along rows
    s2: int               # lattice step along columns
    transposed: bool      # stored as the transpose of the natural array
    cone: str = 'L'
    a: int = 0

    @property
    def size(self):
        return self.rows * self.cols


def subband_table(height, width, levels, dirs):
    """Packed layout of one plane: list of Subband in storage order."""
    validate(height, width, levels, dirs)
    R, C = padded_size(height, width, levels, dirs)
    table = []
    off = 0
    lr, lc = R >> levels, C >> levels
    table.append(Subband(levels + 1, -1, lr, lc, 0, 0, 0, 1, 1, False))
    off += lr * lc
    for j in range(levels, 0, -1):
        Rj, Cj = level_size(R, C, j)
        l = log2_exact(dirs[j - 1])
        leaves = tree_levels(l)[l]
        for k, node in enumerate(leaves):
            rows, cols = Rj // node.D[0], Cj // node.D[1]
            table.append(Subband(j, k, rows, cols, off, node.o[0], node.o[1],
                                 node.D[0], node.D[1], node.cone == 'V',
                                 node.cone, node.a))
            off += rows * cols
    return table


def ncoef(height, width, levels, dirs):
    """Number of coefficients per plane."""
    t = subband_table(height, width, levels, dirs)
    return t[-1].offset + t[-1].size
