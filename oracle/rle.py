"""Zero-run length coding of the quantised components (paper section 3.8)
and the DEFLATE stage after it (section 3.9).

TEST INFRASTRUCTURE ONLY: the plain reference of the device run-length
coder; the product path never imports it.

Paper:
  * section 3.8: quantisation leaves long runs of zero-valued coefficients.
    The zero-valued coefficients of the directional subbands of K-frames,
    and of every component (lowpass included) of P-frames, are run-length
    coded along the horizontal direction; other values go on unchanged, and
    the K-frame lowpass (after the column differencing of section 3.7) is
    not run-length coded;
  * section 3.9: the components are then compressed with DEFLATE, either
    each component on its own (the lowpass and every directional subband of
    every scale: transmission scalability) or all components of a frame
    together (CVC-NTS).

Readings (the paper gives no bit format):
  * "along the horizontal direction" is along the rows of a component in its
    natural orientation (image rows). Vertical-cone subbands, stored
    transposed, are therefore read along their stored columns. A run never
    crosses the end of a row.
  * symbols are int16. A non-zero value is one symbol, itself. A maximal run
    of n >= 1 zeros inside a row is two symbols: 0, then n. A zero symbol
    thus always starts a run, and a row of known length parses
    unambiguously.
  * a component that is not run-length coded enters the stream unchanged, in
    its stored order.
  * the stream of a plane follows the packed layout: component by component
    (lowpass first), each row by row; sub_off[s] is the symbol offset of
    component s and sub_off[nsub] the plane's symbol count.
  * DEFLATE works on the symbols as little-endian int16 bytes (zlib format,
    level 6).
"""
import zlib

import numpy as np


def rle_row(row):
    """Symbols of one row: non-zero values as they are, zero runs as (0, n)."""
    out = []
    n = len(row)
    e = 0
    while e < n:
        v = int(row[e])
        if v != 0:
            out.append(v)
            e += 1
            continue
        f = e
        while f < n and int(row[f]) == 0:
            f += 1
        out.extend((0, f - e))
        e = f
    return out


def unrle_row(sym, pos, n):
    """Parse one row of length n from sym[pos:]; returns (row, new pos)."""
    row = []
    while len(row) < n:
        v = int(sym[pos])
        if v != 0:
            row.append(v)
            pos += 1
        else:
            run = int(sym[pos + 1])
            if run < 1 or len(row) + run > n:
                raise ValueError("zero run past the end of the row")
            row.extend([0] * run)
            pos += 2
    return row, pos


def natural(component, sb):
    """The component's stored elements as its natural rows x cols array."""
    a = np.asarray(component)
    if sb.transposed:
        return a.reshape(sb.cols, sb.rows).T
    return a.reshape(sb.rows, sb.cols)


def coded(sb, p_frame):
    """Whether component sb is run-length coded (section 3.8)."""
    return p_frame or sb.k >= 0


def encode_plane(idx, table, p_frame):
    """(symbols int16 array, sub_off int64 array of nsub + 1) of one plane."""
    idx = np.asarray(idx)
    sym = []
    sub_off = [0]
    for sb in table:
        comp = idx[sb.offset:sb.offset + sb.size]
        if coded(sb, p_frame):
            if max(sb.rows, sb.cols) > 32767:
                raise ValueError("rows longer than an int16 run")
            for row in natural(comp, sb):
                sym.extend(rle_row(row))
        else:
            sym.extend(int(v) for v in comp)
        sub_off.append(len(sym))
    return np.asarray(sym, dtype=np.int16), np.asarray(sub_off, dtype=np.int64)


def decode_plane(sym, sub_off, table, p_frame):
    """Inverse of encode_plane: the plane's int16 indices."""
    ncoef = table[-1].offset + table[-1].size
    out = np.empty(ncoef, dtype=np.int16)
    for s, sb in enumerate(table):
        pos, end = int(sub_off[s]), int(sub_off[s + 1])
        if coded(sb, p_frame):
            rows = []
            for _ in range(sb.rows):
                row, pos = unrle_row(sym, pos, sb.cols)
                rows.append(row)
            nat = np.asarray(rows, dtype=np.int16).reshape(sb.rows, sb.cols)
            stored = nat.T if sb.transposed else nat
            out[sb.offset:sb.offset + sb.size] = stored.reshape(-1)
        else:
            out[sb.offset:sb.offset + sb.size] = np.asarray(sym[pos:pos + sb.size], dtype=np.int16)
            pos += sb.size
        if pos != end:
            raise ValueError(f"component {s}: symbols do not end at the next offset")
    return out


def deflate_sizes(sym, sub_off, level=6):
    """DEFLATE byte counts of one plane's stream: (per component list, whole plane)."""
    sym = np.asarray(sym, dtype='<i2')
    per = [len(zlib.compress(sym[int(a):int(b)].tobytes(), level))
           for a, b in zip(sub_off[:-1], sub_off[1:])]
    return per, len(zlib.compress(sym.tobytes(), level))
