"""Edit stream of a correction: what a compressor stores next to its own
output so that a decompressor can rebuild g' from g_hat.

The monotone edit of Sec. 3.3 moves a vertex down by the step Delta a
number of times (its edit count, 0 .. N + 1); a vertex that needed more than
N edits holds its lower bound f - xi instead, which the paper stores
losslessly (and compresses all edits with a general lossless coder).  A
decompressor has g_hat and Delta but not f, so it can replay c steps
(each one rounded to the field type) but cannot know the lower bound: every
vertex whose value is not the replay of its count -- the (N+1)-th edits, and
edits clamped at the bound earlier -- is stored exactly.

Stream layout (little endian):
  header   magic "EXZE", version 1, dtype code (0 float32, 1 float64),
           N, n, number of edited vertices E, number of exact values X
  records  E varints, one per edited vertex in index order:
           (index - previous index - 1) << 5 | exact << 4 | count
  values   X raw values of the field type, in record order
The whole stream may then go through a general-purpose coder (zlib here,
standing in for the ZSTD of the paper).
"""
from __future__ import annotations

import struct
import zlib
from dataclasses import dataclass

import numpy as np

MAGIC = b"EXZE"
VERSION = 1
_HEADER = struct.Struct("<4sBBBxQQQ")


def step(xi: float, dtype, n_steps: int):
    """Delta of the edit (Sec. 3.3) in the field type: xi_T = the largest
    value of the type not above xi, Delta = xi_T / N rounded to nearest."""
    if np.dtype(dtype) == np.float32:
        x = np.float32(xi)
        if float(x) > xi:
            x = np.nextafter(x, np.float32(-np.inf))
        return np.float32(x / np.float32(n_steps))
    return np.float64(xi) / np.float64(n_steps)


def replay(g_hat: np.ndarray, counts: np.ndarray, delta) -> np.ndarray:
    """g_hat moved down `counts` times by delta, each step rounded to the
    field type (the decompressor's view; no lower bound)."""
    g = np.array(g_hat, copy=True)
    d = g.dtype.type(delta)
    c = np.asarray(counts)
    for k in range(1, int(c.max(initial=0)) + 1):
        sel = c >= k
        g[sel] = g[sel] - d
    return g


def _varints(v: np.ndarray) -> bytes:
    """LEB128 varints of non-negative integers, vectorised."""
    v = np.asarray(v, dtype=np.uint64)
    if v.size == 0:
        return b""
    nbytes = np.ones(v.size, dtype=np.int64)
    t = v >> np.uint64(7)
    while np.any(t):
        nbytes += (t > 0)
        t >>= np.uint64(7)
    out = np.zeros(int(nbytes.sum()), dtype=np.uint8)
    starts = np.concatenate(([0], np.cumsum(nbytes)[:-1]))
    rem = v.copy()
    for k in range(int(nbytes.max())):
        live = nbytes > k
        byte = (rem[live] & np.uint64(0x7F)).astype(np.uint8)
        more = nbytes[live] > k + 1
        out[starts[live] + k] = byte | (more.astype(np.uint8) << 7)
        rem[live] >>= np.uint64(7)
    return out.tobytes()


def _read_varints(buf: bytes, count: int, pos: int):
    vals = np.zeros(count, dtype=np.uint64)
    for j in range(count):
        shift = 0
        x = 0
        while True:
            b = buf[pos]
            pos += 1
            x |= (b & 0x7F) << shift
            shift += 7
            if not b & 0x80:
                break
        vals[j] = x
    return vals, pos


@dataclass
class EditStream:
    data: bytes          # the stream itself
    edited: int          # vertices with a nonzero count
    exact: int           # vertices stored as exact values
    record_bytes: int    # bytes of the index/count records
    value_bytes: int     # bytes of the exact values

    def compressed(self, level: int = 6) -> int:
        """Size after the general-purpose coder."""
        return len(zlib.compress(self.data, level))


def encode(g_hat: np.ndarray, g_out: np.ndarray, counts: np.ndarray, delta, n_steps: int) -> EditStream:
    g_hat = np.ascontiguousarray(g_hat).ravel()
    g_out = np.ascontiguousarray(g_out, dtype=g_hat.dtype).ravel()
    counts = np.ascontiguousarray(counts, dtype=np.uint8).ravel()
    if not (g_hat.size == g_out.size == counts.size):
        raise ValueError("g_hat, g_out and counts must have the same size")
    if n_steps < 1 or n_steps > 14:
        raise ValueError("n_steps must be 1..14 (a count fits in four bits)")
    idx = np.flatnonzero(counts)
    c = counts[idx].astype(np.uint64)
    rep = replay(g_hat[idx], c, delta)
    # exact unless the replay reproduces the value bit for bit
    b = g_hat.itemsize
    exact = np.any(rep.view(np.uint8).reshape(idx.size, b) !=
                   g_out[idx].view(np.uint8).reshape(idx.size, b), axis=1)
    gaps = np.diff(np.concatenate(([-1], idx))) - 1
    rec = (gaps.astype(np.uint64) << np.uint64(5)) | (exact.astype(np.uint64) << np.uint64(4)) | c
    records = _varints(rec)
    values = g_out[idx[exact]].tobytes()
    code = 0 if g_hat.dtype == np.float32 else 1
    header = _HEADER.pack(MAGIC, VERSION, code, n_steps, g_hat.size, idx.size, int(exact.sum()))
    return EditStream(header + records + values, int(idx.size), int(exact.sum()), len(records),
                      len(values))


def decode(data: bytes, g_hat: np.ndarray, delta) -> tuple:
    """(g', counts) rebuilt from g_hat and the stream."""
    magic, ver, code, n_steps, n, e, x = _HEADER.unpack_from(data, 0)
    if magic != MAGIC or ver != VERSION:
        raise ValueError("not an edit stream")
    dt = np.float32 if code == 0 else np.float64
    g_hat = np.ascontiguousarray(g_hat, dtype=dt).ravel()
    if g_hat.size != n:
        raise ValueError("g_hat has %d values, the stream %d" % (g_hat.size, n))
    rec, pos = _read_varints(data, e, _HEADER.size)
    counts = np.zeros(n, dtype=np.uint8)
    idx = np.cumsum((rec >> np.uint64(5)).astype(np.int64) + 1) - 1
    c = (rec & np.uint64(15)).astype(np.uint8)
    exact = ((rec >> np.uint64(4)) & np.uint64(1)).astype(bool)
    counts[idx] = c
    g = replay(g_hat, counts, delta)
    vals = np.frombuffer(data, dtype=dt, count=x, offset=pos)
    g[idx[exact]] = vals
    return g, counts
