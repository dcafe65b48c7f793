"""Independent pure-Python reading of the FSZ stream format, for tests only.

Written separately from both the oracle and the HIP library: it parses
streams, recomputes per-tile choices by brute force (four full residual
passes, no cancellation shortcut) and can encode a stream with arbitrary
(even non-optimal) per-tile variant choices, which every decoder must accept.

Format (see the design notes): 32-byte header, one rate byte per 32-element
block (Sec. III-A) zero-padded to 16 bytes, then per 256-element tile its
optional int32 mean and, per block with rate r > 0, a sign word and r
bit-plane words, element j of the block at bit 31 - j, words written
most-significant byte first (Sec. IV-C).

Tile configurations (Sec. VI-C, Table V): every helper takes the block size
B (32 or 64) and the blocks per tile T (4, 8, 16); header flags bits 2-4 hold
them (bit 2: B = 64; bits 3-4: 0 -> T = 8, 1 -> T = 4, 2 -> T = 16).  A
64-element block's sign map and planes are 64-bit big-endian words.
"""
import struct

import numpy as np

HEADER = 32
BLOCK = 32
TILE = 256


def ceil_div(a, b):
    return -(-a // b)


def pad16(a):
    return (a + 15) // 16 * 16


def data_start(n, B=BLOCK):
    return HEADER + pad16(ceil_div(n, B))


def config_flags(B=BLOCK, T=8):
    return (4 if B == 64 else 0) | {8: 0, 4: 8, 16: 16}[T]


def header_config(flags):
    """(B, T) from header flags, or None for the reserved T code."""
    tc = (flags >> 3) & 3
    if tc == 3:
        return None
    return (64 if flags & 4 else 32), {0: 8, 1: 4, 2: 16}[tc]


def parse_header(s: bytes) -> dict:
    magic, version, mode, flags, n, E, value, total = struct.unpack_from("<4sHBBQffQ", s, 0)
    return dict(magic=magic, version=version, mode=mode, flags=flags, n=n, E=E, value=value,
                total=total)


def rate_bytes(s: bytes, n: int, B=BLOCK) -> np.ndarray:
    return np.frombuffer(s, dtype=np.uint8, count=ceil_div(n, B), offset=HEADER)


def bitlen(v: int) -> int:
    return int(v).bit_length()


def block_cost(r: int, B=BLOCK) -> int:
    """Sign map + r planes of B bits each (Eq. 3 for B = 32)."""
    return 0 if r == 0 else (B // 8) * (1 + r)


def tile_choices(s: bytes, n: int, B=BLOCK, T=8):
    """Per tile: (order2, centred, [T rates]) read from the rate header
    (blocks past the end of a ragged last tile read as rate 0)."""
    rb = rate_bytes(s, n, B)
    out = []
    for t in range(ceil_div(n, B * T)):
        blk = rb[t * T:(t + 1) * T]
        rates = [int(b) & 0x1F for b in blk] + [0] * (T - blk.size)
        out.append((int(blk[0] >> 7) & 1, int(blk[0] >> 6) & 1, rates))
    return out


def tile_sizes(s: bytes, n: int, B=BLOCK, T=8):
    return [sum(block_cost(r, B) for r in rates) + 4 * c for (_, c, rates) in tile_choices(s, n, B, T)]


def tile_sizes_np(s: bytes, n: int, B=BLOCK, T=8) -> np.ndarray:
    """tile_sizes as one int64 array, computed with array operations (for
    rate headers of millions of tiles)."""
    rb = np.frombuffer(s, dtype=np.uint8, count=ceil_div(n, B), offset=HEADER)
    nt = ceil_div(n, B * T)
    r = np.zeros(nt * T, dtype=np.int64)
    r[:rb.size] = rb & 0x1F
    cost = np.where(r > 0, (B // 8) * (1 + r), 0).reshape(nt, T).sum(axis=1)
    return cost + 4 * ((rb[::T].astype(np.int64) >> 6) & 1)


def quantize(x: np.ndarray, inv: float) -> np.ndarray:
    """q = rint(fl32(x * inv)) in binary32, as int64."""
    y = (np.asarray(x, dtype=np.float32) * np.float32(inv)).astype(np.float32)
    return np.rint(y).astype(np.int64)


def closed_form(x: np.ndarray, E: float, inv: float) -> np.ndarray:
    """Reconstruction fl32((float)q * E): independent of variant and mean."""
    q = quantize(x, inv)
    return (q.astype(np.float32) * np.float32(E)).astype(np.float32)


def pairwise_mean(xt: np.ndarray, inv: float, tile=TILE):
    """(finite, mu): index-order pairwise binary32 sum of `tile` slots (+0
    padded), times 1/tile (exact: a power of two)."""
    s = np.zeros(tile, dtype=np.float32)
    s[:xt.size] = xt
    with np.errstate(over="ignore", invalid="ignore"):
        while s.size > 1:
            s = (s[0::2] + s[1::2]).astype(np.float32)
        v = np.float32(np.float32(s[0] * np.float32(1.0 / tile)) * np.float32(inv))
    if not np.isfinite(v):
        return False, 0
    return True, int(np.rint(v))


def residuals(q: np.ndarray, order2: int, mu: int, independent: bool = False, B=BLOCK) -> np.ndarray:
    """Lorenzo residuals of q - mu with zero state before the tile start
    (independent: before every block start)."""
    qc = np.asarray(q, dtype=np.int64) - mu
    if independent:
        return np.concatenate([residuals(qc[b:b + B], order2, 0)
                               for b in range(0, qc.size, B)]).astype(np.int64)
    p1 = np.concatenate([[0], qc[:-1]])
    if not order2:
        return qc - p1
    p2 = np.concatenate([[0, 0], qc[:-2]])[:qc.size]
    return qc - 2 * p1 + p2


# feature switches of the ablation (Sec. VI-B)
CROSS_BLOCK, CENTERING, LZ2, ALL = 1, 2, 4, 7


def allowed(v: int, features: int, centre_ok: bool) -> bool:
    if (v & 1) and not features & LZ2:
        return False
    if (v >> 1) and (not features & CENTERING or not centre_ok):
        return False
    return True


def brute_force_tile(xt: np.ndarray, inv: float, features: int = ALL, B=BLOCK, T=8):
    """Four separate full passes; returns (mu, centre_ok, costs[4], rates[4][T], best)."""
    m = xt.size
    nb = ceil_div(m, B)
    q = quantize(xt, inv)
    ok, mu = pairwise_mean(xt, inv, B * T)
    indep = not features & CROSS_BLOCK
    costs, rates = [], []
    for v in range(4):
        order2, cen = v & 1, v >> 1
        res = np.zeros(B * T, dtype=np.int64)
        res[:m] = residuals(q, order2, mu if cen else 0, indep, B)
        rv = [bitlen(int(np.abs(res[b * B:(b + 1) * B]).max())) if b < nb else 0
              for b in range(T)]
        rates.append(rv)
        costs.append(sum(block_cost(r, B) for r in rv) + (4 if cen else 0))
    best = 0
    for v in (1, 2, 3):
        if allowed(v, features, ok) and costs[v] < costs[best]:
            best = v
    return mu, ok, costs, rates, best


def _word_bytes(w: int, B=BLOCK) -> bytes:
    return struct.pack(">I" if B == 32 else ">Q", w)


def encode_stream(x: np.ndarray, E: float, inv: float, mode: int, value: float, flags: int,
                  choices, B=BLOCK, T=8) -> bytes:
    """Encode x with the given per-tile (order2, centred, mu) choices
    (flags bit 1: independent blocks; the configuration bits of (B, T) are
    added here)."""
    x = np.asarray(x, dtype=np.float32).reshape(-1)
    n = x.size
    q = quantize(x, inv)
    nblocks = ceil_div(n, B)
    tile = B * T
    flags |= config_flags(B, T)
    rate_hdr = bytearray(pad16(nblocks))
    body = bytearray()
    for t in range(ceil_div(n, tile)):
        qt = q[t * tile:(t + 1) * tile]
        m = qt.size
        order2, cen, mu = choices[t]
        res = np.zeros(tile, dtype=np.int64)
        res[:m] = residuals(qt, order2, mu if cen else 0, bool(flags & 2), B)
        if cen:
            body += struct.pack("<i", mu)
        for b in range(ceil_div(m, B)):
            blk = res[b * B:(b + 1) * B]
            r = bitlen(int(np.abs(blk).max()))
            byte = r
            if b == 0:
                byte |= (order2 << 7) | (cen << 6)
            rate_hdr[t * T + b] = byte
            if r == 0:
                continue
            sign = 0
            for j in range(B):
                if blk[j] < 0:
                    sign |= 1 << (B - 1 - j)
            body += _word_bytes(sign, B)
            mag = np.abs(blk)
            for p in range(r):
                w = 0
                for j in range(B):
                    w |= ((int(mag[j]) >> p) & 1) << (B - 1 - j)
                body += _word_bytes(w, B)
    total = HEADER + len(rate_hdr) + len(body)
    hdr = struct.pack("<4sHBBQffQ", b"FSZ1", 1, mode, flags, n, E, value, total)
    return bytes(hdr) + bytes(rate_hdr) + bytes(body)
