"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the SpMM itself: it only draws patterns and
values and rounds them to the storage formats the library consumes. The paper
benchmarks on randomly generated patterns and values (Section 4); the laws here
are this library's readings of that:

* a pattern of density d holds exactly round(d * mb * kb) distinct blocks drawn
  uniformly without replacement (PCG64 seeded generator), so FLOPs are exact;
* values and dense inputs are N(0, 1) unless stated;
* seeds: pattern s, weight values s + 1, X s + 2, dynamic call i uses s + 3 + i.

Storage formats: float32; float16 (IEEE binary16, round to nearest even);
bfloat16 as uint16 bit patterns (round to nearest even); FP8 E4M3FN as uint8
codes plus one float32 scale per block.
"""
import math

import numpy as np

DTYPES = ("f32", "f16", "bf16", "fp8")


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def nnzb_for_density(mb, kb, d):
    return int(math.floor(d * mb * kb + 0.5))


def block_mask(mb, kb, d, seed):
    """uint8 mb x kb mask with exactly round(d * mb * kb) ones, uniform positions."""
    nnzb = nnzb_for_density(mb, kb, d)
    flat = rng(seed).choice(mb * kb, size=nnzb, replace=False) if nnzb else np.zeros(0, np.int64)
    M = np.zeros(mb * kb, dtype=np.uint8)
    M[flat] = 1
    return M.reshape(mb, kb)


def skewed_mask(mb, kb, d, alpha, seed):
    """Mask with exactly round(d * mb * kb) blocks whose row counts follow a
    power law: row of rank t (ranks in random order) gets a share of
    (t + 1)^-alpha, capped at kb; columns uniform without replacement."""
    g = rng(seed)
    nnzb = nnzb_for_density(mb, kb, d)
    w = (np.arange(mb, dtype=np.float64) + 1.0) ** (-float(alpha))
    w = w[g.permutation(mb)]
    counts = np.zeros(mb, np.int64)
    left = nnzb
    free = np.ones(mb, bool)
    while left > 0 and free.any():
        share = w * free
        raw = left * share / share.sum()
        add = np.minimum(np.floor(raw).astype(np.int64), kb - counts)
        rem = left - int(add.sum())
        if rem > 0:  # largest remainders among rows with room
            frac = np.where(free & (counts + add < kb), raw - np.floor(raw), -1.0)
            for r in np.argsort(-frac, kind="stable")[:rem]:
                if frac[r] >= 0:
                    add[r] += 1
        counts += add
        left = nnzb - int(counts.sum())
        free = counts < kb
    M = np.zeros((mb, kb), np.uint8)
    for r in range(mb):
        if counts[r]:
            M[r, g.choice(kb, size=int(counts[r]), replace=False)] = 1
    return M


def concentrated_mask(mb, kb, d, seed):
    """Mask with exactly round(d * mb * kb) blocks packed into as few block
    rows as possible (random rows, fully dense but the last): the load-balance
    worst case of a partitioned SpMM."""
    g = rng(seed)
    nnzb = nnzb_for_density(mb, kb, d)
    rows = g.permutation(mb)
    M = np.zeros((mb, kb), np.uint8)
    full, rest = divmod(nnzb, kb)
    M[rows[:full]] = 1
    if rest:
        M[rows[full], g.choice(kb, size=rest, replace=False)] = 1
    return M


def ell_from_mask(M, width, seed):
    """Blocked-ELL description of a mask: int32 [mb, width], each row's block
    columns in a seeded random slot order, -1 in the remaining slots."""
    M = np.asarray(M)
    counts = M.sum(1)
    if counts.max(initial=0) > width:
        raise ValueError("ELL width below the longest row")
    g = rng(seed)
    cols = np.full((M.shape[0], width), -1, np.int32)
    for r in range(M.shape[0]):
        c = np.nonzero(M[r])[0]
        slots = g.permutation(width)[: c.size]
        cols[r, slots] = c
    return cols


def mask_coo(M):
    """Row-major (CSR-order) list of the nonzero blocks of a mask."""
    rr, cc = np.nonzero(np.asarray(M))
    return rr.astype(np.int32), cc.astype(np.int32)


def normal(shape, seed):
    return rng(seed).standard_normal(size=shape, dtype=np.float64).astype(np.float32)


def integers(shape, seed, lo=-2, hi=2):
    return rng(seed).integers(lo, hi + 1, size=shape).astype(np.float32)


def scaled_block_values(nnzb, b, seed, lo=0.1, hi=10.0):
    """N(0,1) * sigma per block with sigma ~ U(lo, hi): the FP8 precision workload."""
    g = rng(seed)
    v = g.standard_normal(size=(nnzb, b, b), dtype=np.float64)
    sig = g.uniform(lo, hi, size=(nnzb, 1, 1))
    return (v * sig).astype(np.float32)


# ---------------------------------------------------------------- storage formats

def to_f16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16)


def to_bf16_bits(x):
    """Round float32 to bfloat16 (nearest even) and return the uint16 bit patterns."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def to_storage(x, dtype):
    """Round float32 data to a storage dtype ('f32', 'f16', 'bf16')."""
    if dtype == "f32":
        return np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if dtype == "f16":
        return np.ascontiguousarray(to_f16(x))
    if dtype == "bf16":
        return np.ascontiguousarray(to_bf16_bits(x))
    raise ValueError("unknown storage dtype %r" % (dtype,))


def storage_to_f64(s, dtype):
    """Exact upcast of stored values to float64."""
    if dtype in ("f32", "f16"):
        return np.asarray(s).astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f32(s).astype(np.float64)
    raise ValueError("unknown storage dtype %r" % (dtype,))


def _e4m3fn_grid():
    """Non-negative finite E4M3FN values for codes 0..126 (ascending)."""
    codes = np.arange(127)
    e = codes >> 3
    f = codes & 7
    return np.where(e == 0, f / 8.0 * 2.0 ** -6, (1 + f / 8.0) * np.power(2.0, e - 7.0))


_GRID = _e4m3fn_grid()


def quantize_e4m3fn_blocks(vals):
    """Per-block FP8 quantisation of [nnz, b, b] values.

    s = amax / 448 computed in float32 (s = 1 for an all-zero block), then each
    value v is encoded as the E4M3FN code nearest to v / s (ties to the even
    code), saturating at +-448. Returns (codes uint8 [nnz, b, b], scales float32 [nnz])."""
    v = np.asarray(vals, dtype=np.float32)
    nnz = v.shape[0]
    amax = np.abs(v.reshape(nnz, -1)).max(axis=1) if nnz else np.zeros(0, np.float32)
    scales = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    t = v.astype(np.float64) / scales.astype(np.float64).reshape(-1, *([1] * (v.ndim - 1)))
    a = np.minimum(np.abs(t), 448.0)
    hi = np.clip(np.searchsorted(_GRID, a, side="left"), 0, 126)
    lo = np.maximum(hi - 1, 0)
    d_hi = _GRID[hi] - a
    d_lo = a - _GRID[lo]
    pick_lo = (d_lo < d_hi) | ((d_lo == d_hi) & (lo % 2 == 0))
    mag = np.where(pick_lo, lo, hi).astype(np.uint8)
    codes = np.where(t < 0, mag | np.uint8(0x80), mag).astype(np.uint8)
    codes = np.where((t < 0) & (mag == 0), np.uint8(0x80), codes)  # keep the sign of -0
    return codes, scales


# ---------------------------------------------------------------- dynamic and serving streams

def dynamic_call(mb, kb, b, max_nnzb, seed, dtype="f16", lo_frac=0.5):
    """One dynamic-mode call: nnz ~ U{ceil(lo_frac*max), max}, distinct random blocks in
    random (unsorted) COO order, N(0,1) values rounded to `dtype`."""
    g = rng(seed)
    lo = int(math.ceil(lo_frac * max_nnzb))
    nnz = int(g.integers(lo, max_nnzb + 1))
    flat = g.choice(mb * kb, size=nnz, replace=False)
    rows = (flat // kb).astype(np.int32)
    cols = (flat % kb).astype(np.int32)
    vals = g.standard_normal(size=(nnz, b, b), dtype=np.float64).astype(np.float32)
    return rows, cols, to_storage(vals, dtype)


def serving_trace(num_requests, rate_per_s, seed, n_max=2048):
    """Poisson arrivals (exponential gaps) and n = floor(exp(U[0, ln(n_max + 1)))) tokens."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_per_s, size=num_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    n = np.floor(np.exp(g.uniform(0.0, math.log(n_max + 1), size=num_requests))).astype(np.int64)
    n = np.clip(n, 1, n_max)
    return arrivals, n
