"""Seeded synthetic inputs, shared by the GPU path's callers and the oracle.

This module holds none of the method's arithmetic.  It draws random numbers and
places them on the cells of the gasket, the domain of every workload: cell
(x, y) (column x, row y, 0-based) belongs to the gasket iff (x & y) == 0, and
every other cell of the n x n embedding holds 0.

Draw order: one draw per gasket cell, in row-major order, from NumPy's
``default_rng(seed)`` (PCG64).  Rows are filled in chunks, which does not change
the stream: consecutive calls of ``Generator.random`` continue it.

States too large to build on the host (r > 16) use a counter-based generator
instead, so that any cell's value can be computed on its own: cell (x, y) takes
output number y * 2^32 + x of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
seeded with the seed, and is alive iff that output is below a threshold.  The
library's sg_compact_init_bernoulli writes the same state on the device.
"""
from dataclasses import dataclass
from typing import List

import numpy as np

DEFAULT_SEED = 1706


def gasket_rows(n: int, y0: int, y1: int) -> np.ndarray:
    """Boolean mask of the gasket cells in rows [y0, y1) of an n x n array."""
    # the narrowest unsigned type that holds every coordinate (the mask of
    # 256 rows of n = 2^16 then takes 32 MB of temporaries, not 128 MB)
    dt = np.uint16 if n <= (1 << 16) else np.uint32
    x = np.arange(n, dtype=dt)[None, :]
    y = np.arange(y0, y1, dtype=dt)[:, None]
    return (x & y) == 0


def _row_chunk(n: int) -> int:
    return max(1, (1 << 24) // n)


def bernoulli_state(r: int, p: float = 0.5, seed: int = DEFAULT_SEED) -> np.ndarray:
    """uint8 n x n state: Bernoulli(p) 0/1 on gasket cells, 0 elsewhere."""
    n = 1 << r
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n), dtype=np.uint8)
    step = _row_chunk(n)
    for y0 in range(0, n, step):
        y1 = min(n, y0 + step)
        m = gasket_rows(n, y0, y1)
        k = int(m.sum())
        a[y0:y1][m] = (rng.random(k) < p).astype(np.uint8)
    return a


def uniform_field(r: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """float32 n x n field: U[0, 1) on gasket cells, 0 elsewhere."""
    n = 1 << r
    rng = np.random.default_rng(seed)
    u = np.zeros((n, n), dtype=np.float32)
    step = _row_chunk(n)
    for y0 in range(0, n, step):
        y1 = min(n, y0 + step)
        m = gasket_rows(n, y0, y1)
        k = int(m.sum())
        u[y0:y1][m] = rng.random(k, dtype=np.float32)
    return u


def fractal_mask(m: int, offsets, r: int) -> np.ndarray:
    """Boolean m^r x m^r mask of a fractal that keeps the m x m sub-squares at
    `offsets` [(dx, dy), ...] at every scale (the domain of the other-fractal
    workloads), built by placing copies of the previous level."""
    mask = np.ones((1, 1), dtype=bool)
    for _ in range(r):
        n = mask.shape[0]
        big = np.zeros((m * n, m * n), dtype=bool)
        for dx, dy in offsets:
            big[dy * n:(dy + 1) * n, dx * n:(dx + 1) * n] = mask
        mask = big
    return mask


def fractal_state(m: int, offsets, r: int, p: float = 0.5,
                  seed: int = DEFAULT_SEED) -> np.ndarray:
    """uint8 state on a fractal: Bernoulli(p) 0/1 on its cells (one draw per
    cell, row-major), 0 elsewhere."""
    mask = fractal_mask(m, offsets, r)
    n = mask.shape[0]
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n), dtype=np.uint8)
    step = _row_chunk(n)
    for y0 in range(0, n, step):
        y1 = min(n, y0 + step)
        mk = mask[y0:y1]
        a[y0:y1][mk] = (rng.random(int(mk.sum())) < p).astype(np.uint8)
    return a


def fractal_state_device(m: int, offsets, r: int, p: float = 0.5, seed: int = DEFAULT_SEED,
                         device="cuda"):
    """A uint8 state on a fractal built on the device with torch, for sizes
    whose host generation would take minutes (r = 10: n = 59,049, 3.5 GB):
    the mask by placing copies of the previous level, as fractal_mask, and
    Bernoulli(p) 0/1 from torch's generator seeded with `seed`, drawn in
    row chunks.  Returns a torch tensor on `device`."""
    import torch
    mask = torch.ones((1, 1), dtype=torch.bool, device=device)
    for _ in range(r):
        n = mask.shape[0]
        big = torch.zeros((m * n, m * n), dtype=torch.bool, device=device)
        for dx, dy in offsets:
            big[dy * n:(dy + 1) * n, dx * n:(dx + 1) * n] = mask
        mask = big
    n = mask.shape[0]
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    a = torch.zeros((n, n), dtype=torch.uint8, device=device)
    rows = max(1, (1 << 28) // n)
    for y0 in range(0, n, rows):
        y1 = min(n, y0 + rows)
        alive = torch.rand((y1 - y0, n), generator=g, device=device) < p
        a[y0:y1] = (alive & mask[y0:y1]).to(torch.uint8)
    del mask
    return a


@dataclass
class InstanceSpec:
    """One gasket of a batch: level r, Bernoulli p, state seed."""
    r: int
    p: float
    seed: int

    def state(self) -> np.ndarray:
        return bernoulli_state(self.r, self.p, self.seed)


def batch_specs(count: int = 512, r_lo: int = 6, r_hi: int = 13,
                seed: int = DEFAULT_SEED) -> List[InstanceSpec]:
    """Uneven batch: r ~ U{r_lo..r_hi}, p ~ U[0.2, 0.8], instance i seeded seed+i."""
    rng = np.random.default_rng(seed)
    rs = rng.integers(r_lo, r_hi + 1, size=count)
    ps = rng.uniform(0.2, 0.8, size=count)
    return [InstanceSpec(int(rs[i]), float(ps[i]), seed + i) for i in range(count)]


@dataclass
class RequestSpec:
    """One serving request: arrival time (s), level r, CA steps, state seed."""
    rid: int
    arrival: float
    r: int
    steps: int
    seed: int

    def state(self) -> np.ndarray:
        return bernoulli_state(self.r, 0.5, self.seed)


def poisson_requests(qps: float, count: int, r_lo: int = 8, r_hi: int = 15,
                     steps_lo: int = 10, steps_hi: int = 200,
                     seed: int = DEFAULT_SEED) -> List[RequestSpec]:
    """Poisson arrivals at rate `qps`; r ~ U{r_lo..r_hi}, steps ~ U{steps_lo..steps_hi}."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    rs = rng.integers(r_lo, r_hi + 1, size=count)
    st = rng.integers(steps_lo, steps_hi + 1, size=count)
    return [RequestSpec(i, float(t[i]), int(rs[i]), int(st[i]), seed + 1000 + i)
            for i in range(count)]


_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64_at(seed: int, counters) -> np.ndarray:
    """Outputs number `counters` (from 0) of SplitMix64 seeded with `seed`:
    the seed plus (c + 1) golden-ratio gammas, through the generator's
    finaliser; uint64, arithmetic modulo 2^64."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & ((1 << 64) - 1)) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


def counter_threshold(p: float) -> int:
    """The uint64 threshold under which an output makes a cell alive with
    probability p."""
    return min(int(p * 2.0 ** 64), (1 << 64) - 1)


def counter_region(r: int, x0: int, y0: int, w: int, h: int, p: float = 0.5,
                   seed: int = DEFAULT_SEED) -> np.ndarray:
    """uint8 h x w block of the counter-based state at columns x0.. and rows
    y0..: 1 on the gasket cells whose output is below the threshold, 0 on the
    other cells and outside the n x n grid."""
    n = 1 << r
    x = np.arange(x0, x0 + w, dtype=np.int64)[None, :]
    y = np.arange(y0, y0 + h, dtype=np.int64)[:, None]
    inside = (x >= 0) & (x < n) & (y >= 0) & (y < n)
    xs, ys = np.clip(x, 0, n - 1), np.clip(y, 0, n - 1)
    on = inside & ((xs & ys) == 0)
    ctr = (ys.astype(np.uint64) << np.uint64(32)) | xs.astype(np.uint64)
    alive = splitmix64_at(seed, ctr) < np.uint64(counter_threshold(p))
    return (on & alive).astype(np.uint8)


def counter_state(r: int, p: float = 0.5, seed: int = DEFAULT_SEED) -> np.ndarray:
    """The whole n x n counter-based state (small r only)."""
    n = 1 << r
    return counter_region(r, 0, 0, n, n, p, seed)
