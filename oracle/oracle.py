"""ctypes front end of the C oracle in ``sg_oracle.c``.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function takes and
returns NumPy arrays; the arithmetic lives in the C file, where each routine
cites the passage of the paper it follows.  No function here calls the HIP
library.

Parity status: every function is pinned by an independent test under
``tests/`` (closed forms, exhaustive enumeration, textbook patterns,
hand-derived worked examples, an independent sparse formulation).
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None

_i64 = ctypes.c_int64
_int = ctypes.c_int
_ptr = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("SG_ORACLE_LIB") or build_oracle.LIB  # another build, e.g. sanitized
    if path == build_oracle.LIB and not os.path.exists(path):
        build_oracle.build()
    lib = ctypes.CDLL(path)
    sig = {
        "sgo_member": (_int, [_i64, _i64]),
        "sgo_member_paper": (_int, [_i64, _i64, _i64]),
        "sgo_count_cells": (_i64, [_int]),
        "sgo_threads": (_int, []),
        "sgo_set_threads": (None, [_int]),
        "sgo_lambda_grid": (None, [_int, _ptr, _ptr]),
        "sgo_lambda": (None, [_int, _i64, _i64, _ptr, _ptr]),
        "sgo_map_lambda": (None, [_int, _ptr]),
        "sgo_map_bbox": (None, [_int, _int, _ptr]),
        "sgo_write_pass": (None, [_int, ctypes.c_uint8, _ptr]),
        "sgo_life_step_plain": (None, [_i64, _i64, _ptr, _ptr]),
        "sgo_life_step": (None, [_int, _ptr, _ptr]),
        "sgo_life_step_sparse": (None, [_int, _ptr, _ptr]),
        "sgo_life_window": (None, [_int, _ptr, _i64, _i64, _i64, _i64, _int, _ptr]),
        "sgo_life_region": (None, [_i64, _i64, _i64, _i64, _int, _ptr]),
        "sgo_row_checksums": (None, [_int, _ptr, _ptr, _ptr]),
        "sgo_diffuse_step": (None, [_int, _ptr, _ptr, ctypes.c_double]),
        "sgo_gasket_graph": (None, [_int, _ptr, _ptr]),
        "sgo_diffuse_step_graph": (None, [_i64, _ptr, _ptr, _ptr, ctypes.c_double]),
        "sgo_diffuse_window": (None, [_int, _ptr, _i64, _i64, _i64, _i64, _int,
                                      ctypes.c_double, _ptr]),
        "sgo_map_lambda_rect": (None, [_int, _int, _int, _ptr]),
        "sgo_map_bbox_rect": (None, [_int, _int, _int, _ptr]),
        "sgo_frac_member": (_int, [_int, _int, _ptr, _ptr, _int, _i64, _i64]),
        "sgo_frac_lambda": (None, [_int, _int, _ptr, _ptr, _int, _i64, _i64, _ptr, _ptr]),
        "sgo_frac_map": (None, [_int, _int, _ptr, _ptr, _int, _ptr]),
        "sgo_frac_write": (None, [_int, _int, _ptr, _ptr, _int, ctypes.c_uint8, _ptr]),
        "sgo_frac_write_rows": (None, [_int, _int, _ptr, _ptr, _int, ctypes.c_uint8, _i64, _i64,
                                       _ptr]),
        "sgo_frac_life_step": (None, [_int, _int, _ptr, _ptr, _int, _ptr, _ptr]),
        "sgo_frac_life_window": (None, [_int, _int, _ptr, _ptr, _int, _ptr, _i64, _i64, _i64,
                                        _i64, _int, _ptr]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_state(r: int, a: np.ndarray, dtype):
    n = 1 << r
    if a.dtype != dtype or a.shape != (n, n):
        raise ValueError(f"expected {dtype} array of shape ({n}, {n}), got {a.dtype} {a.shape}")
    return np.ascontiguousarray(a)


def threads() -> int:
    """Threads the oracle's OpenMP row loops use."""
    return int(_load().sgo_threads())


def set_threads(t: int) -> None:
    """Threads for the OpenMP row loops from now on."""
    _load().sgo_set_threads(int(t))


# ---------------------------------------------------------------- membership

def member(x: int, y: int) -> bool:
    """Build-frame membership (x & y) == 0."""
    return bool(_load().sgo_member(x, y))


def member_paper(n: int, x: int, y: int) -> bool:
    """Paper-frame membership x & (n-1-y) == 0 (Section III-D)."""
    return bool(_load().sgo_member_paper(n, x, y))


def count_cells(r: int) -> int:
    """Gasket cells in the 2^r x 2^r array, by scanning every cell."""
    return int(_load().sgo_count_cells(r))


# ---------------------------------------------------------------- lambda

def lambda_grid(rb: int):
    """(W, H) of the launch orthotope for block level r_b (Lemma 2, Eq. 4)."""
    W, H = ctypes.c_int64(), ctypes.c_int64()
    _load().sgo_lambda_grid(rb, ctypes.byref(W), ctypes.byref(H))
    return W.value, H.value


def lambda_paper(rb: int, wx: int, wy: int):
    """lambda(omega) in the paper frame (Eq. 4-10)."""
    lx, ly = ctypes.c_int64(), ctypes.c_int64()
    _load().sgo_lambda(rb, wx, wy, ctypes.byref(lx), ctypes.byref(ly))
    return lx.value, ly.value


def map_lambda(rb: int) -> np.ndarray:
    """Build-frame table: row i = (bx, by) of omega with linear index i."""
    W, H = lambda_grid(rb)
    out = np.zeros((W * H, 2), dtype=np.uint32)
    _load().sgo_map_lambda(rb, _p(out))
    return out


def map_bbox(r: int, rho: int) -> np.ndarray:
    """Bounding-box block mask, shape (n_b, n_b), indexed [by, bx]."""
    nb = (1 << r) // rho
    out = np.zeros((nb, nb), dtype=np.uint8)
    _load().sgo_map_bbox(r, rho, _p(out))
    return out


def map_lambda_rect(r: int, rho_x: int, rho_y: int) -> np.ndarray:
    """Rows (bx, by) of the map onto rho_x x rho_y blocks (powers of two)."""
    a, b = rho_x.bit_length() - 1, rho_y.bit_length() - 1
    hi, d = max(a, b), abs(a - b)
    out = np.zeros((3 ** (r - hi) * 2 ** d, 2), dtype=np.uint32)
    _load().sgo_map_lambda_rect(r, a, b, _p(out))
    return out


def map_bbox_rect(r: int, rho_x: int, rho_y: int) -> np.ndarray:
    """Bounding-box block mask, shape (n/rho_y, n/rho_x), indexed [by, bx]."""
    n = 1 << r
    out = np.zeros((n // rho_y, n // rho_x), dtype=np.uint8)
    _load().sgo_map_bbox_rect(r, rho_x, rho_y, _p(out))
    return out


# ---------------------------------------------------------------- passes

def write_pass(r: int, value: int) -> np.ndarray:
    n = 1 << r
    a = np.zeros((n, n), dtype=np.uint8)
    _load().sgo_write_pass(r, value, _p(a))
    return a


def life_step_plain(a: np.ndarray) -> np.ndarray:
    """Plain B3/S23 on an h x w grid with dead outside cells."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    h, w = a.shape
    out = np.empty_like(a)
    _load().sgo_life_step_plain(w, h, _p(a), _p(out))
    return out


def life_step(r: int, a: np.ndarray) -> np.ndarray:
    a = _check_state(r, a, np.uint8)
    out = np.empty_like(a)
    _load().sgo_life_step(r, _p(a), _p(out))
    return out


def life_steps(r: int, a: np.ndarray, steps: int) -> np.ndarray:
    a = _check_state(r, a, np.uint8)
    cur, nxt = a.copy(), np.empty_like(a)
    lib = _load()
    for _ in range(steps):
        lib.sgo_life_step(r, _p(cur), _p(nxt))
        cur, nxt = nxt, cur
    return cur


def life_step_sparse(r: int, a: np.ndarray) -> np.ndarray:
    """One step visiting only the gasket's cells (same result as life_step)."""
    a = _check_state(r, a, np.uint8)
    out = np.zeros_like(a)
    _load().sgo_life_step_sparse(r, _p(a), _p(out))
    return out


def life_steps_sparse(r: int, a: np.ndarray, steps: int, snapshots=()) -> np.ndarray:
    """`steps` steps visiting only the gasket's cells (same result as
    life_steps).  With `snapshots`, returns {t: state after t steps} for each
    t listed (0 <= t <= steps) instead."""
    a = _check_state(r, a, np.uint8)
    cur = a.copy()
    nxt = np.zeros_like(a)  # cells off the gasket stay 0
    lib = _load()
    want = sorted(set(int(t) for t in snapshots))
    shots = {}
    if 0 in want:
        shots[0] = cur.copy()
    for t in range(1, steps + 1):
        lib.sgo_life_step_sparse(r, _p(cur), _p(nxt))
        cur, nxt = nxt, cur
        if t in want:
            shots[t] = cur.copy() if t != steps else cur
    return shots if want else cur


def life_window(r: int, a: np.ndarray, x0: int, y0: int, w: int, h: int,
                steps: int) -> np.ndarray:
    """State after `steps` on the window [x0, x0+w) x [y0, y0+h)."""
    a = _check_state(r, a, np.uint8)
    out = np.zeros((h, w), dtype=np.uint8)
    _load().sgo_life_window(r, _p(a), x0, y0, w, h, steps, _p(out))
    return out


def life_region(gx0: int, gy0: int, a: np.ndarray, steps: int) -> np.ndarray:
    """`steps` gasket life steps on the region of the grid whose top-left cell
    is (gx0, gy0), held in `a`, with every cell outside it taken as dead (the
    region must lie inside the grid; cells within Chebyshev distance `steps`
    of an edge where the region is cut short of the grid's come out wrong)."""
    out = np.ascontiguousarray(a, dtype=np.uint8).copy()
    h, w = out.shape
    _load().sgo_life_region(gx0, gy0, w, h, steps, _p(out))
    return out


def row_checksums(r: int, a: np.ndarray):
    a = _check_state(r, a, np.uint8)
    n = 1 << r
    xr = np.zeros(n, dtype=np.uint8)
    pop = np.zeros(n, dtype=np.uint32)
    _load().sgo_row_checksums(r, _p(a), _p(xr), _p(pop))
    return xr, pop


def diffuse_step(r: int, u: np.ndarray, alpha: float = 0.2) -> np.ndarray:
    u = _check_state(r, u, np.float64)
    out = np.empty_like(u)
    _load().sgo_diffuse_step(r, _p(u), _p(out), alpha)
    return out


def diffuse_steps(r: int, u0: np.ndarray, steps: int, alpha: float = 0.2) -> np.ndarray:
    """FP64 diffusion from an FP32 (or FP64) initial state."""
    cur = np.ascontiguousarray(u0, dtype=np.float64).copy()
    _check_state(r, cur, np.float64)
    nxt = np.empty_like(cur)
    lib = _load()
    for _ in range(steps):
        lib.sgo_diffuse_step(r, _p(cur), _p(nxt), alpha)
        cur, nxt = nxt, cur
    return cur


def gasket_graph(r: int):
    """The gasket's cells in row-major order and their 4-neighbours:
    pos[i] = y * n + x of cell i; nb[i, k] = the number of its neighbour
    k = W, E, N, S, or -1 (off the grid or off the gasket).  r <= 19."""
    if not 0 <= r <= 19:
        raise ValueError("gasket_graph numbers cells in int32: r <= 19")
    N = 3 ** r
    pos = np.empty(N, dtype=np.int64)
    nb = np.empty(4 * N, dtype=np.int32)
    _load().sgo_gasket_graph(r, _p(pos), _p(nb))
    return pos, nb.reshape(N, 4)


def diffuse_steps_graph(r: int, u0: np.ndarray, steps: int, alpha: float = 0.2,
                        snapshots=()):
    """FP64 diffusion over the gasket graph from an n x n field (FP32 or
    FP64): the sum of diffuse_step term for term, so the gasket cells' values
    are identical to diffuse_steps'.  Returns (pos, u) with u[i] the value of
    the cell at flat position pos[i] after `steps` steps, or (pos, {t: u})
    for the steps listed in `snapshots`."""
    n = 1 << r
    u0 = np.ascontiguousarray(u0)
    if u0.shape != (n, n):
        raise ValueError(f"expected shape ({n}, {n})")
    pos, nb = gasket_graph(r)
    cur = u0.reshape(-1)[pos].astype(np.float64)
    nxt = np.empty_like(cur)
    lib = _load()
    want = sorted(set(int(t) for t in snapshots))
    shots = {}
    if 0 in want:
        shots[0] = cur.copy()
    for t in range(1, steps + 1):
        lib.sgo_diffuse_step_graph(len(cur), _p(nb), _p(cur), _p(nxt), alpha)
        cur, nxt = nxt, cur
        if t in want:
            shots[t] = cur.copy()
    return pos, (shots if want else cur)


def diffuse_window(r: int, u0: np.ndarray, x0: int, y0: int, w: int, h: int,
                   steps: int, alpha: float = 0.2) -> np.ndarray:
    u0 = _check_state(r, u0, np.float32)
    out = np.zeros((h, w), dtype=np.float64)
    _load().sgo_diffuse_window(r, _p(u0), x0, y0, w, h, steps, alpha, _p(out))
    return out


# ---------------------------------------------------------------- other fractals F^{k,1/m}

class Fractal:
    """k kept sub-squares of an m x m subdivision, at offsets (dx[i], dy[i])
    listed in the order the map's digit enumerates them (build frame)."""

    def __init__(self, m: int, offsets):
        self.m = int(m)
        self.offsets = [(int(a), int(b)) for a, b in offsets]
        self.k = len(self.offsets)
        self._dx = np.array([a for a, _ in self.offsets], dtype=np.int32)
        self._dy = np.array([b for _, b in self.offsets], dtype=np.int32)

    def args(self):
        return (self.m, self.k, _p(self._dx), _p(self._dy))

    def n(self, r: int) -> int:
        return self.m ** r


GASKET = Fractal(2, [(0, 1), (0, 0), (1, 0)])  # beta = 0, 1, 2 after the build-frame reflection
CARPET = Fractal(3, [(x, y) for y in range(3) for x in range(3) if (x, y) != (1, 1)])
VICSEK = Fractal(3, [(1, 0), (0, 1), (1, 1), (2, 1), (1, 2)])


def frac_member(f: Fractal, r: int, x: int, y: int) -> bool:
    return bool(_load().sgo_frac_member(*f.args(), r, x, y))


def frac_lambda(f: Fractal, rb: int, wx: int, wy: int):
    lx, ly = ctypes.c_int64(), ctypes.c_int64()
    _load().sgo_frac_lambda(*f.args(), rb, wx, wy, ctypes.byref(lx), ctypes.byref(ly))
    return lx.value, ly.value


def frac_map(f: Fractal, rb: int) -> np.ndarray:
    """Rows (bx, by) of the generalised map, linear index wy * W + wx."""
    out = np.zeros((f.k ** rb, 2), dtype=np.uint32)
    _load().sgo_frac_map(*f.args(), rb, _p(out))
    return out


def frac_write(f: Fractal, r: int, value: int) -> np.ndarray:
    n = f.n(r)
    a = np.zeros((n, n), dtype=np.uint8)
    _load().sgo_frac_write(*f.args(), r, value, _p(a))
    return a


def frac_write_rows(f: Fractal, r: int, value: int, y0: int, rows: int) -> np.ndarray:
    """Rows [y0, y0 + rows) of frac_write(f, r, value)."""
    n = f.n(r)
    out = np.zeros((rows, n), dtype=np.uint8)
    _load().sgo_frac_write_rows(*f.args(), r, value, y0, rows, _p(out))
    return out


def frac_life_steps(f: Fractal, r: int, a: np.ndarray, steps: int) -> np.ndarray:
    n = f.n(r)
    assert a.shape == (n, n) and a.dtype == np.uint8
    cur = np.ascontiguousarray(a).copy()
    nxt = np.zeros_like(cur)
    for _ in range(steps):
        _load().sgo_frac_life_step(*f.args(), r, _p(cur), _p(nxt))
        cur, nxt = nxt, cur
    return cur


def frac_life_window(f: Fractal, r: int, a: np.ndarray, x0: int, y0: int, w: int, h: int,
                     steps: int) -> np.ndarray:
    """State after `steps` fractal life steps on the window [x0, x0+w) x [y0, y0+h)."""
    n = f.n(r)
    a = np.ascontiguousarray(a)
    assert a.shape == (n, n) and a.dtype == np.uint8
    out = np.zeros((h, w), dtype=np.uint8)
    _load().sgo_frac_life_window(*f.args(), r, _p(a), x0, y0, w, h, steps, _p(out))
    return out
