"""Thin ctypes binding of libsg (``include/sg.h``) over torch device tensors.

Each function has the name and argument order of its C entry point; it only
checks and marshals arguments (tensor device, dtype, shape, contiguity) and
passes raw device pointers plus the current HIP stream.  All computation runs
in the HIP kernels of ``libsg.so``; there is no CPU fallback: if the library
is missing or the device is not a GPU, the call raises.
"""
import ctypes
import os
from typing import Optional, Tuple

import torch  # must load before libsg so both share torch's HIP runtime

from . import build as _build

SG_OK, SG_EINVAL, SG_EALIAS, SG_EHIP, SG_ENOMEM = 0, -1, -2, -3, -4
SG_MAP_LAMBDA, SG_MAP_BBOX = 0, 1
SG_INTRA_SUBBOX, SG_INTRA_UNROLL, SG_INTRA_LUT = 0, 1, 2
INTRA = {"subbox": SG_INTRA_SUBBOX, "unroll": SG_INTRA_UNROLL, "lut": SG_INTRA_LUT}
SG_MAX_R, SG_MAX_RHO = 20, 256
SG_PASS_STATIC_MAX = 4096  # items of sg_pass_run_static
MAPS = {"lambda": SG_MAP_LAMBDA, "bbox": SG_MAP_BBOX}

class sg_tune(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("threads", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class sg_gasket(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("r", ctypes.c_int32), ("steps", ctypes.c_int32)]


class sg_pass_item(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("r", ctypes.c_int32), ("steps", ctypes.c_int32)]


SG_FRAC_MAX_K = 16


class sg_fractal(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("dx", ctypes.c_uint8 * SG_FRAC_MAX_K), ("dy", ctypes.c_uint8 * SG_FRAC_MAX_K)]


def fractal(m: int, offsets) -> sg_fractal:
    """A fractal keeping the m x m sub-squares at `offsets` [(dx, dy), ...]."""
    f = sg_fractal()
    f.m, f.k = m, len(offsets)
    for i, (a, b) in enumerate(offsets):
        f.dx[i], f.dy[i] = a, b
    return f


class sg_server_done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("result", ctypes.c_void_p), ("rejected", ctypes.c_int32)]


class sg_server_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("rounds", "passes", "completed", "rejected", "cell_steps", "max_resident_bytes",
                 "max_active", "queued", "active", "resident_bytes", "allocated_bytes",
                 "max_allocated_bytes", "transferring")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class sg_server_request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("r", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("init", ctypes.c_void_p), ("out", ctypes.c_void_p), ("host", ctypes.c_int32)]


# Every symbol declared in include/sg.h, with its ctypes signature.
_u64p = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p
_tunep = ctypes.POINTER(sg_tune)
_SIGNATURES = {
    "sg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sg_last_hip_error": (ctypes.c_char_p, []),
    "sg_version": (ctypes.c_int, []),
    "sg_lambda_grid": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _u64p, _u64p]),
    "sg_block_count": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64p]),
    "sg_map_lambda": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "sg_map_bbox": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "sg_write_pass": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_uint8, ctypes.c_void_p]),
    "sg_write_pass_intra": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_uint8, ctypes.c_void_p]),
    "sg_ca_step": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "sg_ca_steps": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "sg_diffuse_step": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "sg_diffuse_steps": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "sg_map_lambda_inverse": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "sg_compact_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _u64p]),
    "sg_compact_init_bernoulli": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                                  ctypes.c_uint64, _vp, _vp]),
    "sg_compact_pack": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "sg_compact_unpack": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "sg_ca_steps_compact": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "sg_block_count_rect": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           _u64p]),
    "sg_map_lambda_rect": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "sg_write_pass_rect": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_uint8, ctypes.c_void_p]),
    "sg_frac_block_count": (ctypes.c_int, [ctypes.POINTER(sg_fractal), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, _u64p]),
    "sg_frac_map": (ctypes.c_int, [ctypes.POINTER(sg_fractal), ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "sg_frac_write": (ctypes.c_int, [ctypes.POINTER(sg_fractal), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_uint8, ctypes.c_void_p]),
    "sg_frac_life_step": (ctypes.c_int, [ctypes.POINTER(sg_fractal), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "sg_server_create": (ctypes.c_int, [_tunep, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_void_p, ctypes.POINTER(_vp)]),
    "sg_server_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.c_int]),
    "sg_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_uint64]),
    "sg_server_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sg_server_done), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]),
    "sg_ca_steps_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]),
    "sg_server_submit_host": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "sg_server_set_max_active": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sg_server_set_transfer_window": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sg_server_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sg_server_request),
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "sg_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sg_server_stats)]),
    "sg_server_destroy": (None, [ctypes.c_void_p]),
    "sg_tune_default": (ctypes.c_int, [_tunep]),
    "sg_batch_create": (ctypes.c_int, [ctypes.POINTER(sg_gasket), ctypes.c_int, _tunep,
                                       ctypes.POINTER(_vp)]),
    "sg_batch_run": (ctypes.c_int, [_vp, _vp]),
    "sg_batch_run_eager": (ctypes.c_int, [_vp, _vp]),
    "sg_batch_stats": (ctypes.c_int, [_vp, _u64p, _u64p]),
    "sg_batch_destroy": (None, [_vp]),
    "sg_batch_autotune": (ctypes.c_int, [ctypes.POINTER(sg_gasket), ctypes.c_int, _tunep,
                                         ctypes.POINTER(ctypes.c_float), _vp]),
    "sg_pass_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "sg_pass_run": (ctypes.c_int, [_vp, ctypes.POINTER(sg_pass_item), ctypes.c_int, _tunep, _vp]),
    "sg_pass_ctx_destroy": (None, [_vp]),
    "sg_pass_run_static": (ctypes.c_int, [ctypes.POINTER(sg_pass_item), ctypes.c_int, _tunep, _vp]),
}


class SgError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib
        msg = lib.sg_strerror(code).decode() if lib is not None else str(code)
        if code == SG_EHIP and lib is not None:
            msg += f" ({lib.sg_last_hip_error().decode()})"
        super().__init__(f"{where}: {msg} [status {code}]")
        self.code = code


_lib = None


def library_path() -> str:
    """libsg.so in the package, or the build named by SG_LIB_PATH (another
    build of the same sources, e.g. with the host code sanitized)."""
    return os.environ.get("SG_LIB_PATH") or _build.LIB


def load() -> ctypes.CDLL:
    """Load libsg.so (building it first only if it has never been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if path == _build.LIB and not os.path.exists(path):
        _build.build()
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int, where: str):
    if code != SG_OK:
        raise SgError(code, where)


def _map(m) -> int:
    if isinstance(m, str):
        return MAPS[m]
    return int(m)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype, numel: Optional[int], name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (got {t.device}); libsg has no CPU path")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _n2(r: int) -> int:
    if not 0 <= r <= SG_MAX_R:
        raise SgError(SG_EINVAL, f"r={r}")
    return (1 << r) * (1 << r)


# ---------------------------------------------------------------- host helpers

def sg_lambda_grid(r: int, rho: int) -> Tuple[int, int]:
    W, H = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().sg_lambda_grid(r, rho, ctypes.byref(W), ctypes.byref(H)), "sg_lambda_grid")
    return W.value, H.value


def sg_block_count(map_kind, r: int, rho: int) -> int:
    b = ctypes.c_uint64()
    _check(load().sg_block_count(_map(map_kind), r, rho, ctypes.byref(b)), "sg_block_count")
    return b.value


def sg_version() -> int:
    return load().sg_version()


# ---------------------------------------------------------------- device calls

def sg_map_lambda(r: int, rho: int, d_bxy: torch.Tensor, stream=None) -> torch.Tensor:
    """Fill d_bxy (int32/uint32 tensor of 2*3^r_b elements) with (bx, by) pairs."""
    W, H = sg_lambda_grid(r, rho)
    if d_bxy.dtype not in (torch.int32, torch.uint32):
        raise TypeError("d_bxy must be int32 or uint32")
    p = _dev(d_bxy, d_bxy.dtype, 2 * W * H, "d_bxy")
    _check(load().sg_map_lambda(r, rho, p, _stream(stream)), "sg_map_lambda")
    return d_bxy


def sg_map_bbox(r: int, rho: int, d_mask: torch.Tensor, stream=None) -> torch.Tensor:
    nb = (1 << r) // rho if rho > 0 else 0
    p = _dev(d_mask, torch.uint8, nb * nb, "d_mask")
    _check(load().sg_map_bbox(r, rho, p, _stream(stream)), "sg_map_bbox")
    return d_mask


def sg_write_pass(map_kind, r: int, rho: int, d_a: torch.Tensor, value: int = 1,
                  stream=None) -> torch.Tensor:
    p = _dev(d_a, torch.uint8, _n2(r), "d_a")
    _check(load().sg_write_pass(_map(map_kind), r, rho, p, value, _stream(stream)), "sg_write_pass")
    return d_a


def sg_write_pass_intra(map_kind, intra, r: int, rho: int, d_a: torch.Tensor, value: int = 1,
                        stream=None) -> torch.Tensor:
    """Write pass with intra-block mapping "subbox", "unroll" or "lut"."""
    p = _dev(d_a, torch.uint8, _n2(r), "d_a")
    k = INTRA[intra] if isinstance(intra, str) else int(intra)
    _check(load().sg_write_pass_intra(_map(map_kind), k, r, rho, p, value, _stream(stream)),
           "sg_write_pass_intra")
    return d_a


def sg_ca_step(map_kind, r: int, rho: int, d_in: torch.Tensor, d_out: torch.Tensor,
               stream=None) -> torch.Tensor:
    n2 = _n2(r)
    pi = _dev(d_in, torch.uint8, n2, "d_in")
    po = _dev(d_out, torch.uint8, n2, "d_out")
    _check(load().sg_ca_step(_map(map_kind), r, rho, pi, po, _stream(stream)), "sg_ca_step")
    return d_out


def sg_ca_steps(map_kind, r: int, rho: int, steps: int, d_in: torch.Tensor,
                d_out: torch.Tensor, d_work: Optional[torch.Tensor] = None,
                steps_per_pass: int = 0, stream=None) -> torch.Tensor:
    """`steps` life generations from d_in into d_out (d_work: third buffer)."""
    n2 = _n2(r)
    pi = _dev(d_in, torch.uint8, n2, "d_in")
    po = _dev(d_out, torch.uint8, n2, "d_out")
    pw = _dev(d_work, torch.uint8, n2, "d_work") if d_work is not None else None
    _check(load().sg_ca_steps(_map(map_kind), r, rho, steps, steps_per_pass, pi, po, pw,
                              _stream(stream)), "sg_ca_steps")
    return d_out


def sg_ca_steps_autotune(map_kind, r: int, steps: int, d_in: torch.Tensor, d_out: torch.Tensor,
                         d_work: torch.Tensor, stream=None):
    """The fastest (rho, steps_per_pass) of sg_ca_steps for this gasket and
    its time in ms, timed on these buffers (d_out and d_work are written)."""
    n2 = _n2(r)
    pi = _dev(d_in, torch.uint8, n2, "d_in")
    po = _dev(d_out, torch.uint8, n2, "d_out")
    pw = _dev(d_work, torch.uint8, n2, "d_work")
    rho, spp, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    _check(load().sg_ca_steps_autotune(_map(map_kind), r, steps, pi, po, pw, ctypes.byref(rho),
                                       ctypes.byref(spp), ctypes.byref(ms), _stream(stream)),
           "sg_ca_steps_autotune")
    return rho.value, spp.value, ms.value


def sg_diffuse_step(map_kind, r: int, rho: int, d_in: torch.Tensor, d_out: torch.Tensor,
                    alpha: float = 0.2, stream=None) -> torch.Tensor:
    n2 = _n2(r)
    pi = _dev(d_in, torch.float32, n2, "d_in")
    po = _dev(d_out, torch.float32, n2, "d_out")
    _check(load().sg_diffuse_step(_map(map_kind), r, rho, pi, po, alpha, _stream(stream)),
           "sg_diffuse_step")
    return d_out


def sg_diffuse_steps(map_kind, r: int, rho: int, steps: int, d_in: torch.Tensor,
                     d_out: torch.Tensor, d_work: Optional[torch.Tensor] = None,
                     alpha: float = 0.2, steps_per_pass: int = 0, stream=None) -> torch.Tensor:
    """`steps` diffusion steps from d_in into d_out (d_work: third buffer)."""
    n2 = _n2(r)
    pi = _dev(d_in, torch.float32, n2, "d_in")
    po = _dev(d_out, torch.float32, n2, "d_out")
    pw = _dev(d_work, torch.float32, n2, "d_work") if d_work is not None else None
    _check(load().sg_diffuse_steps(_map(map_kind), r, rho, steps, steps_per_pass, pi, po, pw,
                                   alpha, _stream(stream)), "sg_diffuse_steps")
    return d_out


def sg_map_lambda_inverse(r: int, rho: int, d_omega: torch.Tensor, stream=None) -> torch.Tensor:
    """d_omega (int32, n_b*n_b): omega of each block, -1 off the gasket."""
    nb = (1 << r) // rho if rho > 0 else 0
    p = _dev(d_omega, torch.int32, nb * nb, "d_omega")
    _check(load().sg_map_lambda_inverse(r, rho, p, _stream(stream)), "sg_map_lambda_inverse")
    return d_omega


def sg_compact_bytes(r: int, rho: int) -> int:
    b = ctypes.c_uint64()
    _check(load().sg_compact_bytes(r, rho, ctypes.byref(b)), "sg_compact_bytes")
    return b.value


def bernoulli_threshold(p: float) -> int:
    """The uint64 threshold under which a SplitMix64 output makes a cell alive
    with probability p."""
    if not 0.0 <= p <= 1.0:
        raise ValueError(f"p={p} outside [0, 1]")
    return min(int(p * 2.0 ** 64), (1 << 64) - 1)


def sg_compact_init_bernoulli(r: int, rho: int, seed: int, p: float, d_compact: torch.Tensor,
                              stream=None) -> torch.Tensor:
    pc = _dev(d_compact, torch.uint8, sg_compact_bytes(r, rho), "d_compact")
    _check(load().sg_compact_init_bernoulli(r, rho, seed & ((1 << 64) - 1), bernoulli_threshold(p),
                                            pc, _stream(stream)), "sg_compact_init_bernoulli")
    return d_compact


def sg_compact_pack(r: int, rho: int, d_dense: torch.Tensor, d_compact: torch.Tensor,
                    stream=None) -> torch.Tensor:
    pd = _dev(d_dense, torch.uint8, _n2(r), "d_dense")
    pc = _dev(d_compact, torch.uint8, sg_compact_bytes(r, rho), "d_compact")
    _check(load().sg_compact_pack(r, rho, pd, pc, _stream(stream)), "sg_compact_pack")
    return d_compact


def sg_compact_unpack(r: int, rho: int, d_compact: torch.Tensor, d_dense: torch.Tensor,
                      stream=None) -> torch.Tensor:
    pc = _dev(d_compact, torch.uint8, sg_compact_bytes(r, rho), "d_compact")
    pd = _dev(d_dense, torch.uint8, _n2(r), "d_dense")
    _check(load().sg_compact_unpack(r, rho, pc, pd, _stream(stream)), "sg_compact_unpack")
    return d_dense


def sg_ca_steps_compact(r: int, rho: int, steps: int, d_in: torch.Tensor, d_out: torch.Tensor,
                        d_work: Optional[torch.Tensor] = None, steps_per_pass: int = 0,
                        stream=None) -> torch.Tensor:
    size = sg_compact_bytes(r, rho)
    pi = _dev(d_in, torch.uint8, size, "d_in")
    po = _dev(d_out, torch.uint8, size, "d_out")
    pw = _dev(d_work, torch.uint8, size, "d_work") if d_work is not None else None
    _check(load().sg_ca_steps_compact(r, rho, steps, steps_per_pass, pi, po, pw, _stream(stream)),
           "sg_ca_steps_compact")
    return d_out


def sg_frac_block_count(f: sg_fractal, map_kind, r: int, rho: int) -> int:
    b = ctypes.c_uint64()
    _check(load().sg_frac_block_count(ctypes.byref(f), _map(map_kind), r, rho, ctypes.byref(b)),
           "sg_frac_block_count")
    return b.value


def _frac_n2(f: sg_fractal, r: int) -> int:
    return (f.m ** r) ** 2


def sg_frac_map(f: sg_fractal, r: int, rho: int, d_bxy: torch.Tensor, stream=None) -> torch.Tensor:
    """d_bxy: int32 CUDA tensor of 2 k^r_b elements (bx, by pairs)."""
    count = sg_frac_block_count(f, "lambda", r, rho)
    p = _dev(d_bxy, torch.int32, 2 * count, "d_bxy")
    _check(load().sg_frac_map(ctypes.byref(f), r, rho, p, _stream(stream)), "sg_frac_map")
    return d_bxy


def sg_frac_write(f: sg_fractal, map_kind, r: int, rho: int, d_a: torch.Tensor, value: int,
                  stream=None) -> torch.Tensor:
    p = _dev(d_a, torch.uint8, _frac_n2(f, r), "d_a")
    _check(load().sg_frac_write(ctypes.byref(f), _map(map_kind), r, rho, p, value, _stream(stream)),
           "sg_frac_write")
    return d_a


def sg_frac_life_step(f: sg_fractal, map_kind, r: int, rho: int, d_in: torch.Tensor,
                      d_out: torch.Tensor, stream=None) -> torch.Tensor:
    pi = _dev(d_in, torch.uint8, _frac_n2(f, r), "d_in")
    po = _dev(d_out, torch.uint8, _frac_n2(f, r), "d_out")
    _check(load().sg_frac_life_step(ctypes.byref(f), _map(map_kind), r, rho, pi, po,
                                    _stream(stream)), "sg_frac_life_step")
    return d_out


def sg_block_count_rect(map_kind, r: int, rho_x: int, rho_y: int) -> int:
    b = ctypes.c_uint64()
    _check(load().sg_block_count_rect(_map(map_kind), r, rho_x, rho_y, ctypes.byref(b)),
           "sg_block_count_rect")
    return b.value


def sg_map_lambda_rect(r: int, rho_x: int, rho_y: int, d_bxy: torch.Tensor,
                       stream=None) -> torch.Tensor:
    count = sg_block_count_rect("lambda", r, rho_x, rho_y)
    p = _dev(d_bxy, torch.int32, 2 * count, "d_bxy")
    _check(load().sg_map_lambda_rect(r, rho_x, rho_y, p, _stream(stream)), "sg_map_lambda_rect")
    return d_bxy


def sg_write_pass_rect(map_kind, r: int, rho_x: int, rho_y: int, d_a: torch.Tensor, value: int,
                       stream=None) -> torch.Tensor:
    p = _dev(d_a, torch.uint8, _n2(r), "d_a")
    _check(load().sg_write_pass_rect(_map(map_kind), r, rho_x, rho_y, p, value, _stream(stream)),
           "sg_write_pass_rect")
    return d_a
