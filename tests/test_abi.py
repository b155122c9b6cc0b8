"""CPU tests of the C ABI: the library loads, exports every symbol that
``include/sg.h`` declares, and rejects invalid arguments on the host before any
HIP call (so no GPU is needed).  Host-only helpers are checked against the
closed forms of Lemma 1-2 and Theorem 2."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SG_API\s+[\w\s\*]+?\b(sg_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1706_04552_amd import sg
    return sg.load()


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ["sg_map_lambda", "sg_map_bbox", "sg_write_pass", "sg_ca_step",
                 "sg_diffuse_step", "sg_strerror"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    from paper_1706_04552_amd import sg
    out = subprocess.run(["nm", "-D", "--defined-only", sg.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(sg_\w+)", out))
    for name in declared_symbols():
        assert name in exported, name
        getattr(lib, name)
    # nothing else leaks from the library's C namespace
    assert exported == set(declared_symbols())


def test_binding_covers_every_declared_symbol():
    from paper_1706_04552_amd import sg
    assert set(sg._SIGNATURES) == set(declared_symbols())


def test_strerror(lib):
    from paper_1706_04552_amd import sg
    for code in (sg.SG_OK, sg.SG_EINVAL, sg.SG_EALIAS, sg.SG_EHIP, sg.SG_ENOMEM, -99):
        assert lib.sg_strerror(code)
    assert b"overlap" in lib.sg_strerror(sg.SG_EALIAS)


@pytest.mark.parametrize("r,rho", [(0, 1), (1, 2), (5, 1), (8, 16), (10, 32), (16, 4), (20, 1)])
def test_lambda_grid_closed_form(r, rho):
    from paper_1706_04552_amd import sg
    rb = r - (rho.bit_length() - 1)
    W, H = sg.sg_lambda_grid(r, rho)
    assert (W, H) == (3 ** (rb // 2), 3 ** ((rb + 1) // 2))
    assert sg.sg_block_count("lambda", r, rho) == 3 ** rb
    assert sg.sg_block_count("bbox", r, rho) == 4 ** rb


@pytest.mark.parametrize("r,rho", [(-1, 1), (21, 1), (3, 16), (5, 3), (5, 0), (8, 512), (7, 256), (8, -4)])
def test_bad_shapes_are_rejected(lib, r, rho):
    from paper_1706_04552_amd import sg
    W, H, b = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    fake = ctypes.c_void_p(0x1000)
    assert lib.sg_lambda_grid(r, rho, ctypes.byref(W), ctypes.byref(H)) == sg.SG_EINVAL
    assert lib.sg_block_count(0, r, rho, ctypes.byref(b)) == sg.SG_EINVAL
    assert lib.sg_map_lambda(r, rho, fake, None) == sg.SG_EINVAL
    assert lib.sg_map_bbox(r, rho, fake, None) == sg.SG_EINVAL
    assert lib.sg_write_pass(0, r, rho, fake, 1, None) == sg.SG_EINVAL
    assert lib.sg_ca_step(0, r, rho, fake, ctypes.c_void_p(0x7000000000), None) == sg.SG_EINVAL
    assert lib.sg_diffuse_step(0, r, rho, fake, ctypes.c_void_p(0x7000000000), 0.2, None) == sg.SG_EINVAL


def test_bad_map_kind_and_null_pointers(lib):
    from paper_1706_04552_amd import sg
    a, b = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x7000000000)
    b64 = ctypes.c_uint64()
    assert lib.sg_block_count(2, 4, 2, ctypes.byref(b64)) == sg.SG_EINVAL
    assert lib.sg_block_count(0, 4, 2, None) == sg.SG_EINVAL
    assert lib.sg_ca_step(2, 4, 2, a, b, None) == sg.SG_EINVAL
    assert lib.sg_ca_step(-1, 4, 2, a, b, None) == sg.SG_EINVAL
    assert lib.sg_ca_step(0, 4, 2, None, b, None) == sg.SG_EINVAL
    assert lib.sg_ca_step(0, 4, 2, a, None, None) == sg.SG_EINVAL
    assert lib.sg_diffuse_step(1, 4, 2, None, b, 0.2, None) == sg.SG_EINVAL
    assert lib.sg_write_pass(0, 4, 2, None, 1, None) == sg.SG_EINVAL
    assert lib.sg_map_lambda(4, 2, None, None) == sg.SG_EINVAL
    assert lib.sg_map_lambda(4, 2, ctypes.c_void_p(0x10004), None) == sg.SG_EINVAL  # misaligned
    assert lib.sg_map_bbox(4, 2, None, None) == sg.SG_EINVAL


def test_overlapping_buffers_are_rejected(lib):
    from paper_1706_04552_amd import sg
    r = 4  # n*n = 256 bytes, 1024 for f32
    base = 0x100000
    a = ctypes.c_void_p(base)
    for off in (0, 16, 240):
        assert lib.sg_ca_step(0, r, 4, a, ctypes.c_void_p(base + off), None) == sg.SG_EALIAS
        assert lib.sg_ca_step(1, r, 4, ctypes.c_void_p(base + off), a, None) == sg.SG_EALIAS
    for off in (0, 16, 1008):
        assert lib.sg_diffuse_step(0, r, 4, a, ctypes.c_void_p(base + off), 0.2, None) == sg.SG_EALIAS


def test_python_binding_refuses_cpu_tensors():
    import torch
    from paper_1706_04552_amd import sg
    a = torch.zeros(16 * 16, dtype=torch.uint8)
    b = torch.zeros(16 * 16, dtype=torch.uint8)
    with pytest.raises(ValueError, match="GPU tensor"):
        sg.sg_ca_step("lambda", 4, 4, a, b)
    with pytest.raises(ValueError, match="GPU tensor"):
        sg.sg_write_pass("bbox", 4, 4, a, 1)


def test_misaligned_state_arrays_are_rejected(lib):
    from paper_1706_04552_amd import sg
    a, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000)
    for off in (1, 4, 8):
        m = ctypes.c_void_p(0x7000000000 + off)
        assert lib.sg_ca_step(0, 6, 4, a, m, None) == sg.SG_EINVAL
        assert lib.sg_ca_step(0, 6, 4, m, b, None) == sg.SG_EINVAL
        assert lib.sg_diffuse_step(0, 6, 4, a, m, 0.2, None) == sg.SG_EINVAL
        assert lib.sg_write_pass(1, 6, 4, m, 1, None) == sg.SG_EINVAL


def test_ca_steps_validation(lib):
    from paper_1706_04552_amd import sg
    a, b, w = (ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000),
               ctypes.c_void_p(0x7100000000))
    r = 8  # n*n = 65536 bytes
    # steps_per_pass out of range, or > 1 where the tile side has no temporal blocking
    assert lib.sg_ca_steps(0, r, 64, 10, 33, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 64, 10, -1, a, b, w, None) == sg.SG_EINVAL
    # side 16 takes up to 16 generations per pass, side 32 up to 32; 8 and below none
    assert lib.sg_ca_steps(0, r, 16, 10, 17, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 32, 10, 33, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 8, 10, 2, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 4, 10, 4, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 16, 17, 16, a, b, None, None) == sg.SG_EINVAL  # needs work
    assert lib.sg_ca_steps(0, r, 64, -1, 4, a, b, w, None) == sg.SG_EINVAL
    # more than one pass needs a work buffer, distinct from in and out
    assert lib.sg_ca_steps(0, r, 64, 17, 16, a, b, None, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 16, 2, 1, a, b, None, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps(0, r, 64, 17, 16, a, b, ctypes.c_void_p(0x100000 + 4096), None) == sg.SG_EALIAS
    assert lib.sg_ca_steps(0, r, 64, 17, 16, a, b, ctypes.c_void_p(0x7000000000 + 65520), None) == sg.SG_EALIAS
    assert lib.sg_ca_steps(0, r, 64, 17, 16, a, ctypes.c_void_p(0x100000 + 16), w, None) == sg.SG_EALIAS
    # misaligned work buffer
    assert lib.sg_ca_steps(0, r, 64, 20, 8, a, b, ctypes.c_void_p(0x7100000004), None) == sg.SG_EINVAL


def test_batch_api_validation_on_the_host(lib):
    from paper_1706_04552_amd import sg
    t = sg.sg_tune()
    assert lib.sg_tune_default(ctypes.byref(t)) == sg.SG_OK
    assert (t.rho, t.steps_per_pass, t.threads) == (64, 32, 256)
    assert lib.sg_tune_default(None) == sg.SG_EINVAL
    h = ctypes.c_void_p()
    a, b, w = 0x100000, 0x7000000000, 0x7100000000

    def gaskets(*specs):
        arr = (sg.sg_gasket * len(specs))()
        for i, (r, steps, work) in enumerate(specs):
            arr[i].in_, arr[i].out, arr[i].work = a + i * (1 << 21), b + i * (1 << 21), work
            arr[i].r, arr[i].steps = r, steps
        return arr

    good = sg.sg_tune(64, 16, 0, 256)
    for bad in [sg.sg_tune(32, 16, 0, 256), sg.sg_tune(64, 33, 0, 256), sg.sg_tune(64, 0, 0, 256),
                sg.sg_tune(64, 16, -1, 256), sg.sg_tune(64, 16, 65, 256), sg.sg_tune(64, 16, 0, 128)]:
        assert lib.sg_batch_create(gaskets((8, 10, w)), 1, ctypes.byref(bad), ctypes.byref(h)) == sg.SG_EINVAL
    # gasket smaller than the tile, negative steps, missing work buffer, aliasing
    assert lib.sg_batch_create(gaskets((5, 3, w)), 1, ctypes.byref(good), ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_batch_create(gaskets((8, -1, w)), 1, ctypes.byref(good), ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_batch_create(gaskets((8, 17, None)), 1, ctypes.byref(good), ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_batch_create(gaskets((8, 17, a + 64)), 1, ctypes.byref(good), ctypes.byref(h)) == sg.SG_EALIAS
    assert lib.sg_batch_create(gaskets((8, 3, w)), 0, ctypes.byref(good), ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_batch_create(None, 2, ctypes.byref(good), ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_batch_create(gaskets((8, 3, w)), 1, ctypes.byref(good), None) == sg.SG_EINVAL
    assert not h.value
    assert lib.sg_batch_run(None, None) == sg.SG_EINVAL
    assert lib.sg_batch_run_eager(None, None) == sg.SG_EINVAL
    assert lib.sg_batch_stats(None, None, None) == sg.SG_EINVAL
    lib.sg_batch_destroy(None)
    assert lib.sg_batch_autotune(gaskets((8, 3, w)), 1, None, None, None) == sg.SG_EINVAL
    assert lib.sg_pass_ctx_create(0, ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_pass_ctx_create(4, None) == sg.SG_EINVAL
    item = (sg.sg_pass_item * 1)()
    assert lib.sg_pass_run(None, item, 1, ctypes.byref(good), None) == sg.SG_EINVAL
    lib.sg_pass_ctx_destroy(None)


def test_hip_errors_surface_as_sg_ehip():
    # a fresh process with the library's fault-injection hook switched on: every
    # entry point validates its arguments, then reports SG_EHIP without launching
    code = r"""
import ctypes, sys
sys.path.insert(0, %r)
from paper_1706_04552_amd import sg
lib = sg.load()
a, b, w = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000), ctypes.c_void_p(0x7100000000)
res = [lib.sg_ca_step(0, 8, 16, a, b, None), lib.sg_write_pass(1, 8, 16, a, 1, None),
       lib.sg_diffuse_step(0, 8, 16, a, b, 0.2, None), lib.sg_map_lambda(8, 16, a, None),
       lib.sg_map_bbox(8, 16, a, None), lib.sg_ca_steps(0, 8, 64, 20, 16, a, b, w, None),
       lib.sg_compact_init_bernoulli(8, 64, 1, 1 << 63, a, None),
       lib.sg_ca_step(0, 8, 3, a, b, None)]
print(res, lib.sg_last_hip_error().decode())
""" % ROOT
    env = dict(os.environ, SG_INJECT_HIP_ERROR="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    line = out.stdout.strip().splitlines()[-1]
    res = eval(line.split("]")[0] + "]")
    assert res[:7] == [-3] * 7 and res[7] == -1  # invalid arguments are still SG_EINVAL
    assert line.split("]", 1)[1].strip()  # the HIP error text is kept


def test_ca_steps_autotune_validation(lib):
    from paper_1706_04552_amd import sg
    a, b, w = 0x100000, 0x7000000000, 0x7100000000
    rho, spp, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    out = (ctypes.byref(rho), ctypes.byref(spp), ctypes.byref(ms))
    assert lib.sg_ca_steps_autotune(0, 10, 0, a, b, w, *out, None) == sg.SG_EINVAL   # steps < 1
    assert lib.sg_ca_steps_autotune(0, 4, 8, a, b, w, *out, None) == sg.SG_EINVAL    # n < 32
    assert lib.sg_ca_steps_autotune(2, 10, 8, a, b, w, *out, None) == sg.SG_EINVAL   # map kind
    assert lib.sg_ca_steps_autotune(0, 10, 8, a, b, None, *out, None) == sg.SG_EINVAL  # no work
    assert lib.sg_ca_steps_autotune(0, 10, 8, a, a + 64, w, *out, None) == sg.SG_EALIAS
    assert lib.sg_ca_steps_autotune(0, 10, 8, a, b, w, None, ctypes.byref(spp),
                                    ctypes.byref(ms), None) == sg.SG_EINVAL


def test_diffuse_steps_validation(lib):
    from paper_1706_04552_amd import sg
    a, b, w = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000), ctypes.c_void_p(0x7100000000)
    r = 8
    assert lib.sg_diffuse_steps(0, r, 64, 10, 17, a, b, w, 0.2, None) == sg.SG_EINVAL
    assert lib.sg_diffuse_steps(0, r, 128, 10, 4, a, b, w, 0.2, None) == sg.SG_EINVAL
    assert lib.sg_diffuse_steps(0, r, 8, 10, 4, a, b, w, 0.2, None) == sg.SG_EINVAL
    assert lib.sg_diffuse_steps(0, r, 64, -2, 4, a, b, w, 0.2, None) == sg.SG_EINVAL
    assert lib.sg_diffuse_steps(0, r, 64, 10, 4, a, b, None, 0.2, None) == sg.SG_EINVAL
    assert lib.sg_diffuse_steps(0, r, 64, 10, 4, a, ctypes.c_void_p(0x100000 + 4096), w, 0.2, None) == sg.SG_EALIAS
    assert lib.sg_diffuse_steps(0, r, 64, 10, 4, a, b, ctypes.c_void_p(0x7000000000 + 16), 0.2, None) == sg.SG_EALIAS


def test_write_pass_intra_validation(lib):
    from paper_1706_04552_amd import sg
    a = ctypes.c_void_p(0x100000)
    assert lib.sg_write_pass_intra(0, 3, 8, 16, a, 1, None) == sg.SG_EINVAL
    assert lib.sg_write_pass_intra(0, -1, 8, 16, a, 1, None) == sg.SG_EINVAL
    assert lib.sg_write_pass_intra(0, sg.SG_INTRA_UNROLL, 8, 64, a, 1, None) == sg.SG_EINVAL
    assert lib.sg_write_pass_intra(1, sg.SG_INTRA_LUT, 8, 128, a, 1, None) == sg.SG_EINVAL
    assert lib.sg_write_pass_intra(2, sg.SG_INTRA_LUT, 8, 16, a, 1, None) == sg.SG_EINVAL
    assert lib.sg_write_pass_intra(0, sg.SG_INTRA_LUT, 8, 16, None, 1, None) == sg.SG_EINVAL


def test_compact_storage_validation(lib):
    from paper_1706_04552_amd import sg
    b64 = ctypes.c_uint64()
    assert lib.sg_compact_bytes(10, 64, ctypes.byref(b64)) == sg.SG_OK
    assert b64.value == 3 ** 4 * 64 * 64
    assert lib.sg_compact_bytes(16, 256, ctypes.byref(b64)) == sg.SG_OK
    assert b64.value == 3 ** 8 * 256 * 256
    # only the temporally blocked tile sides, and a gasket at least a tile wide
    for r, rho in ((10, 32), (10, 16), (5, 64), (10, 512), (21, 256)):
        assert lib.sg_compact_bytes(r, rho, ctypes.byref(b64)) == sg.SG_EINVAL
    assert lib.sg_compact_bytes(10, 64, None) == sg.SG_EINVAL
    r, rho = 10, 64  # dense 1 MiB, compact 324 KiB
    dense, comp = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000)
    assert lib.sg_compact_pack(r, 32, dense, comp, None) == sg.SG_EINVAL
    assert lib.sg_compact_pack(r, rho, None, comp, None) == sg.SG_EINVAL
    assert lib.sg_compact_unpack(r, rho, comp, None, None) == sg.SG_EINVAL
    assert lib.sg_compact_pack(r, rho, ctypes.c_void_p(0x100008), comp, None) == sg.SG_EINVAL
    # the dense array reaches 1 MiB past its start, the compact one 324 KiB
    assert lib.sg_compact_pack(r, rho, dense, ctypes.c_void_p(0x100000 + (1 << 20) - 16),
                               None) == sg.SG_EALIAS
    assert lib.sg_compact_unpack(r, rho, ctypes.c_void_p(0x100000 - 81 * 4096 + 16), dense,
                                 None) == sg.SG_EALIAS
    a, b, w = (ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000),
               ctypes.c_void_p(0x7100000000))
    assert lib.sg_ca_steps_compact(r, rho, 10, 33, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps_compact(r, 32, 10, 4, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps_compact(r, rho, -1, 4, a, b, w, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps_compact(r, rho, 17, 16, a, b, None, None) == sg.SG_EINVAL
    assert lib.sg_ca_steps_compact(r, rho, 17, 16, a, ctypes.c_void_p(0x100000 + 81 * 4096 - 16),
                                   w, None) == sg.SG_EALIAS
    assert lib.sg_ca_steps_compact(r, rho, 17, 16, a, b, ctypes.c_void_p(0x7000000000 + 16),
                                   None) == sg.SG_EALIAS
    # the device-written initial state: tile sides and shapes as above, an aligned array
    for rr, rr_rho in ((r, 32), (5, 64), (21, 256), (10, 512)):
        assert lib.sg_compact_init_bernoulli(rr, rr_rho, 1, 1 << 63, comp, None) == sg.SG_EINVAL
    assert lib.sg_compact_init_bernoulli(r, rho, 1, 1 << 63, None, None) == sg.SG_EINVAL
    assert lib.sg_compact_init_bernoulli(r, rho, 1, 1 << 63, ctypes.c_void_p(0x7000000004),
                                         None) == sg.SG_EINVAL
    # the inverse map: omega must fit an int32, the output array 4-byte aligned
    assert lib.sg_map_lambda_inverse(r, rho, None, None) == sg.SG_EINVAL
    assert lib.sg_map_lambda_inverse(r, rho, ctypes.c_void_p(0x100002), None) == sg.SG_EINVAL
    assert lib.sg_map_lambda_inverse(20, 1, ctypes.c_void_p(0x100000), None) == sg.SG_EINVAL


def test_fractal_validation(lib):
    from paper_1706_04552_amd import sg
    carpet = sg.fractal(3, [(x, y) for y in range(3) for x in range(3) if (x, y) != (1, 1)])
    b = ctypes.c_uint64()
    assert lib.sg_frac_block_count(ctypes.byref(carpet), 0, 5, 9, ctypes.byref(b)) == sg.SG_OK
    assert b.value == 8 ** 3
    assert lib.sg_frac_block_count(ctypes.byref(carpet), 1, 5, 9, ctypes.byref(b)) == sg.SG_OK
    assert b.value == 27 ** 2
    assert lib.sg_frac_block_count(ctypes.byref(carpet), 0, 5, 1, ctypes.byref(b)) == sg.SG_OK
    assert b.value == 8 ** 5
    # rho must be a power of m within n; n within the limit; map kind valid
    for r, rho, m in ((5, 4, 0), (5, 2, 0), (2, 27, 0), (12, 3, 0), (5, 9, 2), (6, 729, 0)):
        assert lib.sg_frac_block_count(ctypes.byref(carpet), m, r, rho, ctypes.byref(b)) == sg.SG_EINVAL
    assert lib.sg_frac_block_count(None, 0, 5, 9, ctypes.byref(b)) == sg.SG_EINVAL
    assert lib.sg_frac_block_count(ctypes.byref(carpet), 0, 5, 9, None) == sg.SG_EINVAL
    # bad motifs: offset out of range, repeated offset, too many, m out of range
    for m, offs in ((3, [(3, 0)]), (3, [(0, 0), (0, 0)]), (2, [(0, 0)] * 5), (5, [(0, 0)]),
                    (1, [(0, 0)])):
        f = sg.fractal(max(m, 2), offs[:16]) if m >= 2 else sg.fractal(2, offs)
        f.m = m
        assert lib.sg_frac_block_count(ctypes.byref(f), 0, 2, 1, ctypes.byref(b)) == sg.SG_EINVAL
    empty = sg.fractal(3, [])
    assert lib.sg_frac_block_count(ctypes.byref(empty), 0, 2, 1, ctypes.byref(b)) == sg.SG_EINVAL
    a, c = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x7000000000)
    assert lib.sg_frac_write(ctypes.byref(carpet), 0, 5, 9, None, 1, None) == sg.SG_EINVAL
    assert lib.sg_frac_life_step(ctypes.byref(carpet), 0, 5, 9, a, None, None) == sg.SG_EINVAL
    assert lib.sg_frac_life_step(ctypes.byref(carpet), 0, 5, 9, a,
                                 ctypes.c_void_p(0x100000 + 243 * 243 - 1), None) == sg.SG_EALIAS
    assert lib.sg_frac_map(ctypes.byref(carpet), 5, 9, ctypes.c_void_p(0x100004), None) == sg.SG_EINVAL
    assert lib.sg_frac_map(ctypes.byref(carpet), 5, 9, None, None) == sg.SG_EINVAL


def test_rect_validation(lib):
    from paper_1706_04552_amd import sg
    b = ctypes.c_uint64()
    assert lib.sg_block_count_rect(0, 10, 64, 4, ctypes.byref(b)) == sg.SG_OK
    assert b.value == 3 ** 4 * 16
    assert lib.sg_block_count_rect(1, 10, 64, 4, ctypes.byref(b)) == sg.SG_OK
    assert b.value == 16 * 256
    assert lib.sg_block_count_rect(0, 10, 4, 64, ctypes.byref(b)) == sg.SG_OK
    assert b.value == 3 ** 4 * 16
    for r, rx, ry in ((10, 48, 4), (10, 64, 3), (3, 16, 4), (10, 512, 4), (10, 0, 4), (21, 4, 4)):
        assert lib.sg_block_count_rect(0, r, rx, ry, ctypes.byref(b)) == sg.SG_EINVAL
    assert lib.sg_block_count_rect(2, 10, 4, 4, ctypes.byref(b)) == sg.SG_EINVAL
    assert lib.sg_write_pass_rect(0, 10, 64, 4, ctypes.c_void_p(0x100008), 1, None) == sg.SG_EINVAL
    assert lib.sg_write_pass_rect(0, 10, 64, 4, None, 1, None) == sg.SG_EINVAL
    assert lib.sg_map_lambda_rect(10, 64, 4, ctypes.c_void_p(0x100004), None) == sg.SG_EINVAL


def test_server_validation_on_the_host(lib):
    from paper_1706_04552_amd import sg
    h = ctypes.c_void_p()
    good = sg.sg_tune(64, 8, 2, 256)
    for bad in [sg.sg_tune(32, 8, 0, 256), sg.sg_tune(64, 33, 0, 256), sg.sg_tune(64, 0, 0, 256),
                sg.sg_tune(64, 8, 65, 256), sg.sg_tune(64, 8, 0, 128)]:
        assert lib.sg_server_create(ctypes.byref(bad), 1 << 30, 8, 0, 0, None,
                                    ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_server_create(None, 1 << 30, 8, 0, 0, None, ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_server_create(ctypes.byref(good), 0, 8, 0, 0, None, ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_server_create(ctypes.byref(good), 1 << 30, 0, 0, 0, None, ctypes.byref(h)) == sg.SG_EINVAL
    assert lib.sg_server_create(ctypes.byref(good), 1 << 30, 8, 0, 0, None, None) == sg.SG_EINVAL
    assert not h.value
    assert lib.sg_server_reserve(None, None, 0) == sg.SG_EINVAL
    assert lib.sg_server_submit(None, 8, 1, 0x1000, None, 0) == sg.SG_EINVAL
    n = ctypes.c_int(-1)
    assert lib.sg_server_step(None, None, 0, ctypes.byref(n)) == sg.SG_EINVAL
    assert lib.sg_server_get_stats(None, None) == sg.SG_EINVAL
    assert lib.sg_server_submit_host(None, 8, 1, 0x1000, None, 0) == sg.SG_EINVAL
    assert lib.sg_server_set_max_active(None, 1) == sg.SG_EINVAL
    assert lib.sg_server_set_transfer_window(None, 1) == sg.SG_EINVAL
    fin = (ctypes.c_double * 1)()
    rej = (ctypes.c_int32 * 1)()
    reqs = (sg.sg_server_request * 1)()
    assert lib.sg_server_replay(None, reqs, 1, fin, rej) == sg.SG_EINVAL
    lib.sg_server_destroy(None)


def test_source_digest_does_not_depend_on_the_checkout_path(tmp_path):
    # a stored profile names the digest of the kernel sources it measured; a
    # copy of the tree elsewhere (another machine's checkout) must agree
    import shutil
    from paper_1706_04552_amd import build
    pkg = tmp_path / "paper_1706_04552_amd"
    shutil.copytree(os.path.join(build.ROOT, "paper_1706_04552_amd", "csrc"), pkg / "csrc")
    shutil.copy(os.path.join(build.ROOT, "paper_1706_04552_amd", "build.py"), pkg / "build.py")
    (pkg / "__init__.py").write_text("")
    shutil.copytree(os.path.join(build.ROOT, "include"), tmp_path / "include")
    code = ("from paper_1706_04552_amd import build as b; "
            "print(b.source_digest(b.LIFE_TB_SOURCES), b.source_digest())")
    out = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True,
                         text=True, check=True).stdout.split()
    assert out == [build.source_digest(build.LIFE_TB_SOURCES), build.source_digest()]
