"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: bit-exact for the block maps, the write pass and the uint8 life; for the
FP32 diffusion, max-abs error <= 1e-5 * max|u_ref| and relative L2 error
<= 1e-5 against the FP64 oracle.  Cases compare every element and span
several tiles with ragged tails, r = 0 and every tile side; the write pass is
compared in full at n = 2^16.  The life and diffusion runs at the benchmark's
full sizes are in test_gpu_full_size.py.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_04552_amd import inputs, sg

pytestmark = pytest.mark.gpu

RHOS = [1, 2, 4, 8, 16, 32, 64, 128, 256]
DIFF_RTOL = 1e-5


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sg.load()
    yield
    torch.cuda.synchronize()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_ca(map_kind, r, rho, a0, steps):
    a = dev(a0)
    b = torch.zeros_like(a)
    for _ in range(steps):
        sg.sg_ca_step(map_kind, r, rho, a, b)
        a, b = b, a
    torch.cuda.synchronize()
    return a


def gpu_diffuse(map_kind, r, rho, u0, steps, alpha=0.2):
    a = dev(u0)
    b = torch.zeros_like(a)
    for _ in range(steps):
        sg.sg_diffuse_step(map_kind, r, rho, a, b, alpha)
        a, b = b, a
    torch.cuda.synchronize()
    return a


def diff_errors(got: np.ndarray, ref: np.ndarray):
    d = got.astype(np.float64) - ref
    max_abs = float(np.abs(d).max()) if d.size else 0.0
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    rel_l2 = float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))
    return max_abs, scale, rel_l2


def cases(rs, rhos=RHOS):
    return [(r, rho) for r in rs for rho in rhos if rho <= (1 << r)]


# ------------------------------------------------------------------ maps

@pytest.mark.parametrize("r,rho", [(0, 1), (1, 1), (1, 2), (3, 2), (5, 4), (6, 1), (8, 16),
                                   (9, 8), (10, 32), (12, 1), (13, 2), (15, 32)])
def test_map_lambda_exact(r, rho):
    rb = r - (rho.bit_length() - 1)
    note(f"map_lambda r={r} rho={rho}")
    d = torch.zeros(2 * 3 ** rb, dtype=torch.int32, device="cuda")
    sg.sg_map_lambda(r, rho, d)
    got = d.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert np.array_equal(got, O.map_lambda(rb))


def test_map_lambda_sampled_r16_rho1():
    r, rho, rb = 16, 1, 16
    note("map_lambda r=16 rho=1 sampled")
    d = torch.zeros(2 * 3 ** rb, dtype=torch.int32, device="cuda")
    sg.sg_map_lambda(r, rho, d)
    got = d.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    W, _ = O.lambda_grid(rb)
    nb = 1 << rb
    rng = np.random.default_rng(7)
    for i in list(rng.integers(0, 3 ** rb, size=3000)) + [0, 3 ** rb - 1]:
        lx, ly = O.lambda_paper(rb, int(i % W), int(i // W))
        assert (got[i, 0], got[i, 1]) == (lx, nb - 1 - ly), i
    assert np.all((got[:, 0] & got[:, 1]) == 0)
    assert len(np.unique(got[:, 1] * nb + got[:, 0])) == 3 ** rb


@pytest.mark.parametrize("r,rho", [(0, 1), (2, 1), (4, 2), (7, 4), (9, 16), (10, 32), (11, 8)])
def test_map_bbox_exact(r, rho):
    note(f"map_bbox r={r} rho={rho}")
    nb = (1 << r) // rho
    d = torch.full((nb * nb,), 9, dtype=torch.uint8, device="cuda")
    sg.sg_map_bbox(r, rho, d)
    assert np.array_equal(d.cpu().numpy().reshape(nb, nb), O.map_bbox(r, rho))


# ------------------------------------------------------------------ write pass

@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("r,rho", cases([0, 1, 3, 6, 9, 11]))
def test_write_pass_exact(map_kind, r, rho):
    note(f"write_pass {map_kind} r={r} rho={rho}")
    n = 1 << r
    for v in (1, 255):
        a = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
        sg.sg_write_pass(map_kind, r, rho, a, v)
        assert np.array_equal(a.cpu().numpy(), O.write_pass(r, v))


@pytest.fixture(scope="module")
def write_pass_r16():
    """The oracle's r = 16 write pass (value 1), on the device: 4 GiB."""
    ref = torch.from_numpy(O.write_pass(16, 1)).cuda()
    yield ref
    del ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("rho", [1, 4, 16, 32, 64, 256])
def test_write_pass_full_size_exact(write_pass_r16, map_kind, rho):
    # the paper's experiment at n = 2^16, every element against the oracle,
    # in the launch configurations the benchmark times
    note(f"write_pass full size {map_kind} r=16 rho={rho}")
    a = torch.zeros((1 << 16, 1 << 16), dtype=torch.uint8, device="cuda")
    sg.sg_write_pass(map_kind, 16, rho, a, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, write_pass_r16)
    del a


@pytest.mark.parametrize("intra", ["unroll", "lut", "subbox"])
@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("r,rho", cases([0, 1, 3, 6, 9, 11], [1, 2, 4, 8, 16, 32]))
def test_write_pass_intra_block_variants(intra, map_kind, r, rho):
    note(f"write_pass_intra {intra} {map_kind} r={r} rho={rho}")
    n = 1 << r
    a = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    sg.sg_write_pass_intra(map_kind, intra, r, rho, a, 9)
    assert np.array_equal(a.cpu().numpy(), O.write_pass(r, 9))


# ------------------------------------------------------------------ life

@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("r,rho", cases([0, 1, 2, 3, 5, 7, 10]))
def test_ca_exact_small(map_kind, r, rho):
    note(f"ca {map_kind} r={r} rho={rho} 10 steps")
    a0 = inputs.bernoulli_state(r, 0.5, 1706 + r)
    got = gpu_ca(map_kind, r, rho, a0, 10).cpu().numpy()
    assert np.array_equal(got, O.life_steps(r, a0, 10))


# ------------------------------------------------------------------ multi-step life

def gpu_ca_steps(map_kind, r, rho, a0, steps, spp):
    a = dev(a0)
    out = torch.zeros_like(a)
    work = torch.zeros_like(a)
    sg.sg_ca_steps(map_kind, r, rho, steps, a, out, work, steps_per_pass=spp)
    torch.cuda.synchronize()
    assert torch.equal(a, dev(a0))  # the input is read only
    return out


@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("r,rho,steps,spp", [
    (6, 64, 1, 16), (6, 64, 16, 16), (7, 64, 23, 8), (7, 128, 5, 5), (8, 256, 40, 16),
    (9, 64, 33, 16), (10, 128, 50, 16), (10, 256, 17, 16), (10, 64, 12, 1), (11, 128, 31, 7),
    (8, 16, 9, 1), (9, 4, 3, 0), (10, 256, 0, 16), (12, 256, 100, 16), (12, 128, 100, 11),
    (7, 64, 17, 17), (8, 64, 40, 32), (9, 128, 70, 24), (10, 256, 33, 32), (12, 256, 100, 32),
    (11, 64, 64, 32),
    # small tiles, up to 16 generations per pass (0: the library's choice, 16)
    (4, 16, 5, 16), (5, 16, 9, 4), (5, 32, 20, 16), (6, 16, 17, 16), (7, 32, 23, 8),
    (8, 32, 40, 16), (9, 16, 33, 16), (10, 32, 50, 16), (10, 16, 7, 3), (11, 32, 31, 7),
    (12, 32, 100, 16), (12, 16, 100, 0), (8, 16, 1, 2), (9, 32, 16, 16),
    (10, 32, 64, 32), (12, 32, 100, 0), (7, 32, 33, 24)])
def test_ca_steps_exact(map_kind, r, rho, steps, spp):
    note(f"ca_steps {map_kind} r={r} rho={rho} steps={steps} per_pass={spp}")
    a0 = inputs.bernoulli_state(r, 0.5, 1706 + 3 * r)
    got = gpu_ca_steps(map_kind, r, rho, a0, steps, spp).cpu().numpy()
    ref = a0 if steps == 0 else O.life_steps(r, a0, steps)
    assert np.array_equal(got, ref)




# ------------------------------------------------------------------ diffusion

@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("r,rho", cases([0, 1, 2, 4, 6, 9]))
def test_diffusion_small(map_kind, r, rho):
    steps = 50
    note(f"diffuse {map_kind} r={r} rho={rho} {steps} steps")
    u0 = inputs.uniform_field(r, 1706 + r)
    got = gpu_diffuse(map_kind, r, rho, u0, steps).cpu().numpy()
    ref = O.diffuse_steps(r, u0, steps)
    max_abs, scale, rel_l2 = diff_errors(got, ref)
    assert max_abs <= DIFF_RTOL * scale
    assert rel_l2 <= DIFF_RTOL
    assert np.all(got[ref == 0.0] == 0.0)


# ------------------------------------------------------------------ multi-step diffusion

@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("rho", [16, 32, 64])
@pytest.mark.parametrize("r,steps,spp", [(6, 1, 8), (6, 8, 8), (7, 13, 8), (8, 30, 5), (9, 17, 3),
                                         (10, 40, 8), (10, 0, 8), (8, 9, 1), (5, 11, 8),
                                         (8, 30, 16), (9, 17, 12), (10, 40, 16), (7, 13, 11),
                                         (6, 16, 16), (10, 33, 9), (9, 20, 0)])
def test_diffuse_steps_equal_one_step_calls_and_oracle(map_kind, rho, r, steps, spp):
    if rho > (1 << r):
        pytest.skip("tile wider than the gasket")
    note(f"diffuse_steps {map_kind} r={r} rho={rho} steps={steps} per_pass={spp}")
    u0 = inputs.uniform_field(r, 1706 + 5 * r)
    a = dev(u0)
    out, work = torch.zeros_like(a), torch.zeros_like(a)
    sg.sg_diffuse_steps(map_kind, r, rho, steps, a, out, work, 0.2, steps_per_pass=spp)
    torch.cuda.synchronize()
    one = gpu_diffuse(map_kind, r, rho, u0, steps)  # one launch per step
    assert torch.equal(out, one)
    ref = O.diffuse_steps(r, u0, steps)
    max_abs, scale, rel_l2 = diff_errors(out.cpu().numpy(), ref)
    assert max_abs <= DIFF_RTOL * scale and rel_l2 <= DIFF_RTOL


# ------------------------------------------------------------------ block-compacted storage

def _compact_reference(r, rho, a0):
    """Tiles of the embedding gathered in omega order (the oracle's lambda table)."""
    tab = O.map_lambda(r - (rho.bit_length() - 1))
    tiles = [a0[by * rho:(by + 1) * rho, bx * rho:(bx + 1) * rho] for bx, by in tab]
    return np.stack(tiles).reshape(-1)


@pytest.mark.parametrize("r,rho", [(1, 1), (4, 2), (6, 1), (8, 16), (10, 64), (12, 4), (16, 256)])
def test_map_lambda_inverse_exact(r, rho):
    note(f"map_lambda_inverse r={r} rho={rho}")
    rb = r - (rho.bit_length() - 1)
    nb = 1 << rb
    tab = O.map_lambda(rb)
    ref = np.full((nb, nb), -1, dtype=np.int32)
    ref[tab[:, 1], tab[:, 0]] = np.arange(len(tab), dtype=np.int32)
    got = torch.full((nb * nb,), -7, dtype=torch.int32, device="cuda")
    sg.sg_map_lambda_inverse(r, rho, got)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().reshape(nb, nb), ref)


@pytest.mark.parametrize("r,rho", [(6, 64), (8, 64), (9, 128), (10, 256), (11, 64)])
def test_compact_round_trip(r, rho):
    note(f"compact pack/unpack r={r} rho={rho}")
    a0 = inputs.bernoulli_state(r, 0.5, 77 + r)
    comp = torch.full((sg.sg_compact_bytes(r, rho),), 0xAB, dtype=torch.uint8, device="cuda")
    sg.sg_compact_pack(r, rho, dev(a0), comp)
    back = torch.zeros((1 << r, 1 << r), dtype=torch.uint8, device="cuda")
    sg.sg_compact_unpack(r, rho, comp, back)
    torch.cuda.synchronize()
    assert np.array_equal(comp.cpu().numpy(), _compact_reference(r, rho, a0))
    assert np.array_equal(back.cpu().numpy(), a0)


def gpu_ca_steps_compact(r, rho, a0, steps, spp):
    size = sg.sg_compact_bytes(r, rho)
    cin = torch.empty(size, dtype=torch.uint8, device="cuda")
    sg.sg_compact_pack(r, rho, dev(a0), cin)
    keep = cin.clone()
    # garbage in the output and work buffers: every pass rewrites whole tiles
    out = torch.full((size,), 0x5A, dtype=torch.uint8, device="cuda")
    work = torch.full((size,), 0xC3, dtype=torch.uint8, device="cuda")
    sg.sg_ca_steps_compact(r, rho, steps, cin, out, work, steps_per_pass=spp)
    dense = torch.zeros((1 << r, 1 << r), dtype=torch.uint8, device="cuda")
    sg.sg_compact_unpack(r, rho, out, dense)
    torch.cuda.synchronize()
    assert torch.equal(cin, keep)  # the input is read only
    return dense


@pytest.mark.parametrize("r,rho,steps,spp", [
    (6, 64, 1, 16), (6, 64, 16, 16), (7, 64, 23, 8), (7, 128, 5, 5), (8, 256, 40, 16),
    (9, 64, 33, 16), (10, 128, 50, 16), (10, 256, 17, 16), (10, 64, 12, 1), (11, 128, 31, 7),
    (10, 256, 0, 16), (12, 256, 100, 16), (12, 64, 100, 16), (10, 256, 64, 32),
    (12, 128, 100, 32), (9, 64, 21, 21)])
def test_ca_steps_compact_exact(r, rho, steps, spp):
    note(f"ca_steps_compact r={r} rho={rho} steps={steps} per_pass={spp}")
    a0 = inputs.bernoulli_state(r, 0.5, 1706 + 3 * r)
    got = gpu_ca_steps_compact(r, rho, a0, steps, spp).cpu().numpy()
    ref = a0 if steps == 0 else O.life_steps(r, a0, steps)
    assert np.array_equal(got, ref)


# ------------------------------------------------------------------ rectangular blocks

RECT = [(6, 8, 2), (6, 2, 8), (7, 32, 4), (7, 4, 32), (5, 32, 1), (5, 1, 32), (8, 16, 16),
        (9, 64, 4), (10, 256, 16), (10, 16, 256), (12, 64, 1), (11, 128, 8), (4, 16, 16)]


@pytest.mark.parametrize("r,rho_x,rho_y", RECT)
def test_map_lambda_rect_exact(r, rho_x, rho_y):
    note(f"map_lambda_rect r={r} {rho_x}x{rho_y}")
    ref = O.map_lambda_rect(r, rho_x, rho_y).astype(np.int64)
    got = torch.zeros(2 * len(ref), dtype=torch.int32, device="cuda")
    sg.sg_map_lambda_rect(r, rho_x, rho_y, got)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().reshape(-1, 2).astype(np.int64), ref)


@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("r,rho_x,rho_y", RECT)
def test_write_pass_rect_exact(map_kind, r, rho_x, rho_y):
    note(f"write_pass_rect {map_kind} r={r} {rho_x}x{rho_y}")
    n = 1 << r
    a = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    sg.sg_write_pass_rect(map_kind, r, rho_x, rho_y, a, 9)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), O.write_pass(r, 9))


def test_write_pass_rect_full_size():
    r = 16
    note(f"write_pass_rect full size r={r} 256x16, both maps")
    n = 1 << r
    a = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    sg.sg_write_pass_rect("lambda", r, 256, 16, a, 1)
    b = torch.zeros_like(a)
    sg.sg_write_pass("lambda", r, 64, b, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert int(a.sum(dtype=torch.int64)) == 3 ** r
