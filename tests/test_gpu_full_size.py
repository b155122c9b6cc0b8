"""GPU parity at the benchmark's own sizes and in the launch configurations it
times.

- Life: every cell of the state after 100 generations at r = 10, 12, 14 and 16
  (n up to 65,536, 4 GiB per state), for every tile side 4..256 and both maps
  with one launch per generation, for the temporally blocked passes at every
  tile side and generations per pass the benchmark times, and for
  block-compacted storage; plus the per-row XOR and popcount checksums of the
  state.  The reference is the oracle's gasket-only life step.
- Diffusion: every gasket cell of the r = 14 FP32 field after 16 and 500 steps
  against the FP64 oracle (the gasket-graph step, equal to the whole-array
  definition term for term), max-abs <= 1e-5 * max|u| and relative L2 <= 1e-5,
  and every cell off the gasket exactly 0.
- Other fractals at r = 10 (n = 59,049, 3.5 GB per state): the write pass on
  sampled row bands, its total, and agreement of every block side and map;
  life steps on windows the oracle evaluates from their dependency cones.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_04552_amd import inputs, sg

pytestmark = pytest.mark.gpu

SEED = 1706
GENS = 100
RHOS = [4, 8, 16, 32, 64, 128, 256]
TB_SHAPES = [(rho, T) for rho in (32, 64, 128, 256) for T in (8, 16, 32)] + [(16, 8), (16, 16)]
COMPACT_SHAPES = [(rho, T) for rho in (64, 128, 256) for T in (8, 16, 32)]
DIFF_RTOL = 1e-5


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sg.load()
    yield
    torch.cuda.synchronize()


# ------------------------------------------------------------------ references

class LifeRef:
    """The benchmark's initial state at level r (Bernoulli(0.5), seed 1706)
    and the oracle's states after the generation counts asked for, on the
    device, with the oracle's row checksums of each; built once per r."""

    SNAPSHOTS = (20, 36, GENS)

    def __init__(self):
        self.cache = {}

    def __call__(self, r):
        if r not in self.cache:
            note(f"oracle: r={r} life, {GENS} generations (gasket-only step)")
            a0 = inputs.bernoulli_state(r, 0.5, SEED)
            shots = O.life_steps_sparse(r, a0, GENS, snapshots=self.SNAPSHOTS)
            refs = {t: torch.from_numpy(s).cuda() for t, s in shots.items()}
            sums = {t: O.row_checksums(r, s) for t, s in shots.items()}
            self.cache[r] = (torch.from_numpy(a0).cuda(), refs, sums)
            del shots
        return self.cache[r]


@pytest.fixture(scope="module")
def life_ref():
    ref = LifeRef()
    yield ref
    ref.cache.clear()
    torch.cuda.empty_cache()


def device_row_checksums(a: torch.Tensor):
    """Row XOR and row popcount of a uint8 n x n device state (n a power of
    two), with plain torch reductions."""
    x = a
    while x.shape[1] > 1:
        h = x.shape[1] // 2
        x = x[:, :h] ^ x[:, h:]
    pop = torch.zeros(a.shape[0], dtype=torch.int64, device=a.device)
    for b in range(8):
        pop += ((a >> b) & 1).sum(dim=1, dtype=torch.int64)
    return x[:, 0].cpu().numpy(), pop.cpu().numpy()


def check_state(got: torch.Tensor, ref: torch.Tensor, sums):
    assert torch.equal(got, ref)
    xr, pop = device_row_checksums(got)
    assert np.array_equal(xr, sums[0])
    assert np.array_equal(pop, sums[1].astype(np.int64))
    assert int(pop.sum()) > 0  # the state has not died out


def one_launch_per_generation(map_kind, r, rho, a0, gens):
    a = a0.clone()
    b = torch.zeros_like(a)
    for _ in range(gens):
        sg.sg_ca_step(map_kind, r, rho, a, b)
        a, b = b, a
    torch.cuda.synchronize()
    del b
    return a


# ------------------------------------------------------------------ life, one launch per generation

@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("rho", RHOS)
@pytest.mark.parametrize("r", [10, 12, 14, 16])
def test_ca_step_every_cell_after_100_generations(life_ref, r, rho, map_kind):
    if rho > (1 << r):
        pytest.skip("tile wider than the gasket")
    note(f"ca_step {map_kind} r={r} rho={rho}, {GENS} launches, every cell")
    a0, refs, sums = life_ref(r)
    got = one_launch_per_generation(map_kind, r, rho, a0, GENS)
    check_state(got, refs[GENS], sums[GENS])
    del got


# ------------------------------------------------------------------ life, several generations per pass

def ca_steps(map_kind, r, rho, a0, gens, T):
    out = torch.zeros_like(a0)
    work = torch.zeros_like(a0)
    sg.sg_ca_steps(map_kind, r, rho, gens, a0, out, work, steps_per_pass=T)
    torch.cuda.synchronize()
    del work
    return out


@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
@pytest.mark.parametrize("rho,T", TB_SHAPES)
@pytest.mark.parametrize("r", [14, 16])
def test_ca_steps_every_cell_after_100_generations(life_ref, r, rho, T, map_kind):
    note(f"ca_steps {map_kind} r={r} rho={rho} {T} per pass, {GENS} generations, every cell")
    a0, refs, sums = life_ref(r)
    keep = a0.clone()
    got = ca_steps(map_kind, r, rho, a0, GENS, T)
    assert torch.equal(a0, keep)  # the input is read only
    del keep
    check_state(got, refs[GENS], sums[GENS])
    del got


@pytest.mark.parametrize("gens,rho,T", [(20, 256, 32), (20, 128, 32), (36, 256, 32),
                                        (36, 32, 32), (36, 16, 16), (20, 64, 8)])
@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
def test_ca_steps_r16_shorter_runs(life_ref, gens, rho, T, map_kind):
    # other splits into passes (20 generations at 32 per pass is one
    # 20-generation launch, the benchmark's shortest run; 36 is 18 + 18)
    note(f"ca_steps {map_kind} r=16 rho={rho} {T} per pass, {gens} generations, every cell")
    a0, refs, sums = life_ref(16)
    got = ca_steps(map_kind, 16, rho, a0, gens, T)
    check_state(got, refs[gens], sums[gens])
    del got


@pytest.mark.parametrize("rho,T", COMPACT_SHAPES)
def test_ca_steps_compact_every_cell_after_100_generations(life_ref, rho, T):
    r = 16
    note(f"ca_steps_compact r={r} rho={rho} {T} per pass, {GENS} generations, every cell")
    a0, refs, sums = life_ref(r)
    size = sg.sg_compact_bytes(r, rho)
    cin = torch.empty(size, dtype=torch.uint8, device="cuda")
    sg.sg_compact_pack(r, rho, a0, cin)
    out = torch.full((size,), 0x5A, dtype=torch.uint8, device="cuda")
    work = torch.full((size,), 0xC3, dtype=torch.uint8, device="cuda")
    sg.sg_ca_steps_compact(r, rho, GENS, cin, out, work, steps_per_pass=T)
    dense = torch.zeros_like(a0)
    sg.sg_compact_unpack(r, rho, out, dense)
    torch.cuda.synchronize()
    del cin, out, work
    check_state(dense, refs[GENS], sums[GENS])
    del dense


# ------------------------------------------------------------------ diffusion

@pytest.fixture(scope="module")
def diffusion_ref():
    r = 14
    note(f"oracle: r={r} FP64 diffusion, 500 steps (gasket graph)")
    u0 = inputs.uniform_field(r, SEED)
    pos, shots = O.diffuse_steps_graph(r, u0, 500, 0.2, snapshots=(16, 500))
    n = 1 << r
    dpos = torch.from_numpy(pos).cuda()
    off = torch.ones(n * n, dtype=torch.bool, device="cuda")
    off[dpos] = False
    refs = {t: torch.from_numpy(v).cuda() for t, v in shots.items()}
    yield r, torch.from_numpy(u0).cuda(), dpos, off, refs
    del dpos, off, refs
    torch.cuda.empty_cache()


def check_field(got, dpos, off, ref):
    g = got.reshape(-1)[dpos].double()
    d = g - ref
    max_abs = float(d.abs().max())
    scale = float(ref.abs().max())
    rel_l2 = float(d.norm() / ref.norm())
    note(f"  max_abs={max_abs:.3e} scale={scale:.3e} rel_l2={rel_l2:.3e}")
    assert max_abs <= DIFF_RTOL * scale
    assert rel_l2 <= DIFF_RTOL
    assert not got.reshape(-1)[off].any()  # cells off the gasket stay 0


@pytest.mark.parametrize("steps", [16, 500])
@pytest.mark.parametrize("rho", [16, 64, 128, 256])
@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
def test_diffuse_step_every_cell(diffusion_ref, steps, rho, map_kind):
    r, u0, dpos, off, refs = diffusion_ref
    note(f"diffuse_step {map_kind} r={r} rho={rho}, {steps} launches, every cell")
    a = u0.clone()
    b = torch.zeros_like(a)
    for _ in range(steps):
        sg.sg_diffuse_step(map_kind, r, rho, a, b, 0.2)
        a, b = b, a
    torch.cuda.synchronize()
    del b
    check_field(a, dpos, off, refs[steps])


@pytest.mark.parametrize("steps", [16, 500])
@pytest.mark.parametrize("rho,T", [(rho, T) for rho in (16, 32, 64) for T in (4, 8, 12, 16)])
@pytest.mark.parametrize("map_kind", ["lambda", "bbox"])
def test_diffuse_steps_every_cell(diffusion_ref, steps, rho, T, map_kind):
    r, u0, dpos, off, refs = diffusion_ref
    note(f"diffuse_steps {map_kind} r={r} rho={rho} {T} per pass, {steps} steps, every cell")
    out, work = torch.zeros_like(u0), torch.zeros_like(u0)
    sg.sg_diffuse_steps(map_kind, r, rho, steps, u0, out, work, 0.2, steps_per_pass=T)
    torch.cuda.synchronize()
    del work
    check_field(out, dpos, off, refs[steps])


# ------------------------------------------------------------------ other fractals at r = 10

FRACTALS = {"carpet": O.CARPET, "vicsek": O.VICSEK}
FRAC_R = 10
FRAC_RHOS = [3, 9, 27, 81, 243]


@pytest.fixture(scope="module")
def fractal_r10():
    cache = {}

    def get(name):
        if name not in cache:
            cache.clear()
            torch.cuda.empty_cache()
            of = FRACTALS[name]
            note(f"{name} r={FRAC_R}: device state (torch generator, seed {SEED})")
            a = inputs.fractal_state_device(of.m, of.offsets, FRAC_R, 0.5, SEED)
            cache[name] = (a, a.cpu().numpy())
        return cache[name]
    yield get
    cache.clear()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["carpet", "vicsek"])
def test_frac_write_r10(name):
    of = FRACTALS[name]
    f = sg.fractal(of.m, of.offsets)
    n = of.n(FRAC_R)
    first = None
    bands = [0, n // 3 - 17, n // 2, n - 64]
    refs = {y0: O.frac_write_rows(of, FRAC_R, 1, y0, 64) for y0 in bands}
    for rho in FRAC_RHOS:
        for map_kind in ("lambda", "bbox"):
            note(f"frac_write {name} {map_kind} r={FRAC_R} rho={rho}")
            w = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
            sg.sg_frac_write(f, map_kind, FRAC_R, rho, w, 1)
            torch.cuda.synchronize()
            if first is None:
                first = w
                assert int(w.sum(dtype=torch.int64)) == of.k ** FRAC_R
                for y0, ref in refs.items():
                    assert np.array_equal(w[y0:y0 + 64].cpu().numpy(), ref), y0
            else:
                assert torch.equal(w, first), (rho, map_kind)
                del w
    del first
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["carpet", "vicsek"])
def test_frac_life_r10(fractal_r10, name):
    steps = 3
    of = FRACTALS[name]
    f = sg.fractal(of.m, of.offsets)
    a0, host = fractal_r10(name)
    n = of.n(FRAC_R)
    first = None
    for rho in FRAC_RHOS:
        for map_kind in ("lambda", "bbox"):
            note(f"frac_life {name} {map_kind} r={FRAC_R} rho={rho} {steps} steps")
            a = a0.clone()
            b = torch.zeros_like(a)
            for _ in range(steps):
                sg.sg_frac_life_step(f, map_kind, FRAC_R, rho, a, b)
                a, b = b, a
            torch.cuda.synchronize()
            del b
            if first is None:
                first = a
            else:
                assert torch.equal(a, first), (rho, map_kind)
                del a
    got = first
    # windows at the corners, across tile edges of every side, and random
    wins = [(0, 0), (n - 40, 0), (0, n - 20), (n - 40, n - 20)]
    wins += [(243 * 7 - 20, 243 * 11 - 10), (81 * 5 - 20, 81 * 40 - 10), (27 * 100 - 20, 9 * 3 - 10)]
    rng = np.random.default_rng(10)
    wins += [(int(rng.integers(0, n - 40)), int(rng.integers(0, n - 20))) for _ in range(4)]
    for (x0, y0) in wins:
        ref = O.frac_life_window(of, FRAC_R, host, x0, y0, 40, 20, steps)
        assert np.array_equal(got[y0:y0 + 20, x0:x0 + 40].cpu().numpy(), ref), (x0, y0)
    assert int(got.max()) <= 1
    del got, first
