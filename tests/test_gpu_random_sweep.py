"""Seeded random sweeps of the multi-step passes against the oracle.

Life (sg_ca_steps) and FP32 diffusion (sg_diffuse_steps) over cases drawn
from a fixed seed: level, tile side, generations per pass (every supported
value, and 0 for the library's choice), step count, map and initial density.
Every case is compared cell by cell: life bit-exact against the oracle;
diffusion bit-exact against one launch per step (the same FP32 arithmetic)
and within 1e-5 (max-abs relative to the field's scale, and relative L2) of
the FP64 oracle, with every cell off the gasket exactly 0.

Batches of gaskets (sg_batch_*) with random launch shapes (tile side,
generations per pass, workgroups per compute unit, threads), item counts,
levels and step counts (0 included), run with and without the hipGraph:
every gasket bit-exact against the oracle.

Embedded fractals with random motifs (m in {2, 3, 4}, a random set of kept
sub-squares listed in a random order): the generalised block map, the write
pass and life steps, bit-exact against the oracle, at random levels and
block sides, both maps.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_04552_amd import batch as B
from paper_1706_04552_amd import inputs, sg

pytestmark = pytest.mark.gpu

DIFF_RTOL = 1e-5


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sg.load()
    yield
    torch.cuda.synchronize()


def _life_cases(count=120, seed=17):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        rho = int(rng.choice([4, 8, 16, 32, 64, 128, 256]))
        r = int(rng.integers(max(rho.bit_length() - 1, 2), 12))  # 2 .. 11, rho <= 2^r
        if rho > (1 << r):
            continue
        if rho >= 32:
            spp = int(rng.integers(0, 33))  # 0 (library's choice) .. 32
        elif rho == 16:
            spp = int(rng.integers(0, 17))
        else:
            spp = int(rng.choice([0, 1]))
        steps = int(rng.integers(0, 70))
        p = round(float(rng.uniform(0.1, 0.9)), 3)
        map_kind = "lambda" if rng.random() < 0.5 else "bbox"
        out.append((map_kind, r, rho, steps, spp, p, int(rng.integers(1 << 30))))
    return out


def _diffusion_cases(count=80, seed=23):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        # mostly the tile sides with several steps per pass
        rho = int(rng.choice([4, 8, 16, 32, 64, 128], p=[0.1, 0.1, 0.25, 0.25, 0.2, 0.1]))
        r = int(rng.integers(max(rho.bit_length() - 1, 2), 12))
        if rho > (1 << r):
            continue
        spp = int(rng.integers(0, 17)) if rho in (16, 32, 64) else int(rng.choice([0, 1]))
        steps = int(rng.integers(0, 60))
        map_kind = "lambda" if rng.random() < 0.5 else "bbox"
        out.append((map_kind, r, rho, steps, spp, int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("case", _life_cases(), ids=lambda c: "-".join(map(str, c[:5])))
def test_ca_steps_random_sweep(case):
    map_kind, r, rho, steps, spp, p, seed = case
    note(f"ca_steps {map_kind} r={r} rho={rho} steps={steps} per_pass={spp} p={p} seed={seed}")
    a0 = inputs.bernoulli_state(r, p, seed)
    a = torch.from_numpy(a0).cuda()
    out, work = torch.zeros_like(a), torch.zeros_like(a)
    sg.sg_ca_steps(map_kind, r, rho, steps, a, out, work, steps_per_pass=spp)
    torch.cuda.synchronize()
    ref = a0 if steps == 0 else O.life_steps(r, a0, steps)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("case", _diffusion_cases(), ids=lambda c: "-".join(map(str, c[:5])))
def test_diffuse_steps_random_sweep(case):
    map_kind, r, rho, steps, spp, seed = case
    note(f"diffuse_steps {map_kind} r={r} rho={rho} steps={steps} per_pass={spp} seed={seed}")
    u0 = inputs.uniform_field(r, seed)
    a = torch.from_numpy(u0).cuda()
    out, work = torch.zeros_like(a), torch.zeros_like(a)
    sg.sg_diffuse_steps(map_kind, r, rho, steps, a, out, work, 0.2, steps_per_pass=spp)
    # one launch per step: the same arithmetic, so the same bits
    x, y = a.clone(), torch.zeros_like(a)
    for _ in range(steps):
        sg.sg_diffuse_step(map_kind, r, rho, x, y, 0.2)
        x, y = y, x
    torch.cuda.synchronize()
    assert torch.equal(out, x)
    got = out.cpu().numpy()
    ref = O.diffuse_steps(r, u0, steps)
    scale = max(float(np.abs(ref).max()), 1e-30)
    assert float(np.abs(got - ref).max()) <= DIFF_RTOL * scale
    assert float(np.linalg.norm(got - ref)) <= DIFF_RTOL * max(float(np.linalg.norm(ref)), 1e-30)
    assert np.all(got[ref == 0.0] == 0.0)


def _fractal_cases(count=60, seed=29):
    rng = np.random.default_rng(seed)
    out = []
    max_r = {2: 11, 3: 7, 4: 5}  # n up to 2048, 2187, 1024
    while len(out) < count:
        m = int(rng.choice([2, 3, 4]))
        k = int(rng.integers(1, min(m * m, 16) + 1))
        cells = rng.permutation(m * m)[:k]
        offsets = [(int(c % m), int(c // m)) for c in cells]
        r = int(rng.integers(0, max_r[m] + 1))
        qs = [q for q in range(r + 1) if m ** q <= 243]
        q = int(rng.choice(qs))
        map_kind = "lambda" if rng.random() < 0.5 else "bbox"
        steps = int(rng.integers(1, 7))
        out.append((m, tuple(offsets), r, m ** q, map_kind, steps, int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("case", _fractal_cases(),
                         ids=lambda c: f"m{c[0]}-k{len(c[1])}-r{c[2]}-rho{c[3]}-{c[4]}")
def test_fractal_random_motifs(case):
    m, offsets, r, rho, map_kind, steps, seed = case
    note(f"fractal m={m} offsets={offsets} r={r} rho={rho} {map_kind} {steps} steps seed={seed}")
    of = O.Fractal(m, offsets)
    f = sg.fractal(m, offsets)
    n = m ** r
    q = round(np.log(rho) / np.log(m))
    # the generalised map (lambda's canonical table)
    ref_map = O.frac_map(of, r - q).astype(np.int64)
    got_map = torch.zeros(2 * len(ref_map), dtype=torch.int32, device="cuda")
    sg.sg_frac_map(f, r, rho, got_map)
    # the write pass
    a = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    sg.sg_frac_write(f, map_kind, r, rho, a, 5)
    # life steps
    s0 = inputs.fractal_state(m, offsets, r, 0.5, seed)
    x = torch.from_numpy(s0).cuda()
    y = torch.zeros_like(x)
    for _ in range(steps):
        sg.sg_frac_life_step(f, map_kind, r, rho, x, y)
        x, y = y, x
    torch.cuda.synchronize()
    assert np.array_equal(got_map.cpu().numpy().reshape(-1, 2).astype(np.int64), ref_map)
    assert np.array_equal(a.cpu().numpy(), O.frac_write(of, r, 5))
    assert np.array_equal(x.cpu().numpy(), O.frac_life_steps(of, r, s0, steps))


def _batch_cases(count=16, seed=31):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        tune = (int(rng.choice([64, 128, 256])), int(rng.integers(1, 33)),
                int(rng.choice([0, 1, 2, 4, 8])), int(rng.choice([256, 512])))
        out.append((tune, int(rng.integers(1, 25)), bool(rng.random() < 0.5),
                    int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("case", _batch_cases(),
                         ids=lambda c: f"rho{c[0][0]}-T{c[0][1]}-g{c[0][2]}-t{c[0][3]}-n{c[1]}")
def test_batch_random_shapes(case):
    tune, count, graph, seed = case
    note(f"batch tune={tune} count={count} graph={graph} seed={seed}")
    rng = np.random.default_rng(seed)
    hosts, gs = [], []
    for i in range(count):
        r = int(rng.integers(6, 12))
        steps = int(rng.integers(0, 41))
        a0 = inputs.bernoulli_state(r, float(rng.uniform(0.1, 0.9)), seed + i)
        inp = torch.from_numpy(a0).cuda()
        gs.append(B.Gasket(r, steps, inp, torch.zeros_like(inp), torch.zeros_like(inp)))
        hosts.append(a0)
    with B.Batch(gs, B.make_tune(*tune)) as bt:
        bt.run(graph=graph)
        torch.cuda.synchronize()
    for g, a0 in zip(gs, hosts):
        ref = a0 if g.steps == 0 else O.life_steps_sparse(g.r, a0, g.steps)
        assert np.array_equal(g.out.cpu().numpy(), ref), (g.r, g.steps)
