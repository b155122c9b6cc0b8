"""GPU parity of the batched paths: many gaskets of uneven levels in one
persistent launch per pass (graph-captured or eager), the per-iteration pass
of continuous batching, the autotuner's choice, and the serving loop.  Each
gasket's result must be bit-exact with the oracle and identical to the same
gasket run alone through sg_ca_steps."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_04552_amd import batch as B
from paper_1706_04552_amd import inputs, sg
from paper_1706_04552_amd.serving import (ContinuousBatcher, GpuExecutor, NativeServer, Request,
                                          footprint, serve_native)

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sg.load()
    yield
    torch.cuda.synchronize()


def make_gaskets(count, r_lo, r_hi, steps_lo, steps_hi, seed):
    rng = np.random.default_rng(seed)
    hosts, gs = [], []
    for i in range(count):
        r = int(rng.integers(r_lo, r_hi + 1))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        p = float(rng.uniform(0.2, 0.8))
        a0 = inputs.bernoulli_state(r, p, seed * 1000 + i)
        inp = torch.from_numpy(a0).cuda()
        gs.append(B.Gasket(r, steps, inp, torch.zeros_like(inp), torch.zeros_like(inp)))
        hosts.append(a0)
    return hosts, gs


def oracle_check(r, a0, steps, got):
    if r <= 11:
        assert np.array_equal(got, O.life_steps_sparse(r, a0, steps) if steps else a0)
    else:
        n = 1 << r
        for (x0, y0) in [(0, 0), (n - 48, 0), (0, n - 8), (n // 3, n // 5)]:
            ref = O.life_window(r, a0, x0, y0, 48, 8, steps)
            assert np.array_equal(got[y0:y0 + 8, x0:x0 + 48], ref), (r, x0, y0)


def solo(g, T=16):
    out = torch.zeros_like(g.inp)
    work = torch.zeros_like(g.inp)
    sg.sg_ca_steps("lambda", g.r, 64, g.steps, g.inp, out, work, steps_per_pass=T)
    return out


def test_batch_graph_replays_equal_eager_solo_and_oracle():
    note("batch of 48 gaskets r=6..11, steps 0..40, graph and eager")
    hosts, gs = make_gaskets(48, 6, 11, 0, 40, 3)
    tune = B.make_tune(rho=64, steps_per_pass=16, groups_per_cu=2, threads=256)
    with B.Batch(gs, tune) as bt:
        st = bt.stats()
        assert st["passes"] == max(-(-g.steps // 16) for g in gs)
        assert st["cell_steps"] == sum(3 ** g.r * g.steps for g in gs)
        bt.run(graph=False)
        torch.cuda.synchronize()
        eager = [g.out.clone() for g in gs]
        for rep in range(3):
            for g in gs:
                g.out.zero_()
                g.work.zero_()
            torch.cuda.synchronize()
            bt.run(graph=True)
            torch.cuda.synchronize()
            for g, e in zip(gs, eager):
                assert torch.equal(g.out, e), rep
    for g, e, a0 in zip(gs, eager, hosts):
        assert torch.equal(e, solo(g))
        oracle_check(g.r, a0, g.steps, e.cpu().numpy())


@pytest.mark.parametrize("rho,spp,gpc,threads", [(64, 8, 0, 512), (128, 16, 4, 256),
                                                 (128, 5, 1, 512), (256, 16, 8, 256),
                                                 (256, 16, 0, 512), (256, 32, 2, 512),
                                                 (64, 32, 0, 256)])
def test_batch_launch_shapes_agree(rho, spp, gpc, threads):
    # levels 6..11: gaskets smaller than rho use tiles of their own side
    note(f"batch shapes rho={rho} per_pass={spp} groups_per_cu={gpc} threads={threads}")
    hosts, gs = make_gaskets(24, 6, 11, 1, 35, 11)
    ref = [solo(g) for g in gs]
    with B.Batch(gs, B.make_tune(rho, spp, gpc, threads)) as bt:
        bt.run(graph=True)
        torch.cuda.synchronize()
    for g, e in zip(gs, ref):
        assert torch.equal(g.out, e)
    oracle_check(gs[0].r, hosts[0], gs[0].steps, gs[0].out.cpu().numpy())


def test_autotune_returns_a_valid_shape():
    note("autotune on 16 gaskets r=7..10")
    hosts, gs = make_gaskets(16, 7, 10, 5, 30, 5)
    tune, ms = B.autotune(gs)
    assert ms > 0 and tune.rho in (64, 128, 256) and tune.threads in (256, 512)
    assert 1 <= tune.steps_per_pass <= 32 and tune.groups_per_cu in (0, 2, 4, 8)
    for g in gs:
        g.out.zero_()
        g.work.zero_()
    with B.Batch(gs, tune) as bt:
        bt.run()
        torch.cuda.synchronize()
    for g, a0 in zip(gs, hosts):
        oracle_check(g.r, a0, g.steps, g.out.cpu().numpy())


def test_pass_context_mixed_steps():
    note("pass context: one pass over gaskets with different generation counts")
    hosts, gs = make_gaskets(20, 6, 10, 0, 12, 9)
    ctx = B.PassContext(64)
    tune = B.make_tune(64, 12, 2, 256)
    items = [(g.inp, g.out, g.r, g.steps) for g in gs]
    ctx.run(items, tune)
    torch.cuda.synchronize()
    for g, a0 in zip(gs, hosts):
        if g.steps:
            oracle_check(g.r, a0, g.steps, g.out.cpu().numpy())
    # a second pass on the same context (staging reuse) continues from out
    ctx.run([(g.out, g.work, g.r, 3) for g in gs], tune)
    torch.cuda.synchronize()
    for g, a0 in zip(gs[:6], hosts[:6]):
        if g.steps:
            oracle_check(g.r, a0, g.steps + 3, g.work.cpu().numpy())
    ctx.close()


@pytest.mark.parametrize("horizon,budget", [(None, None), (3 ** 10 * 64, None),
                                            (10 ** 12, 3 ** 9 * 8)])
def test_serving_results_equal_alone_and_respect_the_cap(horizon, budget):
    note(f"continuous batching: 40 requests r=6..10, horizon {horizon}, budget {budget}")
    rng = np.random.default_rng(21)
    reqs = []
    for i in range(40):
        r = int(rng.integers(6, 11))
        steps = int(rng.integers(0, 60))
        reqs.append(Request(i, float(rng.uniform(0, 0.02)), r, steps,
                            inputs.bernoulli_state(r, 0.5, 500 + i)))
    cap = 6 * footprint(10)
    ex = GpuExecutor(B.make_tune(64, 8, 2, 256), capacity=64)
    st = ContinuousBatcher(ex, cap_bytes=cap, steps_per_pass=8, keep_outputs=True,
                           max_cells_per_pass=budget, horizon_cells=horizon).serve(reqs)
    ex.close()
    assert st.max_resident_bytes <= cap and st.max_active >= 2
    assert len(st.results) == 40 and not any(x.rejected for x in st.results)
    for res in st.results:
        q = reqs[res.rid]
        inp = torch.from_numpy(q.state).cuda()
        g = B.Gasket(q.r, q.steps, inp, torch.zeros_like(inp), torch.zeros_like(inp))
        alone = solo(g, T=8).cpu().numpy()
        assert np.array_equal(res.output, alone), res.rid
        oracle_check(q.r, q.state, q.steps, res.output)


def test_batch_benchmark_configuration_every_instance():
    """The benchmark's batch: 512 gaskets (r ~ U{6..13}, p ~ U[0.2, 0.8]),
    50 generations, the autotuner's launch shape, one hipGraph; every
    instance against the oracle (whole state for r <= 11, sampled windows
    from the dependency cone above)."""
    steps = 50
    specs = inputs.batch_specs(512)
    note(f"benchmark batch: {len(specs)} gaskets, {steps} generations, autotuned")
    hosts, gs = [], []
    for spec in specs:
        a0 = spec.state()
        inp = torch.from_numpy(a0).cuda()
        gs.append(B.Gasket(spec.r, steps, inp, torch.zeros_like(inp), torch.zeros_like(inp)))
        hosts.append(a0)
    tune, _ = B.autotune(gs)
    with B.Batch(gs, tune) as bt:
        bt.run(graph=True)
        torch.cuda.synchronize()
    for spec, g, a0 in zip(specs, gs, hosts):
        got = g.out.cpu().numpy()
        if spec.r <= 11:
            assert np.array_equal(got, O.life_steps_sparse(spec.r, a0, steps)), spec
        else:
            n = 1 << spec.r
            for (x0, y0) in [(0, 0), (n - 40, n // 2), (n // 3, n - 6)]:
                ref = O.life_window(spec.r, a0, x0, y0, 40, 6, steps)
                assert np.array_equal(got[y0:y0 + 6, x0:x0 + 40], ref), (spec, x0, y0)


@pytest.mark.parametrize("horizon,budget", [(0, 0), (3 ** 10 * 64, 0), (10 ** 12, 3 ** 9 * 8)])
def test_native_server_results_equal_alone_and_respect_the_cap(horizon, budget):
    note(f"native server: 41 requests r=6..10 (+1 too large), horizon {horizon}, budget {budget}")
    rng = np.random.default_rng(23)
    reqs = []
    for i in range(40):
        r = int(rng.integers(6, 11))
        steps = int(rng.integers(0, 60))
        # half arrive together, so the first round admits several at once
        arrival = 0.0 if i < 20 else float(rng.uniform(0, 0.02))
        reqs.append(Request(i, arrival, r, steps, inputs.bernoulli_state(r, 0.5, 700 + i)))
    reqs.append(Request(40, 0.005, 12, 3, inputs.bernoulli_state(12, 0.5, 740)))  # never fits
    cap = 6 * footprint(10)
    server = NativeServer(B.make_tune(64, 8, 2, 256), cap, 64, horizon, budget)
    server.reserve([10, 10, 9, 9, 8, 8])
    inits = {q.rid: torch.from_numpy(q.state).cuda() for q in reqs}
    outs = {q.rid: torch.zeros_like(inits[q.rid]) for q in reqs}
    st = serve_native(server, reqs, inits, outs)
    stats = server.stats()
    server.close()
    assert st.max_resident_bytes <= cap and st.max_active >= 2
    assert len(st.results) == 41 and stats["completed"] == 40 and stats["rejected"] == 1
    assert stats["cell_steps"] == sum(3 ** q.r * q.steps for q in reqs[:40])
    assert stats["queued"] == stats["active"] == stats["resident_bytes"] == 0
    for res in st.results:
        q = reqs[res.rid]
        assert res.rejected == (q.rid == 40)
        if res.rejected:
            continue
        g = B.Gasket(q.r, q.steps, inits[q.rid], torch.zeros_like(inits[q.rid]),
                     torch.zeros_like(inits[q.rid]))
        alone = solo(g, T=8)
        assert torch.equal(outs[q.rid], alone), res.rid
        oracle_check(q.r, q.state, q.steps, outs[q.rid].cpu().numpy())


def test_native_server_reuses_its_pool_across_waves():
    """Two waves through one server: the second reuses the buffers the first
    released, which must again hold 0 off the gasket."""
    note("native server: two waves of 12 requests r=7..9")
    server = NativeServer(B.make_tune(64, 16, 0, 256), 8 * footprint(9), 16)
    for wave in range(2):
        reqs = [Request(i, 0.0, 7 + i % 3, 5 + 7 * i, inputs.bernoulli_state(7 + i % 3, 0.6, 800 + 50 * wave + i))
                for i in range(12)]
        inits = {q.rid: torch.from_numpy(q.state).cuda() for q in reqs}
        outs = {q.rid: torch.zeros_like(inits[q.rid]) for q in reqs}
        st = serve_native(server, reqs, inits, outs)
        assert len(st.results) == 12 and not any(x.rejected for x in st.results)
        for q in reqs:
            oracle_check(q.r, q.state, q.steps, outs[q.rid].cpu().numpy())
    server.close()


def test_native_server_device_memory_stays_under_the_cap():
    """Requests of levels outside the reserved pool, in waves of shifting
    levels: buffers the pool holds for one level must be freed before new
    ones of another level would take the device bytes held past the cap."""
    cap = 6 * footprint(10)
    server = NativeServer(B.make_tune(64, 8, 0, 256), cap, 64)
    server.reserve([10, 10, 10])  # pool of level 10 only
    rng = np.random.default_rng(31)
    waves = [[6, 7, 8, 9] * 3, [11], [9, 9, 10, 10, 8, 8], [11, 6, 7], [10] * 6]
    rid = 0
    for levels in waves:
        reqs = []
        for r in levels:
            reqs.append(Request(rid, 0.0, r, int(rng.integers(1, 20)),
                                inputs.bernoulli_state(r, 0.5, 900 + rid)))
            rid += 1
        note(f"native server cap: wave of levels {levels}")
        inits = {q.rid: torch.from_numpy(q.state).cuda() for q in reqs}
        outs = {q.rid: torch.zeros_like(inits[q.rid]) for q in reqs}
        st = serve_native(server, reqs, inits, outs)
        assert len(st.results) == len(reqs) and not any(x.rejected for x in st.results)
        stats = server.stats()
        assert stats["max_allocated_bytes"] <= cap, stats
        assert stats["allocated_bytes"] <= cap
        for q in reqs:
            oracle_check(q.r, q.state, q.steps, outs[q.rid].cpu().numpy())
    server.close()


def test_python_executor_device_memory_stays_under_the_cap():
    cap = 6 * footprint(10)
    ex = GpuExecutor(B.make_tune(64, 8, 0, 256), capacity=32, cap_bytes=cap)
    ex.reserve([10, 10, 10], cap)
    rng = np.random.default_rng(37)
    rid = 0
    for levels in ([6, 7, 8, 9] * 3, [11], [9, 9, 10, 10, 8, 8], [11, 6, 7]):
        reqs = []
        for r in levels:
            reqs.append(Request(rid, 0.0, r, int(rng.integers(1, 20)),
                                inputs.bernoulli_state(r, 0.5, 950 + rid)))
            rid += 1
        note(f"python executor cap: wave of levels {levels}")
        st = ContinuousBatcher(ex, cap_bytes=cap, steps_per_pass=8, keep_outputs=True).serve(reqs)
        assert ex.max_allocated <= cap and ex.allocated <= cap
        for res in st.results:
            q = reqs[res.rid - reqs[0].rid]
            oracle_check(q.r, q.state, q.steps, res.output)
    ex.close()


def _pinned(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


@pytest.mark.parametrize("max_active,window", [(0, 1), (1, 1), (3, 1), (0, 0), (0, 2)])
def test_native_server_replay_host_and_device_requests(max_active, window):
    """Requests arriving in real time through the native replay loop, half
    with pinned host states (uploaded at admission, read back when done) and
    half with device states; every result equals the gasket run alone and
    the oracle, and max_active bounds the requests in flight."""
    rng = np.random.default_rng(41 + max_active)
    reqs, inits, outs = [], {}, {}
    for i in range(24):
        r = int(rng.integers(6, 11))
        steps = int(rng.integers(0, 50))
        a0 = inputs.bernoulli_state(r, 0.5, 1200 + i)
        q = Request(i, float(rng.uniform(0, 0.01)), r, steps, a0)
        reqs.append(q)
        if i % 2:
            inits[i], outs[i] = _pinned(a0), torch.zeros(a0.shape, dtype=torch.uint8).pin_memory()
        else:
            inits[i] = torch.from_numpy(a0).cuda()
            outs[i] = torch.zeros_like(inits[i])
    note(f"native server replay: 24 requests (12 host, 12 device), max_active={max_active}")
    server = NativeServer(B.make_tune(64, 8, 2, 256), 8 * footprint(10), 64)
    server.set_max_active(max_active)
    server.set_transfer_window(window)
    st = server.replay(reqs, inits, outs)
    stats = server.stats()
    server.close()
    assert len(st.results) == 24 and not any(x.rejected for x in st.results)
    assert all(x.finished >= x.arrival for x in st.results)
    if max_active:
        assert stats["max_active"] <= max_active
    assert stats["completed"] == 24 and stats["transferring"] == 0
    for q in reqs:
        got = outs[q.rid].cpu().numpy() if not outs[q.rid].is_cuda else outs[q.rid].cpu().numpy()
        g = B.Gasket(q.r, q.steps, torch.from_numpy(q.state).cuda(),
                     torch.zeros(q.state.shape, dtype=torch.uint8, device="cuda"),
                     torch.zeros(q.state.shape, dtype=torch.uint8, device="cuda"))
        assert np.array_equal(got, solo(g, T=8).cpu().numpy()), q.rid
        oracle_check(q.r, q.state, q.steps, got)


def test_ca_steps_autotune_single_gasket():
    r, steps = 12, 40
    note(f"sg_ca_steps_autotune r={r} {steps} generations")
    a0 = inputs.bernoulli_state(r, 0.5, 1300)
    inp = torch.from_numpy(a0).cuda()
    out, work = torch.zeros_like(inp), torch.zeros_like(inp)
    rho, spp, ms = sg.sg_ca_steps_autotune("lambda", r, steps, inp, out, work)
    assert rho in (32, 64, 128, 256) and spp in (8, 16, 32) and ms > 0
    assert torch.equal(inp, torch.from_numpy(a0).cuda())  # the input is read only
    out.zero_()
    sg.sg_ca_steps("lambda", r, rho, steps, inp, out, work, steps_per_pass=spp)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), O.life_steps_sparse(r, a0, steps))
