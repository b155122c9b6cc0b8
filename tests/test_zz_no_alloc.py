"""The allocation-free batched pass (sg_pass_run_static) against the pass with
a context (sg_pass_run), through the C ABI: two calls in a row, the second
over fewer and smaller gaskets, each bit-exact with the context pass and
with the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_04552_amd import batch as B
from paper_1706_04552_amd import inputs, sg

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


def gaskets(count, r_lo, r_hi, max_steps, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        r = int(rng.integers(r_lo, r_hi + 1))
        steps = int(rng.integers(0, max_steps + 1))
        a0 = inputs.bernoulli_state(r, float(rng.uniform(0.2, 0.8)), seed * 100 + i)
        t = torch.from_numpy(a0).cuda()
        out.append((a0, r, steps, t, torch.zeros_like(t), torch.zeros_like(t)))
    return out


@pytest.mark.parametrize("rho,T,gpc,threads", [(128, 12, 2, 256), (256, 16, 0, 512)])
def test_static_pass_equals_context_pass(rho, T, gpc, threads):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sg.load()
    tune = B.make_tune(rho, T, gpc, threads)
    ctx = B.PassContext(200)
    # the second call is smaller: fewer gaskets, lower levels, and its table
    # overwrites only the start of the first call's
    for call, (count, r_lo, r_hi, seed) in enumerate([(150, 6, 11, 61), (9, 6, 8, 62)]):
        note(f"static pass call {call}: {count} gaskets r={r_lo}..{r_hi}, rho={rho} T={T}")
        gs = gaskets(count, r_lo, r_hi, T, seed)
        ctx.run([(t, ref, r, k) for _, r, k, t, ref, _ in gs], tune)
        B.run_static([(t, got, r, k) for _, r, k, t, _, got in gs], tune)
        torch.cuda.synchronize()
        for a0, r, k, t, ref, got in gs:
            assert torch.equal(got, ref), (call, r, k)
            if k > 0 and r <= 9:
                assert np.array_equal(got.cpu().numpy(), O.life_steps_sparse(r, a0, k))
    ctx.close()


def test_static_pass_rejects_more_items_than_its_table():
    sg.load()
    tune = B.make_tune(64, 8, 0, 256)
    arr = (sg.sg_pass_item * (sg.SG_PASS_STATIC_MAX + 1))()
    rc = sg.load().sg_pass_run_static(arr, sg.SG_PASS_STATIC_MAX + 1, tune, None)
    assert rc == sg.SG_EINVAL
