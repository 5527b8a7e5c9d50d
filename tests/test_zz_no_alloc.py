"""The allocation-free training step (scratch in the library's static device array)
against the training step on a caller-provided work buffer: two calls in a row, the
second with a smaller batch, through the C ABI.  Both run the same kernels in the same
order, so parameters, Adam moments and loss agree bit for bit."""
import sys

import numpy as np
import pytest

from paper_1912_10192_amd import grmhd, learned

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_noalloc_train_step_matches_workspace_step():
    import torch
    dev = torch.device("cuda:0")
    gen = torch.Generator(device="cpu").manual_seed(11)
    n = 20000
    X = torch.randn(n, 8, generator=gen).to(dev)
    Y = torch.randn(n, 2, generator=gen).to(dev)
    p0 = learned.init_params(7, dev)
    ref = grmhd.MLPTrainer(p0, batch=grmhd.NOALLOC_MAX_BATCH)
    params, m, v = p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    for step, batch in ((1, grmhd.NOALLOC_MAX_BATCH), (2, 1000)):
        idx = torch.randint(0, n, (batch,), generator=gen, dtype=torch.int32).to(dev)
        say(f"[noalloc] step {step} batch {batch}")
        ref.step(X, Y, idx, 1e-3)
        grmhd.mlp_train_step_noalloc(params, m, v, step, X, Y, idx, 1e-3, loss)
        torch.cuda.synchronize()
        for a, b, name in ((params, ref.params, "params"), (m, ref.m, "m"), (v, ref.v, "v"),
                           (loss, ref.loss, "loss")):
            assert torch.equal(a, b), name
        say(f"  loss {float(loss[0]):.6f}, parameters equal")
    assert not torch.equal(params, p0)


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    import torch
    dev = torch.device("cuda:0")
    p = learned.init_params(7, dev)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    X = torch.zeros(10, 8, device=dev)
    Y = torch.zeros(10, 2, device=dev)
    idx = torch.zeros(grmhd.NOALLOC_MAX_BATCH + 1, dtype=torch.int32, device=dev)
    loss = torch.zeros(1, device=dev)
    with pytest.raises(grmhd.GrmhdError, match="NOALLOC_MAX_BATCH"):
        grmhd.mlp_train_step_noalloc(p, m, v, 1, X, Y, idx, 1e-3, loss)
