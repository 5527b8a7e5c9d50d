"""GPU checks of the learned inversion guess: the BF16-MFMA kernels against the
BF16-emulating oracle, the device dataset against the oracle's features and targets,
training progress, and that the learned guess leaves the evolution unchanged."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_1912_10192_amd import configs, grmhd, initdata, learned

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _torch():
    import torch
    return torch


def _params_list(flat):
    out, o = [], 0
    for a, b in zip(omlp.SIZES[:-1], omlp.SIZES[1:]):
        out.append(flat[o:o + a * b].reshape(a, b).astype(np.float64))
        o += a * b
        out.append(flat[o:o + b].astype(np.float64))
        o += b
    return out


def test_forward_and_gradients_match_bf16_oracle():
    torch = _torch()
    dev = torch.device("cuda")
    rng = np.random.default_rng(0)
    n, batch = 1000, 256
    X = rng.normal(size=(n, 8)).astype(np.float32)
    Y = rng.normal(size=(n, 2)).astype(np.float32)
    idx = rng.integers(0, n, batch).astype(np.int32)
    flat = learned.init_params(3, "cpu").numpy()
    params = _params_list(flat)
    say("[mlp] gradients and forward vs oracle (bf16 emulation)")
    tp = torch.from_numpy(flat).to(dev)
    tX, tY, ti = (torch.from_numpy(a).to(dev) for a in (X, Y, idx))
    grad, loss = grmhd.mlp_gradients(tp, tX, tY, ti)
    grad = grad.cpu().numpy()
    l_ref, g_ref = omlp.loss_and_grads(params, X[idx].astype(np.float64), Y[idx].astype(np.float64), "bf16")
    assert float(loss.item()) == pytest.approx(l_ref, rel=1e-3)
    o = 0
    for g in g_ref:
        seg = grad[o:o + g.size].reshape(g.shape)
        o += g.size
        err = np.abs(seg - g).max() / max(np.abs(g).max(), 1e-30)
        say(f"  gradient block {g.shape}: max error / max |grad| = {err:.2e}")
        assert err < 1e-2, err
    norm = torch.tensor([0.0] * 8 + [1.0] * 8 + [0.0, 0.0, 1.0, 1.0], dtype=torch.float32, device=dev)
    blob = grmhd.mlp_pack(tp, norm)
    out = grmhd.mlp_forward(blob, tX).cpu().numpy()
    ref, _ = omlp.forward(params, X.astype(np.float64), "bf16")
    assert np.abs(out - ref).max() / np.abs(ref).max() < 2e-2


def test_adam_steps_match_oracle():
    """three training steps on the device (gradients, then the Adam update of the FP32
    masters) against the oracle's Adam applied to the same gradients in FP64: parameters
    and both moment estimates agree to FP32 rounding (beta2 = 0.999 held in FP32 makes
    1 - beta2 larger by 1.3e-5 relative, which the second moment carries)"""
    torch = _torch()
    dev = torch.device("cuda")
    rng = np.random.default_rng(1)
    n, batch, lr = 2000, 512, 3e-3
    X = rng.normal(size=(n, 8)).astype(np.float32)
    Y = rng.normal(size=(n, 2)).astype(np.float32)
    flat = learned.init_params(5, "cpu").numpy()
    tX, tY = (torch.from_numpy(a).to(dev) for a in (X, Y))
    trainer = grmhd.MLPTrainer(torch.from_numpy(flat).to(dev), batch=batch)
    params = _params_list(flat)
    state = (0, [np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params])
    say("[mlp] three Adam steps vs oracle")
    for step in range(3):
        idx = torch.from_numpy(rng.integers(0, n, batch).astype(np.int32)).to(dev)
        grad, _ = grmhd.mlp_gradients(trainer.params, tX, tY, idx)
        trainer.step(tX, tY, idx, lr)
        state = omlp.adam_step(params, _params_list(grad.cpu().numpy()), state, lr)
        got = _params_list(trainer.params.cpu().numpy())
        m = _params_list(trainer.m.cpu().numpy())
        v = _params_list(trainer.v.cpu().numpy())
        for a, b in zip(got, params):
            assert np.abs(a - b).max() <= 1e-6, step
        for a, b in zip(m, state[1]):
            assert np.abs(a - b).max() <= 1e-6 * max(np.abs(b).max(), 1e-30), step
        for a, b in zip(v, state[2]):
            assert np.abs(a - b).max() <= 5e-5 * max(np.abs(b).max(), 1e-30), step


def test_device_dataset_matches_oracle_features():
    torch = _torch()
    cfg = configs.scaled(configs.TORUS_UNIFORM, (32, 16, 16), block=(16, 16, 16))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    grid = grmhd.Grid(cfg, state=state)
    grid.step(2)
    P, B, G = grid.extract_cells()
    P2, B2, G2 = learned.synthetic_states(G, 2000, seed=3)
    gam = cfg["gam"]
    for (p, b, g) in ((P, B, G), (P2, B2, G2)):
        U = grmhd.prim2cons_batch(p, b, g, gam)
        X, Y, ok = grmhd.mlp_dataset(U, p, g, gam)
        gn = g.cpu().numpy()
        n = gn.shape[1]
        gcov = np.zeros((4, 4, n))
        gcon = np.zeros((4, 4, n))
        for q, (a, c) in enumerate([(0, 0), (0, 1), (0, 3), (1, 1), (1, 3), (2, 2), (3, 3)]):
            gcov[a, c] = gcov[c, a] = gn[q]
        for q, (a, c) in enumerate([(0, 0), (0, 1), (1, 1), (1, 3), (2, 2), (3, 3)]):
            gcon[a, c] = gcon[c, a] = gn[7 + q]
        Un = U.cpu().numpy()
        fx = omlp.features(Un, gcov, gcon, gn[13], gn[14], gam).T
        fy = omlp.targets(p.cpu().numpy(), gcov, gam).T
        okn = ok.cpu().numpy().astype(bool)
        assert okn.mean() > 0.99
        Xn, Yn = X.cpu().numpy()[okn], Y.cpu().numpy()[okn]
        scale = np.maximum(np.abs(fx[okn]), 1.0)
        assert np.abs(Xn - fx[okn]).max() / 1.0 < 1e-4 * np.abs(fx[okn]).max()
        assert np.allclose(Yn, fy[okn], rtol=1e-5, atol=1e-5)


def _trained_blob(cfg, state, steps=400):
    torch = _torch()
    grid = grmhd.Grid(cfg, state=state)
    chunks = []
    for _ in range(2):
        grid.step(2)
        chunks.append(grid.extract_cells())
    chunks.append(learned.synthetic_states(chunks[0][2], 50000, seed=5))
    X, Y, norm = learned.build_dataset(chunks, cfg["gam"])
    trainer, losses = learned.train(X, Y, steps=steps, batch=2048, lr=3e-3, log_every=50)
    say(f"[mlp] training losses {losses}")
    return grmhd.mlp_pack(trainer.params, norm), losses


def test_training_reduces_loss():
    cfg = configs.scaled(configs.TORUS_UNIFORM, (32, 16, 16), block=(16, 16, 16))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    _, losses = _trained_blob(cfg, state, steps=300)
    assert losses[-1][1] < 0.2 * losses[0][1]


def test_learned_guess_keeps_the_evolution():
    """the Newton solve still converges to the same root: learned-guess and plain-guess
    runs agree to the parity bar; report the Newton iteration counts of both"""
    cfg = configs.scaled(configs.TORUS_UNIFORM, (64, 32, 32), block=(32, 32, 32))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    blob, _ = _trained_blob(cfg, state)
    gp = grmhd.Grid(cfg, state=state)
    gm = grmhd.Grid(cfg, state=state, mlp_blob=blob)
    sp = gp.step(4)
    sm = gm.step(4)
    ip = np.array(sp.c2p_iter_hist[:63])
    im = np.array(sm.c2p_iter_hist[:63])
    mean = lambda h: (np.arange(63) * h).sum() / h.sum()
    say(f"[mlp] mean Newton iterations plain {mean(ip):.3f} learned {mean(im):.3f}; "
        f"tiers plain {list(sp.c2p_tier)} learned {list(sm.c2p_tier)}")
    a = gp.get_state()
    b = gm.get_state()
    assert np.max(np.abs(a[0][0] - b[0][0]) / a[0][0]) < 1e-11
    assert np.max(np.abs(a[0][1] - b[0][1]) / (a[0][0] + a[0][1])) < 1e-11
    for v in (2, 3, 4):
        assert np.abs(a[0][v] - b[0][v]).max() <= 1e-11 * np.abs(a[0][v]).max()
    assert sm.c2p_tier[4] == 0


def test_learned_guess_runs_where_the_plain_guess_is_poor():
    """The in-loop gate: with a strongly perturbed initial state (50% pressure noise,
    velocity kicks) some workgroups' plain guesses are poor, the network runs there
    (mlp_guesses > 0), and the evolution still matches the plain-guess run to the parity
    bar, with no more fallbacks or failed inversions than the plain-guess run."""
    cfg = configs.scaled(configs.TORUS_UNIFORM, (64, 32, 32), block=(32, 32, 32))
    init = dict(configs.TORUS_INIT, amp=0.5)
    state = initdata.torus_state(cfg["n"], **init)
    rng = np.random.default_rng(11)
    P = state[0].copy()
    P[2:5] += 0.1 * rng.standard_normal(P[2:5].shape) * (P[0] > 1e-2)
    state = (P, *state[1:])
    blob, _ = _trained_blob(cfg, state, steps=300)
    gp = grmhd.Grid(cfg, state=state)
    gm = grmhd.Grid(cfg, state=state, mlp_blob=blob)
    sp = gp.step(2)
    sm = gm.step(2)
    say(f"[mlp] gated learned starts {sm.mlp_guesses} of {sum(sm.c2p_tier)} inversions; "
        f"tiers plain {list(sp.c2p_tier)} learned {list(sm.c2p_tier)}")
    assert sm.mlp_guesses > 0 and sp.mlp_guesses == 0
    assert sum(sm.c2p_tier[2:]) <= sum(sp.c2p_tier[2:]) and sm.c2p_tier[4] <= sp.c2p_tier[4]
    a = gp.get_state()
    b = gm.get_state()
    assert np.max(np.abs(a[0][0] - b[0][0]) / a[0][0]) < 1e-11
    assert np.max(np.abs(a[0][1] - b[0][1]) / (a[0][0] + a[0][1])) < 1e-11
    for v in (2, 3, 4):
        assert np.abs(a[0][v] - b[0][v]).max() <= 1e-11 * np.abs(a[0][v]).max()


def test_learned_guess_gain_over_a_cold_start():
    """What the network adds where no previous state exists (a standalone inversion of
    conserved states): Newton from the learned guess against Newton from a generic
    start (density D, internal energy D, at rest), both at tolerance 1e-12 with the
    same fallbacks.  Inside the evolution the previous step's state is already an
    excellent start (see the test above); this measures the cold-start case."""
    torch = _torch()
    cfg = configs.scaled(configs.TORUS_UNIFORM, (64, 32, 32), block=(32, 32, 32))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    blob, _ = _trained_blob(cfg, state)
    grid = grmhd.Grid(cfg, state=state)
    grid.step(6)
    P, B, G = grid.extract_cells()
    P2, B2, G2 = learned.synthetic_states(G, 200000, seed=99)      # held-out draws
    gam = cfg["gam"]
    for name, (p, b, g) in (("torus cells", (P, B, G)), ("synthetic", (P2, B2, G2))):
        U = grmhd.prim2cons_batch(p, b, g, gam)
        D = g[14] * U[0] / g[13]
        cold = torch.zeros_like(p)
        cold[0] = D
        cold[1] = D
        Pc, ic, tc = grmhd.cons2prim_batch(U, g, cold, cold, gam)
        Pm, im, tm = grmhd.cons2prim_batch(U, g, None, cold, gam, mlp_blob=blob)
        ic, tc, im, tm = (x.cpu().numpy() for x in (ic, tc, im, tm))
        ok = (tc <= 1) & (tm <= 1)
        mc, mm = ic[tc == 0].mean(), im[tm == 0].mean()
        say(f"[mlp] cold start, {name}: mean Newton iterations generic {mc:.2f} learned {mm:.2f}; "
            f"first-guess failures generic {(tc >= 1).mean():.4f} learned {(tm >= 1).mean():.4f}; "
            f"tiers generic {np.bincount(tc, minlength=5)} learned {np.bincount(tm, minlength=5)}")
        # both reach the same root where both Newton solves converged
        a, b2 = Pc.cpu().numpy()[:, ok], Pm.cpu().numpy()[:, ok]
        assert np.max(np.abs(a[0] - b2[0]) / a[0]) < 1e-10
        assert mm < mc
        assert (tm >= 1).mean() <= (tc >= 1).mean()
