"""Execution forms and launch tuning through the C ABI: the persistent
single-launch operator pair (against batched launches and the oracle, and
its bounded barrier wait forced to give up), two concurrent launch chains
(against one, bitwise, and the oracle), the autotuner (a valid choice, the
window and image left as they were, results against the oracle after
tuning) and the 3-D z chunk."""
import numpy as np
import pytest

import synth
from gpu_helpers import (add_shot, f32, open_ctx, oracle_problem, ragged2d,
                         rel, split)
from test_gpu_3d import small3d

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
IMG_TOL = 1e-4
SEGMENT_VARIANTS = [21, 22, 23, 24]


@pytest.fixture(scope="module")
def P():
    import paper_1801_00819_amd as P
    return P


@pytest.mark.parametrize("variant", SEGMENT_VARIANTS)
def test_persistent_matches_batched_and_oracle(P, variant):
    """The ragged 3-shot window (three nt, a repeated and deep receivers):
    the persistent launch gives the batched launches' results bitwise (the
    same work items, one grid barrier between two-step levels instead of a
    launch boundary), and both match the oracle."""
    w = ragged2d()
    idx = [0, 1, 2]
    print(f"persistent, variant {variant}", flush=True)
    ctx = open_ctx(w, q_max=3)
    ctx.set_tuning(variant, 2, 5, 2, 4)
    for i in idx:
        add_shot(ctx, w, i)
    m32 = f32(w.m_true)
    r = np.concatenate([f32(synth.gaussian((w.shots[i].nt, w.shots[i].nrec),
                                           50 + i)).ravel() for i in idx])
    ctx.set_exec(P.BRLS_EXEC_BATCHED)
    d_b, g_b = ctx.apply_born(m32), ctx.apply_adjoint(r)
    ctx.set_exec(P.BRLS_EXEC_PERSISTENT)
    d_p, g_p = ctx.apply_born(m32), ctx.apply_adjoint(r)
    assert np.array_equal(d_p, d_b) and np.array_equal(g_p, g_b)
    prob = oracle_problem(w)
    for g_, w_ in zip(split(w, idx, d_p),
                      prob.born(m32.astype(np.float64), idx)):
        assert rel(g_, w_) <= OP_TOL
    parts = split(w, idx, r)
    assert rel(g_p, prob.adjoint([x.astype(np.float64) for x in parts],
                                 idx)) <= OP_TOL
    ctx.close()


def test_persistent_chain_matches_oracle(P):
    """The 64 x 64 block-row chain (3 windows of 2 shots, 10 iterations)
    with every operator application one persistent launch."""
    import oracle
    from test_gpu_parity import _chain_inputs, _gpu_chain
    w = synth.layers2d_64x64()
    prob, data, lam = _chain_inputs(w, 0)
    ref = oracle.chain(prob, [d.astype(np.float64) for d in data],
                       w.windows(), lam, w.niter)
    ctx = open_ctx(w, lam=lam, q_max=w.Q)
    ctx.set_tuning(24, 4, 5, 4, 5)
    ctx.set_exec(P.BRLS_EXEC_PERSISTENT)
    img = _gpu_chain(ctx, w, data, w.niter)
    ctx.close()
    assert rel(img, ref.m) <= IMG_TOL


def test_persistent_barrier_gives_up_and_recovers(P):
    """Spin limit 0: every block that arrives at a grid barrier before the
    last gives up at once, the launch ends and the call reports
    BRLS_EDEVICE (no wait can hang). With the limit restored the next
    application is right again."""
    from paper_1801_00819_amd import _lib as L
    w = synth.layers2d_64x64()
    ctx = open_ctx(w, q_max=2)
    ctx.set_tuning(24, 4, 5, 4, 5)
    for i in (0, 1):
        add_shot(ctx, w, i)
    m32 = f32(w.m_true)
    ctx.set_exec(P.BRLS_EXEC_BATCHED)
    want = ctx.apply_born(m32)
    ctx.set_exec(P.BRLS_EXEC_PERSISTENT)
    ctx.set_spin_limit(0)
    with pytest.raises(P.BrlsError) as e:
        ctx.apply_born(m32)
    assert e.value.code == L.BRLS_EDEVICE and "gave up" in str(e.value)
    ctx.set_spin_limit(1 << 20)
    assert np.array_equal(ctx.apply_born(m32), want)
    ctx.close()


def test_persistent_needs_a_segment_variant(P):
    w = synth.layers2d_64x64()
    ctx = open_ctx(w, q_max=2)
    ctx.set_tuning(18, 1, 0, 4, 1)
    with pytest.raises(P.BrlsError):
        ctx.set_exec(P.BRLS_EXEC_PERSISTENT)
    ctx.set_tuning(24, 4, 5, 4, 5)
    ctx.set_exec(P.BRLS_EXEC_PERSISTENT)
    with pytest.raises(P.BrlsError):
        ctx.set_tuning(18, 1, 0, 4, 1)
    ctx.close()
    ck = open_ctx(w, q_max=2, ckpt_interval=-1)
    with pytest.raises(P.BrlsError):
        ck.set_exec(P.BRLS_EXEC_PERSISTENT)
    ck.close()


def test_autotune_2d(P):
    """brls_autotune on the ragged window: the chosen variant is valid, the
    choice is the context's tuning, the window and the image are as before,
    and the operators after tuning match the oracle."""
    w = ragged2d()
    idx = [0, 1, 2]
    ctx = open_ctx(w, q_max=3)
    for i in idx:
        add_shot(ctx, w, i)
    img0 = f32(synth.gaussian(w.model_shape, 8) * 1e-3)
    ctx.set_image(img0)
    best = ctx.autotune()
    t = ctx.get_tuning()
    print(f"autotune 2-D: variant {best}, {t}", flush=True)
    assert 0 <= best < len(P.tile_variants()) and t["variant"] == best
    assert ctx.window() == idx
    assert np.array_equal(ctx.image(), img0)
    prob = oracle_problem(w)
    m32 = f32(w.m_true)
    for g_, w_ in zip(split(w, idx, ctx.apply_born(m32)),
                      prob.born(m32.astype(np.float64), idx)):
        assert rel(g_, w_) <= OP_TOL
    r = [f32(synth.gaussian((w.shots[i].nt, w.shots[i].nrec), 60 + i))
         for i in idx]
    g = ctx.apply_adjoint(np.concatenate([x.ravel() for x in r]))
    assert rel(g, prob.adjoint([x.astype(np.float64) for x in r],
                               idx)) <= OP_TOL
    ctx.close()


def test_autotune_3d_and_z_chunks(P):
    """The 3-D window: every z chunk (the autotuner's 8, 16, 32, 64 planes
    and a ragged 7) gives the oracle's operators; brls_autotune picks one
    of the tried chunks and its results match the oracle."""
    w = small3d()
    idx = [0, 1, 2]
    prob = oracle_problem(w)
    m32 = f32(w.m_true)
    born = prob.born(m32.astype(np.float64), idx)
    r = [f32(synth.gaussian((s.nt, s.nrec), 70 + i))
         for i, s in enumerate(w.shots)]
    adj = prob.adjoint([x.astype(np.float64) for x in r], idx)
    ctx = open_ctx(w, q_max=3)
    for i in idx:
        add_shot(ctx, w, i)
    assert ctx.get_zchunk() == 32
    for zc in (8, 16, 7, 64, 32):
        ctx.set_zchunk(zc)
        assert ctx.get_zchunk() == zc
        for g_, w_ in zip(split(w, idx, ctx.apply_born(m32)), born):
            assert rel(g_, w_) <= OP_TOL
        g = ctx.apply_adjoint(np.concatenate([x.ravel() for x in r]))
        assert rel(g, adj) <= OP_TOL
    best = ctx.autotune()
    print(f"autotune 3-D: variant {best}, z chunk {ctx.get_zchunk()}, "
          f"{ctx.get_tuning()}", flush=True)
    assert ctx.get_zchunk() in (8, 16, 32, 64)
    for g_, w_ in zip(split(w, idx, ctx.apply_born(m32)), born):
        assert rel(g_, w_) <= OP_TOL
    ctx.close()
    c2 = open_ctx(synth.layers2d_64x64(), q_max=1)
    with pytest.raises(P.BrlsError):
        c2.set_zchunk(16)
    c2.close()


@pytest.mark.parametrize("tuning", [(24, 1, 5, 1, 5), (18, 1, 0, 1, 1),
                                    (12, 2, 1, 2, 0)])
def test_two_chains_bitwise_and_oracle(P, tuning):
    """The ragged 3-shot window (nt 3 ways, a repeated and deep receivers)
    with one shot per work item (3 groups: chains of 2 and 1 groups,
    different lengths): two concurrent launch chains give one chain's
    results bitwise, in batched and graph modes, and match the oracle."""
    w = ragged2d()
    idx = [0, 1, 2]
    print(f"two chains, launch choice {tuning}", flush=True)
    ctx = open_ctx(w, q_max=3)
    ctx.set_tuning(*tuning)
    assert ctx.get_chains() == 2
    for i in idx:
        add_shot(ctx, w, i)
    m32 = f32(w.m_true)
    r = np.concatenate([f32(synth.gaussian((w.shots[i].nt, w.shots[i].nrec),
                                           60 + i)).ravel() for i in idx])
    out = {}
    for mode in (P.BRLS_EXEC_BATCHED, P.BRLS_EXEC_GRAPH):
        ctx.set_exec(mode)
        for ch in (1, 2):
            ctx.set_chains(ch)
            out[(mode, ch)] = (ctx.apply_born(m32), ctx.apply_adjoint(r))
    d1, g1 = out[(P.BRLS_EXEC_BATCHED, 1)]
    for d, g in out.values():
        assert np.array_equal(d, d1) and np.array_equal(g, g1)
    prob = oracle_problem(w)
    for g_, w_ in zip(split(w, idx, d1),
                      prob.born(m32.astype(np.float64), idx)):
        assert rel(g_, w_) <= OP_TOL
    assert rel(g1, prob.adjoint([x.astype(np.float64)
                                 for x in split(w, idx, r)], idx)) <= OP_TOL
    with pytest.raises(P.BrlsError):
        ctx.set_chains(3)
    assert ctx.get_chains() == 2
    ctx.close()


def test_two_chains_window_chain_matches_oracle(P):
    """The 64 x 64 block-row chain (3 windows of 2 shots, 10 iterations),
    one shot per work item so that every window's operators run as two
    concurrent chains, graph mode: the final image against the oracle's."""
    import oracle
    w = synth.layers2d_64x64()
    prob = oracle_problem(w)
    clean = [prob.born_shot(i, f32(w.m_true).astype(np.float64))
             for i in range(len(w.shots))]
    sig = w.noise_rel * np.sqrt(np.mean(np.concatenate(
        [c.ravel() for c in clean]) ** 2))
    data = [f32(c + sig * synth.gaussian(c.shape, 4200 + i))
            for i, c in enumerate(clean)]
    wins = w.windows()
    lam = w.lam_rel * oracle.power_norm(prob, wins[0], 10, seed=3)
    ref = oracle.chain(prob, [d.astype(np.float64) for d in data], wins, lam,
                       w.niter)
    ctx = open_ctx(w, lam=lam, q_max=w.Q)
    ctx.set_tuning(24, 1, 5, 1, 5)
    held = []
    for win in wins:
        for i in list(held):
            if i not in win:
                ctx.downdate(i)
                held.remove(i)
        for i in win:
            if i not in held:
                add_shot(ctx, w, i, data[i])
                held.append(i)
        ctx.solve_window(w.niter)
    img = ctx.image()
    ctx.close()
    e = rel(img, ref.m)
    print(f"two-chain 64x64 chain vs oracle: {e:.2e}")
    assert e <= IMG_TOL


@pytest.mark.parametrize("case", ["3d-stored", "3d-ckpt", "2d-ckpt"])
def test_two_chains_with_checkpoints_bitwise(P, case):
    """Two launch chains against one, bitwise, where they are not the
    default: 3-D, and checkpointed backgrounds (each chain restores its
    shots' checkpoints and recomputes their backgrounds segment by segment;
    interval 7 in 3-D, 5 in 2-D); graph mode, and the oracle."""
    w = small3d() if case.startswith("3d") else ragged2d()
    idx = [0, 1, 2]
    ckpt = 0 if case == "3d-stored" else (7 if case == "3d-ckpt" else 5)
    print(f"two chains, {case}", flush=True)
    ctx = open_ctx(w, q_max=3, ckpt_interval=ckpt)
    if case == "2d-ckpt":
        ctx.set_tuning(12, 1, 0, 1, 0)
    assert ctx.get_chains() == 1  # not the default here
    for i in idx:
        add_shot(ctx, w, i)
    m32 = f32(w.m_true)
    r = np.concatenate([f32(synth.gaussian((w.shots[i].nt, w.shots[i].nrec),
                                           80 + i)).ravel() for i in idx])
    out = {}
    for ch in (1, 2):
        ctx.set_chains(ch)
        out[ch] = (ctx.apply_born(m32), ctx.apply_adjoint(r))
    ctx.close()
    assert np.array_equal(out[1][0], out[2][0])
    assert np.array_equal(out[1][1], out[2][1])
    prob = oracle_problem(w)
    for g_, w_ in zip(split(w, idx, out[2][0]),
                      prob.born(m32.astype(np.float64), idx)):
        assert rel(g_, w_) <= OP_TOL
    assert rel(out[2][1], prob.adjoint([x.astype(np.float64)
                                        for x in split(w, idx, r)],
                                       idx)) <= OP_TOL
