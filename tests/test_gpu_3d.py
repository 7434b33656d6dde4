"""3-D operator pair on the GPU vs the FP64 oracle (relative L2 <= 1e-5 per
application), every 3-D tile variant, both background strategies, and the
dot-product identity at the 256 x 320 x 320 workload's full size."""
import numpy as np
import pytest

import synth
from gpu_helpers import add_shot, f32, open_ctx, oracle_problem, rel, split

pytestmark = pytest.mark.gpu
OP_TOL = 1e-5


def small3d():
    """Several XY tiles with ragged edges, two z chunks, a sponge width that
    is not a multiple of 32, shots of different length, receivers on a
    plane plus one deep receiver and one repeated position."""
    nz, ny, nx, nb = 30, 19, 37, 7
    r = np.random.default_rng(33)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    vel = 1700.0 + 800.0 * z / (nz - 1) + 60.0 * r.uniform(-1, 1, (nz, ny, nx))
    m = r.uniform(-0.1, 0.1, (nz, ny, nx)) * (r.uniform(size=(nz, ny, nx)) < 0.2)
    ry, rx = np.meshgrid(np.arange(1, ny - 1, 3), np.arange(2, nx - 1, 4),
                         indexing="ij")
    rec = np.stack([np.full(rx.size, 2), ry.ravel(), rx.ravel()], 1)
    rec = np.concatenate([rec, [[nz - 2, ny // 2, nx // 2]], rec[5:6]], 0)
    rec = rec.astype(np.int32)
    shots = [synth.Shot(0, (2, 4, 5), rec.copy(), 140, 30.0),
             synth.Shot(1, (3, ny - 3, nx - 6), rec.copy(), 121, 26.0),
             synth.Shot(2, (1, ny // 2, nx // 2), rec[:40].copy(), 133, 28.0)]
    return synth.Workload("small3d", -1, 3, nz, ny, nx, nb, 10.0, 1e-3, 140,
                          30.0, vel, m, shots, Q=3, S=1, niter=5,
                          lam_rel=0.01)


@pytest.fixture(scope="module")
def case():
    w = small3d()
    prob = oracle_problem(w)
    idx = [0, 1, 2]
    m32 = f32(w.m_true)
    born = prob.born(m32.astype(np.float64), idx)
    r = [f32(synth.gaussian((s.nt, s.nrec), 70 + i))
         for i, s in enumerate(w.shots)]
    adj = prob.adjoint([x.astype(np.float64) for x in r], idx)
    return w, idx, m32, born, r, adj


def _check(ctx, w, idx, m32, born, r, adj):
    got = split(w, idx, ctx.apply_born(m32))
    for g_, w_ in zip(got, born):
        assert rel(g_, w_) <= OP_TOL
    g = ctx.apply_adjoint(np.concatenate([x.ravel() for x in r]))
    assert rel(g, adj) <= OP_TOL


@pytest.mark.parametrize("ckpt", [0, 9])
@pytest.mark.parametrize("variant", range(8))
def test_every_3d_tile_matches_oracle(case, variant, ckpt):
    w, idx, m32, born, r, adj = case
    print(f"3-D variant {variant} ckpt={ckpt}", flush=True)
    ctx = open_ctx(w, q_max=3, ckpt_interval=ckpt)
    ctx.set_tile(variant)
    for i in idx:
        add_shot(ctx, w, i)
    for rg in (0, 1):
        ctx.set_resident_grid(rg)
        _check(ctx, w, idx, m32, born, r, adj)
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_3d_exec_modes_match_oracle(case, mode):
    w, idx, m32, born, r, adj = case
    ctx = open_ctx(w, q_max=3, ckpt_interval=-1)
    ctx.set_exec(mode)
    for i in idx:
        add_shot(ctx, w, i)
    _check(ctx, w, idx, m32, born, r, adj)
    ctx.close()


def test_3d_window_solve_matches_oracle(case):
    import oracle
    w, idx, m32, born, r, adj = case
    prob = oracle_problem(w)
    d = [f32(x) for x in born]
    lam = 0.01 * oracle.power_norm(prob, idx, 10, seed=2)
    ref = oracle.cgls(prob, idx, [x.astype(np.float64) for x in d], lam, 4)
    ctx = open_ctx(w, lam=lam, q_max=3, ckpt_interval=-1)
    for i in idx:
        add_shot(ctx, w, i, d[i])
    st = ctx.solve_window(4)
    assert st["iters"] == 4
    assert rel(ctx.image(), ref.m) <= 1e-4
    ctx.close()


def test_3d_full_size_shot_matches_oracle():
    """Shot 0 of the 256 x 320 x 320 workload at full spatial size (296 x
    360 x 360 padded, 128 x 128 receivers) in the bench's launch choice
    (tile variant 0, background checkpointed every 45 steps), for its first
    120 time steps so the oracle finishes in about half a minute: A m and
    A^T r against the oracle, m a smoothed seeded Gaussian field (the early
    wavefield only reaches the top cells, where the layered reflectivity is
    zero), r seeded Gaussian samples."""
    import bench
    from scipy.ndimage import gaussian_filter
    w = synth.layered3d_256x320x320()
    s0 = w.shots[0]
    nt = 120
    shot = synth.Shot(0, s0.src, s0.rec, nt, s0.f0)
    m = f32(gaussian_filter(synth.gaussian(w.model_shape, 11), 3.0))
    r = f32(synth.gaussian((nt, s0.nrec), 12))
    print("256x320x320 shot 0, 120 steps, bench launch choice", flush=True)
    ctx = open_ctx(w, q_max=1, ckpt_interval=-1)
    ctx.set_tile(bench.DEFAULT_TILE3)
    ctx.update(0, shot.src, shot.rec, nt, shot.f0, None)
    d = np.asarray(ctx.apply_born(m)).reshape(nt, s0.nrec)
    g = np.asarray(ctx.apply_adjoint(r.ravel()))
    ctx.close()
    prob = oracle_problem(w, shots=[shot])
    want_d = prob.born_shot(0, m.astype(np.float64))
    want_g = prob.adjoint_shot(0, r.astype(np.float64))
    eb, ea = rel(d, want_d), rel(g, want_g)
    print(f"full-size 3-D shot: born {eb:.2e} adjoint {ea:.2e}", flush=True)
    assert eb <= 1e-5 and ea <= 1e-5


def test_3d_full_size_dot_product():
    """<A m1, d> = <m1, A^T d> on the 256 x 320 x 320 model (padded
    296 x 360 x 360), 128 x 128 receivers, nt = 2000, two shots,
    checkpointed background. m1 and m2 are seeded Gaussian fields smoothed
    over 3 cells and d = A m2, so neither inner product is a small remainder
    of cancelling terms."""
    import torch
    from scipy.ndimage import gaussian_filter
    w = synth.layered3d_256x320x320()
    print("256x320x320 full-size dot test", flush=True)
    ctx = open_ctx(w, q_max=2, device=True, ckpt_interval=-1)
    for i in (0, 9):
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
    m1, m2 = (torch.from_numpy(f32(gaussian_filter(
        synth.gaussian(w.model_shape, k), 3.0))).cuda() for k in (5, 7))
    d = ctx.apply_born(m2)
    lhs = float(torch.dot(ctx.apply_born(m1).double(), d.double()))
    rhs = float(torch.dot(m1.double().ravel(),
                          ctx.apply_adjoint(d).double().ravel()))
    ctx.close()
    err = abs(lhs - rhs) / abs(lhs)
    print(f"dot test: lhs {lhs:.9e} rhs {rhs:.9e} rel {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("ckpt", [0, 9])
def test_3d_background_window_matches_oracle(case, ckpt):
    """3-D finite-difference modelling (background wavefield at the
    receivers, shots of different length, a deep and a repeated receiver)
    against the oracle's."""
    w, idx = case[0], case[1]
    ctx = open_ctx(w, q_max=3, ckpt_interval=ckpt)
    for i in idx:
        add_shot(ctx, w, i)
    got = split(w, idx, ctx.background_window())
    prob = oracle_problem(w)
    for k, i in enumerate(idx):
        _, want = prob.background_shot(i, want_rec=True)
        assert rel(got[k], want) <= OP_TOL
    ctx.close()
