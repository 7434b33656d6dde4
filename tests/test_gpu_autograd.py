"""Differentiable Born modelling (BornFn) on the GPU: gradients of
0.5 ||A m - d||^2 against the FP64 oracle's adjoint and against central
finite differences, with background checkpoints every ceil(sqrt(nt)) steps."""
import numpy as np
import pytest

import synth
from gpu_helpers import f32, open_ctx, oracle_problem, rel

pytestmark = pytest.mark.gpu


def _window(ctx, w, idx):
    for i in idx:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, None)


def test_gradient_matches_oracle_adjoint():
    import torch

    from paper_1801_00819_amd.autograd import misfit
    w = synth.layers2d_64x64()
    idx = [0, 1]
    ctx = open_ctx(w, q_max=2, device=True, ckpt_interval=-1)
    _window(ctx, w, idx)
    prob = oracle_problem(w)
    d = [f32(x) for x in prob.born(f32(w.m_true).astype(np.float64), idx)]
    m0 = f32(0.5 * w.m_true)
    m = torch.from_numpy(m0).cuda().requires_grad_(True)
    dt = torch.from_numpy(np.concatenate([x.ravel() for x in d])).cuda()
    loss = misfit(m, dt, ctx)
    loss.backward()
    r = [a - b.astype(np.float64) for a, b in
         zip(prob.born(m0.astype(np.float64), idx), d)]
    want = prob.adjoint(r, idx)
    assert rel(m.grad.cpu().numpy(), want) <= 1e-5
    ctx.close()


def test_checkpointed_and_cached_backgrounds_agree():
    import torch
    w = synth.layers2d_64x64()
    idx = [0, 1]
    a = open_ctx(w, q_max=2, device=True, ckpt_interval=-1)
    b = open_ctx(w, q_max=2, device=True, ckpt_interval=0)
    # the same float32 background arithmetic in both (stored sources
    # default to a float64 background)
    b.set_precision(32, 64)
    _window(a, w, idx)
    _window(b, w, idx)
    m = torch.from_numpy(f32(w.m_true)).cuda()
    da, db = a.apply_born(m), b.apply_born(m)
    assert rel(da.cpu().numpy(), db.cpu().numpy()) <= 1e-6
    ga, gb = a.apply_adjoint(da), b.apply_adjoint(da)
    assert rel(ga.cpu().numpy(), gb.cpu().numpy()) <= 1e-6
    assert a.memory_bytes() < b.memory_bytes()
    a.close()
    b.close()


@pytest.fixture(scope="module")
def big_window():
    import torch
    w = synth.faulted2d_512x1024()
    idx = list(range(8))
    ctx = open_ctx(w, q_max=8, device=True, ckpt_interval=-1)
    _window(ctx, w, idx)
    m_true = torch.from_numpy(f32(w.m_true)).cuda()
    d = ctx.apply_born(m_true)
    yield w, idx, ctx, m_true, d
    ctx.close()


def test_full_size_gradient_vs_finite_differences(big_window):
    """Central differences of the exactly quadratic misfit along 16 seeded
    directions, 512 x 1024 model, 8-shot window, nt = 3000, step h = 1e-3
    of ||m||. Directions are Gaussian fields smoothed over 4 cells: white
    noise lies mostly outside the band the Born operator sees, where the
    float32 rounding of the two misfit evaluations dominates their small
    difference. Compared as a vector over the 16 directions, and each
    direction against the largest directional derivative."""
    import torch
    from scipy.ndimage import gaussian_filter

    from paper_1801_00819_amd.autograd import misfit
    w, idx, ctx, m_true, d = big_window
    m0 = 0.5 * m_true
    m = m0.clone().requires_grad_(True)
    loss = misfit(m, d, ctx)
    loss.backward()
    g = m.grad.double()
    fds, ans = [], []
    h = 1e-3
    for k in range(16):
        p = gaussian_filter(synth.gaussian(w.model_shape, 2000 + k)[:, 0, :],
                            4.0)[:, None, :]
        p = torch.from_numpy(np.ascontiguousarray(p)).cuda()
        p *= torch.linalg.vector_norm(m0.double()) / torch.linalg.vector_norm(p)
        mp = (m0.double() + h * p).float()
        mm = (m0.double() - h * p).float()
        # the direction actually applied after rounding m0 +- h p to float32
        p_eff = (mp.double() - mm.double()) / (2 * h)
        with torch.no_grad():
            fp = misfit(mp, d, ctx)
            fm = misfit(mm, d, ctx)
        fds.append(float((fp - fm) / (2 * h)))
        ans.append(float(torch.sum(g * p_eff)))
    fds, ans = np.array(fds), np.array(ans)
    err = np.linalg.norm(fds - ans) / np.linalg.norm(ans)
    worst = np.max(np.abs(fds - ans)) / np.max(np.abs(ans))
    print(f"FD vs autograd over 16 directions: rel L2 {err:.2e}, worst "
          f"direction {worst:.2e} of the largest directional derivative, "
          f"worst own-relative {np.max(np.abs(fds - ans) / np.abs(ans)):.2e}")
    assert err <= 1e-4
    # every direction, against the common scale of the directional
    # derivatives (a direction nearly orthogonal to the gradient has a tiny
    # derivative that the misfits' rounding dominates)
    assert worst <= 1e-4


def test_full_size_gradient_matches_oracle_adjoint_one_shot(big_window):
    """Backward of the checkpointed Born operator vs the FP64 oracle adjoint
    for one shot of the 512 x 1024 window (residual zero on the others)."""
    import torch

    from paper_1801_00819_amd.autograd import born
    w, idx, ctx, m_true, d = big_window
    s = w.shots[3]
    n = s.nt * s.nrec
    r3 = f32(synth.gaussian((s.nt, s.nrec), 303))
    gd = torch.zeros(8 * n, dtype=torch.float32, device="cuda")
    gd[3 * n:4 * n] = torch.from_numpy(r3.ravel()).cuda()
    m = m_true.clone().requires_grad_(True)
    out = born(m, ctx)
    out.backward(gd)
    prob = oracle_problem(w, shots=[s])
    want = prob.adjoint_shot(0, r3.astype(np.float64))
    assert rel(m.grad.cpu().numpy(), want) <= 1e-5
