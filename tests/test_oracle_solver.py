"""Pins of the oracle's damped least-squares solver and block-row recursion
against dense linear algebra (eqs. 3-11 of the paper) on tiny problems."""
import json
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def dense_problem(orc):
    w = synth.tiny2d(nz=8, nx=9, nb=4, nt=150, nrec=6, nshots=3, seed=3)
    prob = orc.Problem.from_workload(w)
    M = int(np.prod(prob.grid.model_shape))
    blocks = []
    for i in range(3):
        cols = []
        for j in range(M):
            e = np.zeros(M)
            e[j] = 1.0
            cols.append(prob.born_shot(i, e).ravel())
        blocks.append(np.stack(cols, 1))
    noise = [synth.gaussian(prob.data_shape(i), 100 + i) for i in range(3)]
    data = orc.synthesize_data(prob, w.m_true, 0.01, noise)
    A = np.concatenate(blocks, 0)
    lam = 0.01 * np.linalg.norm(A, 2) ** 2
    return dict(w=w, prob=prob, blocks=blocks, data=data, lam=lam, M=M)


def _textbook_cg(H, b, x0, niter):
    """Hestenes-Stiefel CG on H x = b."""
    x = x0.copy()
    r = b - H @ x
    p = r.copy()
    rr = r @ r
    xs = [x.copy()]
    for _ in range(niter):
        Hp = H @ p
        a = rr / (p @ Hp)
        x = x + a * p
        r = r - a * Hp
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        xs.append(x.copy())
    return xs


def _normal(dp, idx):
    A = np.concatenate([dp["blocks"][i] for i in idx], 0)
    d = np.concatenate([dp["data"][i].ravel() for i in idx])
    H = A.T @ A + dp["lam"] * np.eye(dp["M"])
    return A, d, H, A.T @ d


@pytest.mark.parametrize("warm", [False, True])
def test_cgls_iterates_equal_textbook_cg_on_normal_equations(orc, dense_problem,
                                                              warm):
    dp = dense_problem
    idx = [0, 1]
    A, d, H, b = _normal(dp, idx)
    x0 = synth.gaussian(dp["M"], 5) * 0.05 if warm else np.zeros(dp["M"])
    ref = _textbook_cg(H, b, x0, 8)
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"], 8,
                   m0=x0.reshape(dp["prob"].grid.model_shape),
                   keep_iterates=True)
    assert res.iters == 8
    for k, (xr, xo) in enumerate(zip(ref, res.iterates)):
        rel = np.linalg.norm(xo.ravel() - xr) / max(np.linalg.norm(xr), 1e-300)
        assert rel < 1e-10, (k, rel)


def test_cgls_converges_to_closed_form(orc, dense_problem):
    """Eq. 4: m = (A^T A + lam I)^-1 A^T d."""
    dp = dense_problem
    idx = [0, 1, 2]
    A, d, H, b = _normal(dp, idx)
    exact = np.linalg.solve(H, b)
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"],
                   120)
    assert np.linalg.norm(res.m.ravel() - exact) <= 1e-9 * np.linalg.norm(
        exact)
    # residual norms of the normal equations shrink overall
    assert res.s_norms[-1] < 1e-9 * res.s_norms[0]


def test_one_window_over_all_shots_is_batch_least_squares(orc, dense_problem):
    dp = dense_problem
    A, d, H, b = _normal(dp, [0, 1, 2])
    ch = orc.chain(dp["prob"], dp["data"], [[0, 1, 2]], dp["lam"], 120)
    assert np.linalg.norm(ch.m.ravel() - np.linalg.solve(H, b)) <= 1e-9 * \
        np.linalg.norm(ch.m)


def test_warm_start_does_not_change_the_window_solution(orc, dense_problem):
    """Eq. 11: the warm-started correction reaches the window's own
    least-squares solution whatever the starting image."""
    dp = dense_problem
    idx = [1, 2]
    d = [dp["data"][i] for i in idx]
    a = orc.cgls(dp["prob"], idx, d, dp["lam"], 120)
    m0 = synth.gaussian(dp["prob"].grid.model_shape, 9)
    b = orc.cgls(dp["prob"], idx, d, dp["lam"], 120, m0=m0)
    assert np.linalg.norm(a.m - b.m) <= 1e-9 * np.linalg.norm(a.m)


def test_rls_update_and_downdate_identities(orc, dense_problem):
    """Eqs. 5-9 with the damping folded into P0: the gain-form update equals
    the batch solution of both blocks; the mirror downdate recovers the
    solution of the remaining block; the chain of converged windows equals
    that recursion."""
    dp = dense_problem
    A0, A1, A2 = dp["blocks"]
    d0, d1, d2 = [x.ravel() for x in dp["data"]]
    lam, I = dp["lam"], np.eye(dp["M"])
    P0inv = A0.T @ A0 + lam * I
    m0 = np.linalg.solve(P0inv, A0.T @ d0)
    P1inv = P0inv + A1.T @ A1  # eq. 8
    m1 = m0 + np.linalg.solve(P1inv, A1.T @ (d1 - A1 @ m0))  # eq. 9
    batch01 = np.linalg.solve(A0.T @ A0 + A1.T @ A1 + lam * I,
                              A0.T @ d0 + A1.T @ d1)  # eq. 7
    assert np.linalg.norm(m1 - batch01) <= 1e-10 * np.linalg.norm(batch01)
    # downdate block 0, then update block 2: the window slides by one shot
    P2inv = P1inv - A0.T @ A0
    m2 = m1 - np.linalg.solve(P2inv, A0.T @ (d0 - A0 @ m1))
    only1 = np.linalg.solve(A1.T @ A1 + lam * I, A1.T @ d1)
    assert np.linalg.norm(m2 - only1) <= 1e-9 * np.linalg.norm(only1)
    P3inv = P2inv + A2.T @ A2
    m3 = m2 + np.linalg.solve(P3inv, A2.T @ (d2 - A2 @ m2))
    ch = orc.chain(dp["prob"], dp["data"], [[0, 1], [1, 2]], lam, 150)
    for img, ref in ((ch.images[0], m1), (ch.images[1], m3)):
        assert np.linalg.norm(img.ravel() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_truncated_chain_replays_dense_cg(orc, dense_problem):
    """The truncated, warm-started chain (the method's actual output) equals
    the same chain run with textbook CG on the dense normal equations."""
    dp = dense_problem
    wins = [[0, 1], [1, 2]]
    ch = orc.chain(dp["prob"], dp["data"], wins, dp["lam"], 6)
    x = np.zeros(dp["M"])
    for w, img in zip(wins, ch.images):
        A, d, H, b = _normal(dp, w)
        x = _textbook_cg(H, b, x, 6)[-1]
        assert np.linalg.norm(img.ravel() - x) <= 1e-10 * np.linalg.norm(x)


def test_power_norm_matches_spectral_norm(orc, dense_problem):
    dp = dense_problem
    A = np.concatenate(dp["blocks"][:2], 0)
    est = orc.power_norm(dp["prob"], [0, 1], 60, seed=4)
    assert abs(est - np.linalg.norm(A, 2) ** 2) <= 1e-6 * est


def test_paper_window_schedule():
    """The paper's example: windows of Q = 5 shots, K = 3 dropped and added
    per step, steps t = Q, Q+K, ... over 240 shots."""
    with open(os.path.join(HERE, "golden", "paper_example.json")) as f:
        g = json.load(f)
    Q, K, N = g["window_shots_Q"], g["update_downdate_rank_K"], g["shots"]
    w = synth.tiny2d(nshots=N, nz=4, nx=N + 4, nb=1)
    w.Q, w.S = Q, K
    wins = w.windows()
    ends = [win[-1] + 1 for win in wins]
    assert ends[:-1] == list(range(Q, N + 1, K))[:len(ends) - 1]
    assert all(len(win) == Q for win in wins)
    for a, b in zip(wins, wins[1:-1]):
        assert len(set(a) - set(b)) == K and len(set(b) - set(a)) == K
    assert wins[-1][-1] == N - 1


# --- preconditioned window CG (diagonal illumination) -------------------

def _textbook_pcg(H, b, x0, minv, niter):
    """Preconditioned CG on H x = b with the diagonal preconditioner
    M = diag(1 / minv)."""
    x = x0.copy()
    r = b - H @ x
    z = minv * r
    p = z.copy()
    rz = r @ z
    xs = [x.copy()]
    for _ in range(niter):
        Hp = H @ p
        a = rz / (p @ Hp)
        x = x + a * p
        r = r - a * Hp
        z = minv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        xs.append(x.copy())
    return xs


def test_pcg_with_identity_is_plain_cgls(orc, dense_problem):
    dp = dense_problem
    idx = [0, 1]
    data = [dp["data"][i] for i in idx]
    a = orc.cgls(dp["prob"], idx, data, dp["lam"], 6, keep_iterates=True)
    b = orc.cgls(dp["prob"], idx, data, dp["lam"], 6, keep_iterates=True,
                 minv=np.ones(dp["prob"].grid.model_shape))
    for xa, xb in zip(a.iterates, b.iterates):
        assert np.linalg.norm(xa - xb) <= 1e-13 * max(np.linalg.norm(xa),
                                                      1e-300)


@pytest.mark.parametrize("warm", [False, True])
def test_pcg_iterates_equal_textbook_pcg(orc, dense_problem, warm):
    """The preconditioned least-squares recurrences against preconditioned
    CG on the dense normal matrix (eq. 4), with the illumination
    preconditioner of the window."""
    dp = dense_problem
    idx = [0, 2]
    A, d, H, b = _normal(dp, idx)
    minv = orc.illumination_minv(orc.illumination(dp["prob"], idx)).ravel()
    assert np.all(minv > 0) and np.ptp(minv) > 0
    x0 = synth.gaussian(dp["M"], 6) * 0.05 if warm else np.zeros(dp["M"])
    ref = _textbook_pcg(H, b, x0, minv, 8)
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"],
                   8, m0=x0.reshape(dp["prob"].grid.model_shape),
                   keep_iterates=True,
                   minv=minv.reshape(dp["prob"].grid.model_shape))
    assert res.iters == 8
    for k, (xr, xo) in enumerate(zip(ref, res.iterates)):
        rel = np.linalg.norm(xo.ravel() - xr) / max(np.linalg.norm(xr), 1e-300)
        assert rel < 1e-10, (k, rel)


def test_pcg_converges_to_closed_form(orc, dense_problem):
    dp = dense_problem
    idx = [0, 1, 2]
    A, d, H, b = _normal(dp, idx)
    minv = orc.illumination_minv(orc.illumination(dp["prob"], idx))
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"],
                   150, minv=minv)
    exact = np.linalg.solve(H, b)
    assert np.linalg.norm(res.m.ravel() - exact) <= 1e-9 * np.linalg.norm(
        exact)


def test_illumination_from_recorded_background(orc):
    """The illumination from the background's stored Born-source frames
    equals the same sum formed from the background wavefield recorded at
    every model point (second differences in time taken here)."""
    w = synth.tiny2d(nz=7, nx=8, nb=4, nt=90, nrec=4, nshots=2, seed=9)
    nz, nx = w.nz, w.nx
    zz, xx = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    every = np.stack([zz.ravel(), np.zeros(zz.size, int), xx.ravel()],
                     1).astype(np.int32)
    shots = [synth.Shot(s.id, s.src, every, s.nt, s.f0) for s in w.shots]
    prob = orc.Problem(orc.Grid(2, nz, 1, nx, w.nb, w.h, w.dt),
                       w.vel.astype(np.float64), shots)
    want = np.zeros(nz * nx)
    for i in range(len(shots)):
        _, u = prob.background_shot(i, want_d2u0=False, want_rec=True)
        # u^{-1} = 0: pad one zero level in front
        u = np.concatenate([np.zeros((1, u.shape[1])), u], 0)
        d2 = u[2:] - 2 * u[1:-1] + u[:-2]          # levels n = 0 .. nt-2
        want += np.sum(d2 * d2, axis=0)
    got = orc.illumination(prob, [0, 1]).ravel()
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    assert np.all(got >= 0)


# --- correction-regularised recursion ------------------------------------

def test_correction_regularised_window_closed_form(orc, dense_problem):
    """min ||A m - d||^2 + lam ||m - m_prev||^2 converges to
    (A^T A + lam I)^-1 (A^T d + lam m_prev)."""
    dp = dense_problem
    idx = [0, 1]
    A, d, H, b = _normal(dp, idx)
    m_prev = synth.gaussian(dp["M"], 8) * 0.05
    exact = np.linalg.solve(H, b + dp["lam"] * m_prev)
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"],
                   150, m0=m_prev.reshape(dp["prob"].grid.model_shape),
                   m_ref=m_prev.reshape(dp["prob"].grid.model_shape))
    assert np.linalg.norm(res.m.ravel() - exact) <= 1e-9 * np.linalg.norm(
        exact)


def test_correction_regularised_iterates_are_cg_on_the_correction(
        orc, dense_problem):
    """From m_prev, the iterates are m_prev + the textbook-CG iterates of
    (A^T A + lam I) delta = A^T (d - A m_prev)."""
    dp = dense_problem
    idx = [1, 2]
    A, d, H, b = _normal(dp, idx)
    m_prev = synth.gaussian(dp["M"], 9) * 0.05
    ref = _textbook_cg(H, A.T @ (d - A @ m_prev), np.zeros(dp["M"]), 7)
    shp = dp["prob"].grid.model_shape
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"],
                   7, m0=m_prev.reshape(shp), m_ref=m_prev.reshape(shp),
                   keep_iterates=True)
    for k, (xr, xo) in enumerate(zip(ref, res.iterates)):
        want = m_prev + xr
        rel = np.linalg.norm(xo.ravel() - want) / np.linalg.norm(want)
        assert rel < 1e-10, (k, rel)


def test_correction_chain_keeps_memory(orc, dense_problem):
    """Converged, the correction-regularised chain depends on the windows
    before (each window solution is pulled towards the last), unlike the
    image-regularised chain whose converged window solution does not."""
    dp = dense_problem
    wins = [[0, 1], [1, 2]]
    a = orc.chain(dp["prob"], dp["data"], wins, dp["lam"], 150,
                  correction=True)
    b = orc.chain(dp["prob"], dp["data"], [wins[1]], dp["lam"], 150,
                  correction=True)
    c = orc.chain(dp["prob"], dp["data"], wins, dp["lam"], 150)
    A, d, H, rhs = _normal(dp, wins[1])
    assert np.linalg.norm(c.m.ravel() - np.linalg.solve(H, rhs)) <= \
        1e-9 * np.linalg.norm(rhs)
    prev = a.images[0].ravel()
    assert np.linalg.norm(a.m.ravel() - np.linalg.solve(
        H, rhs + dp["lam"] * prev)) <= 1e-9 * np.linalg.norm(a.m)
    assert np.linalg.norm(a.m - b.m) > 1e-3 * np.linalg.norm(b.m)


# --- per-shot weights: the exponentially weighted window ------------------

def test_weighted_window_closed_form(orc, dense_problem):
    """min sum_j w_j ||A_j m - d_j||^2 + lam ||m||^2 converges to
    (A^T W A + lam I)^-1 A^T W d, W the per-shot weights spread over each
    shot's samples (dense blocks)."""
    dp = dense_problem
    idx, wts = [0, 1, 2], [0.5, 2.0, 0.8]
    A = np.concatenate([dp["blocks"][i] for i in idx], 0)
    d = np.concatenate([dp["data"][i].ravel() for i in idx])
    wv = np.concatenate([np.full(dp["blocks"][i].shape[0], w)
                         for i, w in zip(idx, wts)])
    H = A.T @ (wv[:, None] * A) + dp["lam"] * np.eye(dp["M"])
    exact = np.linalg.solve(H, A.T @ (wv * d))
    res = orc.cgls(dp["prob"], idx, [dp["data"][i] for i in idx], dp["lam"],
                   150, weights=wts)
    assert np.linalg.norm(res.m.ravel() - exact) <= 1e-9 * np.linalg.norm(
        exact)


def test_integer_weight_equals_a_repeated_shot(orc, dense_problem):
    """Weight 2 on a shot gives the iterates of the window that holds the
    shot twice."""
    dp = dense_problem
    d = dp["data"]
    a = orc.cgls(dp["prob"], [0, 1], [d[0], d[1]], dp["lam"], 6,
                 weights=[1.0, 2.0], keep_iterates=True)
    b = orc.cgls(dp["prob"], [0, 1, 1], [d[0], d[1], d[1]], dp["lam"], 6,
                 keep_iterates=True)
    for xa, xb in zip(a.iterates, b.iterates):
        assert np.linalg.norm(xa - xb) <= 1e-11 * max(np.linalg.norm(xb),
                                                       1e-300)


def test_zero_weight_drops_the_shot(orc, dense_problem):
    dp = dense_problem
    d = dp["data"]
    a = orc.cgls(dp["prob"], [0, 1, 2], [d[0], d[1], d[2]], dp["lam"], 6,
                 weights=[1.0, 0.0, 1.0])
    b = orc.cgls(dp["prob"], [0, 2], [d[0], d[2]], dp["lam"], 6)
    assert np.linalg.norm(a.m - b.m) <= 1e-12 * np.linalg.norm(b.m)


def test_forgetting_chain_weights_shots_by_age(orc, dense_problem):
    """Windows {0, 1} then {1, 2} with beta: in the second window shot 1
    (held once before) weighs beta and shot 2 weighs 1; the chain's
    windows are the weighted CG runs from the previous image."""
    dp = dense_problem
    wins, beta = [[0, 1], [1, 2]], 0.6
    ch = orc.chain(dp["prob"], dp["data"], wins, dp["lam"], 5,
                   forgetting=beta)
    first = orc.cgls(dp["prob"], wins[0], [dp["data"][i] for i in wins[0]],
                     dp["lam"], 5)
    second = orc.cgls(dp["prob"], wins[1], [dp["data"][i] for i in wins[1]],
                      dp["lam"], 5, m0=first.m, weights=[beta, 1.0])
    assert np.array_equal(ch.images[0], first.m)
    assert np.array_equal(ch.m, second.m)
    plain = orc.chain(dp["prob"], dp["data"], wins, dp["lam"], 5)
    assert np.linalg.norm(ch.m - plain.m) > 1e-3 * np.linalg.norm(plain.m)


def test_weights_are_checked(orc, dense_problem):
    dp = dense_problem
    d = dp["data"]
    for bad in ([1.0], [1.0, -1.0], [1.0, float("nan")]):
        with pytest.raises(ValueError):
            orc.cgls(dp["prob"], [0, 1], [d[0], d[1]], dp["lam"], 2,
                     weights=bad)
