"""Pins of the FP64 oracle's operator pair against mathematics and physics.

Nothing here compares the oracle with itself: each check is a closed form, a
brute-force matrix construction, a library routine or an invariant.
"""
import numpy as np
import pytest

import synth


# ---------------------------------------------------------------------------
# Stencil: the 8th-order central second difference is exact on polynomials of
# degree <= 9 and must give d2/dx2 (x^p) = p (p-1) x^(p-2) exactly.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ndim,axis", [(2, 0), (2, 2), (3, 0), (3, 1), (3, 2)])
def test_laplacian_exact_on_polynomials(orc, ndim, axis):
    nb = 5
    n = 11
    grid = orc.Grid(ndim, n, n if ndim == 3 else 1, n, nb, 0.5, 1.0)
    shp = grid.padded_shape
    coords = (np.arange(shp[axis]) - (shp[axis] - 1) / 2.0) * grid.h
    sl = [None, None, None]
    sl[axis] = slice(None)
    x = coords[tuple(sl)]
    inner = [slice(4, s - 4) if s > 1 else slice(None) for s in shp]
    for p in range(0, 10):
        u = np.broadcast_to(x ** p, shp).copy()
        lap = orc.laplacian(grid, u)
        exact = np.broadcast_to(p * (p - 1) * x ** max(p - 2, 0) if p >= 2
                                else 0.0 * x, shp)
        err = np.abs(lap[tuple(inner)] - exact[tuple(inner)]).max()
        scale = max(1.0, np.abs(exact[tuple(inner)]).max())
        assert err <= 1e-9 * scale, (p, err)
    # degree 10 is the first the 8th-order scheme gets wrong
    u = np.broadcast_to(x ** 10, shp).copy()
    lap = orc.laplacian(grid, u)
    exact = np.broadcast_to(90 * x ** 8, shp)
    assert np.abs(lap[tuple(inner)] - exact[tuple(inner)]).max() > 1e-3


def test_laplacian_is_symmetric_and_zero_outside(orc):
    grid = orc.Grid(2, 5, 1, 6, 2, 7.0, 1.0)
    N = int(np.prod(grid.padded_shape))
    Lm = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        Lm[:, j] = orc.laplacian(grid, e).ravel()
    assert np.abs(Lm - Lm.T).max() <= 1e-15 * np.abs(Lm).max()
    # Dirichlet: the row of a corner point only sees points inside the grid;
    # the stencil weights sum to zero, so the row sum there is negative.
    assert Lm[0].sum() < 0
    # a point far from every face sees the full 17-point stencil -> row sum 0
    grid2 = orc.Grid(2, 12, 1, 12, 2, 1.0, 1.0)
    e = np.zeros(grid2.padded_shape)
    e[8, 0, 8] = 1.0
    assert abs(orc.laplacian(grid2, np.ones(grid2.padded_shape))[8, 0, 8]) \
        < 1e-12
    assert np.count_nonzero(orc.laplacian(grid2, e)) == 17


# ---------------------------------------------------------------------------
# Medium
# ---------------------------------------------------------------------------
def test_medium_interior_undamped_and_sponge_monotone(orc):
    w = synth.tiny2d(nz=10, nx=14, nb=8)
    grid = orc.Grid(2, w.nz, 1, w.nx, w.nb, w.h, w.dt)
    med = orc.Medium(grid, w.vel)
    nb = w.nb
    core = (slice(nb, nb + w.nz), 0, slice(nb, nb + w.nx))
    assert np.all(med.C1[core] == 1.0) and np.all(med.C2[core] == 1.0)
    np.testing.assert_allclose(med.W[core], (w.vel[:, 0, :] * w.dt) ** 2,
                               rtol=1e-15)
    # velocity edge-replicated into the padding
    np.testing.assert_allclose(med.W[0, 0, nb:nb + w.nx], med.W[nb, 0,
                                                              nb:nb + w.nx])
    # damping grows monotonically into the sponge, C2 < C1 < 1 there
    row = med.C1[nb + 3, 0, :nb]
    assert np.all(np.diff(row) > 0)
    sp = med.C1 < 1.0
    assert np.all(med.C2[sp] < med.C1[sp])
    assert np.all(med.C2 > 0)


# ---------------------------------------------------------------------------
# Ricker wavelet
# ---------------------------------------------------------------------------
def test_ricker_shape(orc):
    f0, dt = 20.0, 1e-4
    nt = 2000
    f = orc.ricker(nt, dt, f0)
    t0 = 1.5 / f0
    n0 = int(round(t0 / dt))
    assert abs(f[n0] - 1.0) < 1e-12 and np.argmax(f) == n0
    # zero crossings at t0 +- 1 / (pi f0 sqrt 2)
    tz = 1.0 / (np.pi * f0 * np.sqrt(2.0))
    t = np.arange(nt) * dt
    sgn = np.sign(f)
    cross = t[1:][np.nonzero(np.diff(sgn))[0]]
    assert np.min(np.abs(cross - (t0 - tz))) < dt
    assert np.min(np.abs(cross - (t0 + tz))) < dt
    # amplitude spectrum proportional to f^2 exp(-f^2/f0^2): peak at f0
    spec = np.abs(np.fft.rfft(f, 1 << 16))
    freqs = np.fft.rfftfreq(1 << 16, dt)
    assert abs(freqs[np.argmax(spec)] - f0) < 0.2
    model = freqs ** 2 * np.exp(-freqs ** 2 / f0 ** 2)
    sel = freqs < 4 * f0
    ratio = spec[sel][1:] / model[sel][1:]
    assert np.std(ratio) / np.mean(ratio) < 1e-3
    assert abs(f[0]) < 1e-7


# ---------------------------------------------------------------------------
# Background field against the analytic Green's functions
# ---------------------------------------------------------------------------
def _ricker_exact(t, f0):
    a = (np.pi * f0 * (t - 1.5 / f0)) ** 2
    return (1 - 2 * a) * np.exp(-a)


def test_direct_arrival_2d_matches_green_function(orc):
    """Homogeneous 2-D: u0 = h^2 (g * f), g = H(t - r/v) / (2 pi sqrt(t^2 -
    r^2/v^2)), the causal Green's function of the scalar wave equation."""
    v, h, dt, f0 = 2000.0, 10.0, 1e-3, 10.0
    n = 160
    nb = 20
    nt = 420
    grid = orc.Grid(2, n, 1, n, nb, h, dt)
    src = (n // 2, 0, n // 2)
    offs = [20, 30]
    rec = np.array([[n // 2, 0, n // 2 + o] for o in offs] +
                   [[n // 2 + 21, 0, n // 2 + 21]], dtype=np.int32)
    shot = orc.ShotGeom(src, rec, nt, f0)
    prob = orc.Problem(grid, np.full((n, 1, n), v), [shot])
    _, u = prob.background_shot(0)
    t = np.arange(nt) * dt
    for j, r in enumerate([offs[0] * h, offs[1] * h, 21 * np.sqrt(2) * h]):
        ana = np.zeros(nt)
        for k, tk in enumerate(t):
            if tk <= r / v:
                continue
            smax = np.arccosh(v * tk / r)
            s = np.linspace(0.0, smax, 4001)
            ana[k] = np.trapezoid(_ricker_exact(tk - (r / v) * np.cosh(s), f0), s)
        ana *= h * h / (2 * np.pi)
        rel = np.linalg.norm(u[:, j] - ana) / np.linalg.norm(ana)
        assert rel < 1e-2, (r, rel)
        assert abs(np.argmax(u[:, j]) - np.argmax(ana)) <= 1


def test_direct_arrival_3d_is_delayed_wavelet(orc):
    """Homogeneous 3-D: u0 = h^3 f(t - r/v) / (4 pi r)."""
    v, h, dt, f0 = 2000.0, 10.0, 1e-3, 10.0
    n = 56
    nb = 12
    nt = 300
    grid = orc.Grid(3, n, n, n, nb, h, dt)
    c = n // 2
    rec = np.array([[c, c, c + 16], [c + 12, c, c]], dtype=np.int32)
    shot = orc.ShotGeom((c, c, c), rec, nt, f0)
    prob = orc.Problem(grid, np.full((n, n, n), v), [shot])
    _, u = prob.background_shot(0)
    t = np.arange(nt) * dt
    for j, r in enumerate([16 * h, 12 * h]):
        ana = h ** 3 * _ricker_exact(t - r / v, f0) / (4 * np.pi * r)
        # the window stops before reflections from the sponge can arrive
        sel = t < 0.15 + r / v + 0.1
        rel = np.linalg.norm(u[sel, j] - ana[sel]) / np.linalg.norm(ana[sel])
        assert rel < 3e-2, (r, rel)
        assert abs(np.argmax(u[:, j]) - np.argmax(ana)) <= 1


def test_sponge_absorbs(orc):
    """After the wavelet has left a homogeneous model, the energy left on the
    model region is tiny compared with its peak (absorbing faces)."""
    v, h, dt, f0 = 2000.0, 10.0, 1e-3, 25.0
    n, nb, nt = 40, 20, 700
    grid = orc.Grid(2, n, 1, n, nb, h, dt)
    zz, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rec = np.stack([zz.ravel(), 0 * zz.ravel(), xx.ravel()], 1).astype(
        np.int32)
    shot = orc.ShotGeom((n // 2, 0, n // 2), rec, nt, f0)
    prob = orc.Problem(grid, np.full((n, 1, n), v), [shot])
    _, u = prob.background_shot(0)
    e = (u ** 2).sum(axis=1)
    assert e[-50:].max() < 1e-4 * e.max()


# ---------------------------------------------------------------------------
# Born operator: the derivative of the modelling with respect to squared
# slowness (W -> W / (1 + eps P m)).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ndim", [2, 3])
def test_born_is_derivative_of_modelling(orc, ndim):
    w = synth.tiny2d(nz=10, nx=14, nb=5, nt=100) if ndim == 2 else \
        synth.tiny3d(nt=60)
    prob = orc.Problem.from_workload(w)
    m = w.m_true
    eps = 1e-4
    nb = w.nb
    pm = np.zeros(prob.grid.padded_shape)
    if ndim == 2:
        pm[nb:nb + w.nz, 0, nb:nb + w.nx] = m[:, 0, :]
    else:
        pm[nb:nb + w.nz, nb:nb + w.ny, nb:nb + w.nx] = m
    for i in range(len(w.shots)):
        outs = []
        for sgn in (+1, -1):
            med = orc.Medium(prob.grid, w.vel)
            med.W = med.W / (1.0 + sgn * eps * pm)
            _, u = prob.background_shot(i, medium=med)
            outs.append(u)
        fd = (outs[0] - outs[1]) / (2 * eps)
        born = prob.born_shot(i, m)
        rel = np.linalg.norm(fd - born) / np.linalg.norm(born)
        assert rel < 1e-8, rel


# ---------------------------------------------------------------------------
# Adjoint: dot-product identity and brute-force transpose
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["layers64", "tiny3d"])
def test_dot_product_identity(orc, which):
    w = synth.layers2d_64x64() if which == "layers64" else synth.tiny3d()
    prob = orc.Problem.from_workload(w)
    idx = list(range(min(2, len(w.shots))))
    m = synth.gaussian(prob.grid.model_shape, 12)
    d = [synth.gaussian(prob.data_shape(i), 13 + i) for i in idx]
    lhs = orc._dot(prob.born(m, idx), d)
    rhs = float(np.vdot(m, prob.adjoint(d, idx)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _dense(orc, prob, idx):
    M = int(np.prod(prob.grid.model_shape))
    cols = []
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        cols.append(np.concatenate([x.ravel() for x in prob.born(e, idx)]))
    return np.stack(cols, axis=1)


def test_adjoint_is_exact_transpose_dense(orc):
    w = synth.tiny2d(nz=8, nx=9, nb=4, nt=50, nrec=5)
    prob = orc.Problem.from_workload(w)
    idx = [0, 1]
    A = _dense(orc, prob, idx)
    rows = []
    shapes = [prob.data_shape(i) for i in idx]
    sizes = [a * b for a, b in shapes]
    for k in range(sum(sizes)):
        e = np.zeros(sum(sizes))
        e[k] = 1.0
        parts = np.split(e, np.cumsum(sizes)[:-1])
        rows.append(prob.adjoint([p.reshape(s) for p, s in zip(parts, shapes)],
                                 idx).ravel())
    AT = np.stack(rows, axis=1)
    assert np.abs(A).max() > 0
    assert np.abs(A.T - AT).max() <= 1e-13 * np.abs(A).max()
    # the first data sample of every trace is identically zero (du^0 = 0)
    nt, nrec = shapes[0]
    assert np.all(A[:nrec] == 0.0)
