"""Pins of the FP64 split-step Fourier oracle (shot-profile de-migration and
migration, the operator family of the paper's examples) against closed
forms, library routines, physics and invariants."""
import numpy as np
import pytest

from oracle import ricker
from oracle.ssf import SsfProblem, SsfShot, band, dft, taper


def _problem(vel, dx=10.0, dz=10.0, nt=512, dt=2e-3, fmin=5.0, fmax=50.0,
             ntap=16, shots=()):
    return SsfProblem(np.asarray(vel, dtype=np.float64), dx, dz, nt, dt,
                      fmin, fmax, ntap, list(shots))


def _layered(nz, nx, seed=0):
    """Velocity increasing with depth plus a smooth lateral perturbation."""
    z = np.arange(nz)[:, None]
    x = np.arange(nx)[None, :]
    v = 1800.0 + 12.0 * z + 150.0 * np.sin(2 * np.pi * x / nx + 0.3 * z / nz)
    v += 60.0 * np.random.default_rng(seed).standard_normal((nz, nx))
    return v


# --- frequency band and DFT -----------------------------------------------
def test_band_is_the_dft_grid_within_the_limits():
    df, k0, nw = band(512, 2e-3, 5.0, 50.0)
    assert df == pytest.approx(1.0 / 1.024)
    f = (k0 + np.arange(nw)) * df
    assert f[0] >= 5.0 and f[0] - df < 5.0
    assert f[-1] <= 50.0 and f[-1] + df > 50.0
    with pytest.raises(ValueError):
        band(512, 2e-3, 5.2, 5.3)


def test_dft_matches_the_fft_library():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((256, 5))
    dt = 4e-3
    df, k0, nw = band(256, dt, 3.0, 60.0)
    om = 2 * np.pi * (k0 + np.arange(nw)) * df
    want = dt * np.fft.rfft(x, axis=0)[k0:k0 + nw]
    assert np.max(np.abs(dft(x, dt, om) - want)) <= 1e-12 * np.max(
        np.abs(want))


def test_wavelet_spectrum_is_the_continuous_ricker_transform():
    """The DFT of the sampled Ricker approximates its Fourier transform
    (2/sqrt(pi)) f^2/f0^3 exp(-f^2/f0^2) exp(-i 2 pi f t0) to the level of
    the truncated tails (the wavelet is 2e-10 of its peak at t = 0)."""
    f0 = 20.0
    p = _problem(np.full((4, 64), 2000.0), nt=1024, dt=1e-3, fmin=2.0,
                 fmax=80.0)
    F = p.wavelet(f0)
    f = p.omegas / (2 * np.pi)
    want = (2 / np.sqrt(np.pi)) * f ** 2 / f0 ** 3 * np.exp(
        -(f / f0) ** 2) * np.exp(-2j * np.pi * f * 1.5 / f0)
    assert np.max(np.abs(F - want)) <= 1e-7 * np.max(np.abs(want))


# --- one depth step ---------------------------------------------------------
@pytest.mark.parametrize("q", [3, 40, 70])
def test_constant_velocity_step_is_the_exact_phase_shift(q):
    """A plane wave exp(i kx x) in a constant medium (no taper) after n steps
    is exp(-i kz n dz) exp(i kx x): kz real (propagating, q = 3, 40 at the
    highest frequencies) or imaginary (evanescent decay, q = 70)."""
    nx, nz, dx, dz, v = 128, 12, 10.0, 10.0, 2000.0
    p = _problem(np.full((nz, nx), v), dx=dx, dz=dz, ntap=0)
    kx = 2 * np.pi * q / (nx * dx)
    x = np.arange(nx) * dx
    u0 = np.exp(1j * kx * x)[None, :].repeat(p.nw, 0)
    u = u0
    for j in range(nz):
        u = p.step(u, j)
    a = (p.omegas / v) ** 2 - kx ** 2
    kz = np.sqrt(np.abs(a))
    fac = np.where(a >= 0, np.exp(-1j * kz * nz * dz), np.exp(-kz * nz * dz))
    assert np.max(np.abs(u - fac[:, None] * u0)) <= 1e-12
    if q == 70:
        assert np.all(a < 0)
    elif q == 3:
        assert np.all(a > 0)


def test_vertical_traveltime_through_a_layered_medium():
    """A vertical plane wave in v(z) picks up the vertical traveltime
    sum_j dz / v_j as phase exp(-i w t)."""
    nz, nx, dz = 30, 64, 8.0
    vz = 1500.0 + 40.0 * np.arange(nz)
    p = _problem(np.repeat(vz[:, None], nx, 1), dz=dz, ntap=0)
    u = np.ones((p.nw, nx), dtype=complex)
    for j in range(nz):
        u = p.step(u, j)
    t = np.sum(dz / vz)
    assert np.max(np.abs(u - np.exp(-1j * p.omegas * t)[:, None])) <= 1e-12


def test_one_step_of_a_flat_field_is_the_local_vertical_traveltime():
    """With lateral variation, a laterally constant field after one step is
    tau(x) exp(-i w s(x) dz): the phase shift moves it by s0 dz, the split
    step adds (s - s0) dz."""
    nz, nx, dz = 3, 64, 10.0
    v = _layered(nz, nx)
    p = _problem(v, dz=dz, ntap=8)
    u = p.step(np.ones((p.nw, nx), dtype=complex), 1)
    want = p.tau * np.exp(-1j * np.outer(p.omegas, dz / v[1]))
    assert np.max(np.abs(u - want)) <= 1e-12


def test_taper_shape():
    t = taper(64, 8)
    assert np.all(t[8:56] == 1.0)
    assert np.all(np.diff(t[:9]) > 0) and np.allclose(t, t[::-1])
    assert 0 < t[0] < 0.05


def test_step_adjoint_and_contraction():
    """<E u, w> = <u, E^H w> for complex vectors, and ||E u|| <= ||u|| (unit
    phase factors, evanescent decay and a taper at most 1)."""
    nz, nx = 4, 64
    p = _problem(_layered(nz, nx, 1), ntap=8)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((p.nw, nx)) + 1j * rng.standard_normal(
        (p.nw, nx))
    w = rng.standard_normal((p.nw, nx)) + 1j * rng.standard_normal(
        (p.nw, nx))
    for j in range(nz):
        lhs = np.vdot(p.step(u, j), w)
        rhs = np.vdot(u, p.step_adj(w, j))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        assert np.all(np.linalg.norm(p.step(u, j), axis=1)
                      <= np.linalg.norm(u, axis=1) * (1 + 1e-14))


# --- the operator pair ---------------------------------------------------------
def _shots(nx, n=2):
    rec = np.arange(8, nx - 8, 3)
    return [SsfShot(xs=nx // 3 + 7 * i, rec=rec, f0=18.0) for i in range(n)]


def test_dot_product_identity():
    nz, nx = 20, 64
    p = _problem(_layered(nz, nx, 2), nt=256, dt=4e-3, fmin=4.0, fmax=40.0,
                 ntap=8, shots=_shots(nx))
    rng = np.random.default_rng(11)
    m = rng.standard_normal((nz, nx))
    d = [rng.standard_normal((p.nw, len(s.rec), 2)) for s in p.shots]
    Am = p.born(m, [0, 1])
    lhs = sum(float(np.sum(a * b)) for a, b in zip(Am, d))
    rhs = float(np.sum(m * p.adjoint(d, [0, 1])))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dense_adjoint_is_the_transpose():
    """Tiny case: A built column by column from unit images, A^T from unit
    data vectors; A^T equals the transpose of A entrywise."""
    nz, nx = 5, 8
    rec = np.array([1, 3, 3, 6])   # a repeated receiver column too
    p = _problem(_layered(nz, nx, 3), dx=12.0, dz=12.0, nt=32, dt=8e-3,
                 fmin=10.0, fmax=30.0, ntap=2,
                 shots=[SsfShot(xs=4, rec=rec, f0=15.0)])
    W = p.weights(0)
    M = nz * nx
    ND = p.nw * len(rec) * 2
    A = np.zeros((ND, M))
    for k in range(M):
        e = np.zeros(M)
        e[k] = 1.0
        D = p.born_shot(0, e.reshape(nz, nx), W)
        A[:, k] = np.stack([D.real, D.imag], -1).ravel()
    AT = np.zeros((M, ND))
    for k in range(ND):
        e = np.zeros(ND)
        e[k] = 1.0
        e = e.reshape(p.nw, len(rec), 2)
        AT[:, k] = p.adjoint_shot(0, e[..., 0] + 1j * e[..., 1], W).ravel()
    assert np.max(np.abs(AT - A.T)) <= 1e-13 * np.max(np.abs(A))


def test_reciprocity_in_a_laterally_invariant_medium():
    """With v = v(z) and no taper the phase-shift kernel is symmetric, so
    swapping source and receiver columns leaves the scattered data of any
    image unchanged."""
    nz, nx = 16, 64
    vz = 1700.0 + 30.0 * np.arange(nz)
    p = _problem(np.repeat(vz[:, None], nx, 1), ntap=0,
                 shots=[SsfShot(20, np.array([45]), 15.0),
                        SsfShot(45, np.array([20]), 15.0)])
    m = np.random.default_rng(5).standard_normal((nz, nx))
    a = p.born_shot(0, m)
    b = p.born_shot(1, m)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def _point_scatterer_case(xd):
    nz, nx, v = 40, 128, 2000.0
    rec = np.arange(16, 112)
    p = _problem(np.full((nz, nx), v), nt=512, dt=2e-3, fmin=5.0, fmax=50.0,
                 ntap=16, shots=[SsfShot(64, rec, 20.0)])
    m = np.zeros((nz, nx))
    m[30, xd] = 1.0
    return p, m, rec


def test_point_scatterer_traveltime():
    """Constant v = 2000 m/s, scatterer 300 m below the source: the envelope
    of the trace at the source column peaks at t0 + 2 z / v = 0.375 s
    (within two samples)."""
    p, m, rec = _point_scatterer_case(64)
    D = p.born_shot(0, m)[:, list(rec).index(64)]
    t = np.arange(p.nt) * p.dt
    analytic = (2 * p.df) * np.exp(1j * np.outer(t, p.omegas)) @ D
    t_peak = t[np.argmax(np.abs(analytic))]
    assert abs(t_peak - (1.5 / 20.0 + 2 * 300.0 / 2000.0)) <= 2 * p.dt


def test_migration_focuses_at_the_scatterer():
    """The migrated image of a point scatterer's data peaks at the
    scatterer (off the source column, to check lateral positioning)."""
    p, m, _ = _point_scatterer_case(80)
    img = p.adjoint([np.stack([x.real, x.imag], -1) for x in
                     [p.born_shot(0, m)]], [0])
    jz, jx = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    assert abs(jz - 30) <= 1 and abs(jx - 80) <= 1


def test_observed_data_are_the_band_dft():
    nz, nx = 4, 64
    p = _problem(np.full((nz, nx), 2000.0), nt=256, dt=4e-3, fmin=4.0,
                 fmax=40.0, ntap=4, shots=_shots(nx, 1))
    d = np.random.default_rng(9).standard_normal((256, len(p.shots[0].rec)))
    got = p.observed(d)
    want = 4e-3 * np.fft.rfft(d, axis=0)[p.k0:p.k0 + p.nw]
    assert np.max(np.abs(got[..., 0] + 1j * got[..., 1] - want)) <= \
        1e-12 * np.max(np.abs(want))


def test_ricker_is_the_oracle_wavelet():
    """The split-step source uses the same Ricker samples as the
    finite-difference operator (peak 1 at 1.5 / f0)."""
    w = ricker(400, 1e-3, 20.0)
    assert np.argmax(w) == 75 and w[75] == pytest.approx(1.0)


def test_born_weight_is_the_split_step_phase_derivative():
    """W_j = c_j S_j with c_j the first-order change of one depth step when
    the squared slowness of level j becomes s^2 (1 + eps m): measured by
    central differences of the step of a perturbed medium (m with zero
    lateral mean of s m, so the reference slowness moves at second order
    only, which the central difference cancels)."""
    nz, nx, j = 3, 64, 1
    v = _layered(nz, nx, 4)
    shot = SsfShot(xs=21, rec=np.arange(4, 60, 5), f0=18.0)
    p = _problem(v, ntap=8, shots=[shot])
    rng = np.random.default_rng(12)
    m = 1.0 + rng.random(nx)
    m -= np.sum(p.s[j] * m) / np.sum(p.s[j])
    eps = 1e-5

    def step_of(sign):
        vv = v.copy()
        vv[j] = v[j] / np.sqrt(1.0 + sign * eps * m)
        return _problem(vv, ntap=8).step(
            np.ones((p.nw, nx), dtype=complex), j)

    u = p.step(np.ones((p.nw, nx), dtype=complex), j)
    c = (step_of(1) - step_of(-1)) / (2 * eps) / (m * u)
    S0 = np.zeros((p.nw, nx), dtype=complex)
    S0[:, shot.xs] = p.wavelet(shot.f0) * (-0.5j / (p.omegas * p.s[0, shot.xs]))
    S1 = p.step(S0, 0)
    W = p.weights(0)
    assert np.max(np.abs(W[j] - c * S1)) <= 1e-8 * np.max(np.abs(W[j]))


def test_split_step_times_have_zero_row_mean():
    """The reference slowness of each level is the row mean, so the split
    step carries only the lateral deviation."""
    p = _problem(_layered(6, 64, 5), ntap=8)
    assert np.max(np.abs(p.theta.mean(axis=1))) <= 1e-18
    assert np.all(p.s0 > p.s.min(axis=1)) and np.all(p.s0 < p.s.max(axis=1))


def test_window_cg_on_split_step_data_reaches_the_closed_form():
    """The window solver runs unchanged on the (re, im) data pairs: on a
    tiny two-shot window it converges to (A^T A + lam I)^{-1} A^T d built
    from the dense operator."""
    import oracle
    nz, nx = 4, 8
    shots = [SsfShot(xs=2, rec=np.array([0, 3, 5]), f0=15.0),
             SsfShot(xs=5, rec=np.array([1, 6]), f0=15.0)]
    p = _problem(_layered(nz, nx, 6), dx=12.0, dz=12.0, nt=32, dt=8e-3,
                 fmin=10.0, fmax=30.0, ntap=2, shots=shots)
    M = nz * nx
    cols = []
    for k in range(M):
        e = np.zeros(M)
        e[k] = 1.0
        cols.append(np.concatenate([x.ravel() for x in
                                    p.born(e.reshape(nz, nx), [0, 1])]))
    A = np.array(cols).T
    rng = np.random.default_rng(13)
    d = [rng.standard_normal((p.nw, len(s.rec), 2)) for s in shots]
    dv = np.concatenate([x.ravel() for x in d])
    lam = 1e-2 * np.linalg.norm(A.T @ A, 2)
    want = np.linalg.solve(A.T @ A + lam * np.eye(M), A.T @ dv)
    got = oracle.cgls(p, [0, 1], d, lam, 200, rtol=1e-13).m
    assert np.linalg.norm(got.ravel() - want) <= 1e-9 * np.linalg.norm(want)


def test_source_field_is_the_2d_greens_function_below_the_source():
    """Constant velocity, a wide taper against the periodic images: the
    source field straight below the source equals
    dx F(w) (-i/4) H0^(2)(w r / v), the outgoing 2-D Helmholtz Green's
    function (time as exp(+i w t)), to 2 % in amplitude and 0.03 rad in
    phase from 10 wavelengths down, the gap shrinking with distance (the
    one-way field is the far-field, vertical-incidence form)."""
    from scipy.special import hankel2
    nz, nx, dx, v = 200, 2048, 5.0, 2000.0
    p = _problem(np.full((nz, nx), v), dx=dx, dz=dx, nt=512, dt=2e-3,
                 fmin=20.0, fmax=40.0, ntap=400,
                 shots=[SsfShot(xs=nx // 2, rec=np.array([0]), f0=25.0)])
    W = p.weights(0)
    j = np.arange(1, nz)
    S = W[j, :, nx // 2] / (-0.5j * p.dz * p.omegas[None, :] / v)
    F = p.wavelet(25.0)
    k = p.omegas / v
    G = dx * F[None, :] * (-0.25j) * hankel2(0, np.outer(j * p.dz, k))
    ratio = S / G
    wl = (2 * np.pi / k)[None, :]
    far = (j * p.dz)[:, None] >= 10 * wl
    farther = (j * p.dz)[:, None] >= 15 * wl
    assert far.sum() > 1000 and farther.sum() > 200
    amp = np.abs(np.abs(ratio) - 1)
    ph = np.abs(np.angle(ratio))
    assert np.max(amp[far]) <= 0.02 and np.max(ph[far]) <= 0.03
    assert np.max(amp[farther]) < np.max(amp[far])
    assert np.max(ph[farther]) < np.max(ph[far])


def test_illumination_is_the_hessian_diagonal_on_one_level():
    """One level, every column a receiver: A is diagonal per frequency, so
    A^T A is diagonal and its diagonal is the illumination (brute force
    over unit images); two shots sum."""
    nx = 16
    shots = [SsfShot(xs=5, rec=np.arange(nx), f0=15.0),
             SsfShot(xs=11, rec=np.arange(nx), f0=15.0)]
    p = _problem(_layered(1, nx, 7), dx=12.0, dz=12.0, nt=64, dt=4e-3,
                 fmin=5.0, fmax=40.0, ntap=2, shots=shots)
    H = np.zeros((nx, nx))
    for k in range(nx):
        e = np.zeros((1, nx))
        e[0, k] = 1.0
        H[:, k] = p.adjoint(p.born(e, [0, 1]), [0, 1]).ravel()
    assert np.max(np.abs(H - np.diag(np.diag(H)))) <= 1e-14 * np.max(H)
    assert np.max(np.abs(np.diag(H) - p.illumination([0, 1]).ravel())) \
        <= 1e-13 * np.max(H)
