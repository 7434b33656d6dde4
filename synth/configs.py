"""Workload descriptions with the shapes, sizes and value distributions of the
method's use cases.

The paper's own example (Examples section) migrates the Marmousi data set
(240 shots, 25 m apart, 20 Hz Ricker, windows of 5 shots sliding by 3). That
model and data are not available here, so every workload below is synthetic
and seeded: a layered, faulted 2-D model whose velocity rises with depth
stands in for Marmousi.

Naming: ``Q`` is the number of shots in a window (the paper's window length)
and ``S`` is the number of shots added and dropped per slide (the paper's
rank of update and downdate).

Seeds: ``numpy.random.default_rng(1000 * c + k)`` with c the workload's seed
group and k = 0 reflectivity, 1 noise, 2 test vectors / finite-difference
directions, 3 faults and drift.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# seed groups of the workloads (first factor of the seeds)
SEED_LAYERS2D_64 = 0
SEED_FAULTED2D_512 = 1
SEED_LAYERED3D_256 = 3
SEED_STREAM2D_512 = 4
SEED_SSF2D_256 = 5
SEED_SSF_SMALL = 6


def rng(seed_group: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(1000 * seed_group + stream)


def gaussian(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


@dataclass
class Shot:
    id: int
    src: tuple  # (z, y, x) on the model grid (y = 0 in 2-D)
    rec: np.ndarray  # int32 [nrec, 3] (z, y, x) on the model grid
    nt: int
    f0: float

    @property
    def nrec(self) -> int:
        return int(self.rec.shape[0])


@dataclass
class Workload:
    name: str
    seed_group: int
    ndim: int
    nz: int
    ny: int
    nx: int
    nb: int
    h: float
    dt: float
    nt: int
    f0: float
    vel: np.ndarray  # float64 [nz, ny, nx], m/s
    m_true: np.ndarray  # float64 [nz, ny, nx]
    shots: List[Shot]
    Q: int
    S: int
    niter: int
    lam_rel: float
    noise_rel: float = 0.01
    extra: dict = field(default_factory=dict)

    @property
    def model_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def npoints_model(self) -> int:
        return self.nz * self.ny * self.nx

    @property
    def npoints_padded(self) -> int:
        py = self.ny + 2 * self.nb if self.ndim == 3 else 1
        return (self.nz + 2 * self.nb) * py * (self.nx + 2 * self.nb)

    def windows(self) -> List[List[int]]:
        """Shot indices of each window: window w holds [wS, wS + Q)."""
        out = []
        n = len(self.shots)
        if n <= self.Q:
            return [list(range(n))]
        w = 0
        while w * self.S + self.Q <= n:
            out.append(list(range(w * self.S, w * self.S + self.Q)))
            w += 1
        last = out[-1][-1]
        if last < n - 1:  # final shorter slide
            out.append(list(range(n - self.Q, n)))
        return out


def _row_receivers(z: int, xs, y: int = 0) -> np.ndarray:
    xs = np.asarray(list(xs), dtype=np.int32)
    out = np.zeros((xs.size, 3), dtype=np.int32)
    out[:, 0] = z
    out[:, 1] = y
    out[:, 2] = xs
    return out


def layers2d_64x64() -> Workload:
    """2-D, 64 x 64, h = 10 m, constant 2000 m/s, three flat reflectors."""
    nz = nx = 64
    r = rng(SEED_LAYERS2D_64, 0)
    amps = r.uniform(-0.1, 0.1, size=3)
    m = np.zeros((nz, 1, nx))
    for a, z in zip(amps, (20, 35, 50)):
        m[z, 0, :] = a
    vel = np.full((nz, 1, nx), 2000.0)
    rec = _row_receivers(2, range(64))
    shots = [Shot(i, (2, 0, x), rec.copy(), 500, 15.0)
             for i, x in enumerate((8, 24, 40, 56))]
    return Workload("layers2d-64x64", SEED_LAYERS2D_64, 2, nz, 1, nx, 20,
                    10.0, 1e-3, 500,
                    15.0, vel, m, shots, Q=2, S=1, niter=10, lam_rel=0.01)


def faulted_blocks(nz: int, nx: int, r_layers, r_faults,
                   nlayers: int = 40, nfaults: int = 10) -> np.ndarray:
    """A random layered model cut by dipping faults: piecewise-constant
    values in [-1, 1]."""
    xc = (nx - 1) / 2.0
    depths = np.sort(r_layers.uniform(16, nz - 12, size=nlayers))
    dips = r_layers.uniform(-0.05, 0.05, size=nlayers)
    values = r_layers.uniform(-1.0, 1.0, size=nlayers + 1)
    faults = []
    for _ in range(nfaults):
        x0 = r_faults.uniform(100, nx - 100) if nx > 240 else r_faults.uniform(
            0.2 * nx, 0.8 * nx)
        ang = np.deg2rad(r_faults.uniform(60.0, 80.0))
        throw = r_faults.uniform(4, 16)
        side = 1.0 if r_faults.uniform() < 0.5 else -1.0
        faults.append((x0, side / np.tan(ang), throw))
    z = np.arange(nz, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    zeff = np.broadcast_to(z, (nz, nx)).copy()
    for x0, slope, throw in faults:
        hanging = x > x0 + slope * z  # right of the fault plane
        zeff = np.where(hanging, zeff - throw, zeff)
    # layer index below each interface
    b = np.full((nz, nx), values[0])
    for i in range(nlayers):
        iface = depths[i] + dips[i] * (x - xc)
        b = np.where(zeff >= iface, values[i + 1], b)
    return b


def faulted_reflectivity(nz: int, nx: int, r_layers, r_faults,
                         nlayers: int = 40, nfaults: int = 10) -> np.ndarray:
    """Vertical derivative of a random layered model cut by dipping faults,
    scaled to max |m| = 0.1."""
    b = faulted_blocks(nz, nx, r_layers, r_faults, nlayers, nfaults)
    m = np.zeros((nz, nx))
    m[:-1] = b[1:] - b[:-1]
    mx = np.abs(m).max()
    if mx > 0:
        m *= 0.1 / mx
    return m


def faulted2d_512x1024(nz: int = 512, nx: int = 1024, nshots: int = 64,
                       nt: int = 3000) -> Workload:
    """2-D, 512 x 1024, h = 5 m, v(z) 1500 -> 4000 m/s with a -300 m/s
    Gaussian anomaly (sigma 200 m), faulted layered reflectivity, 64 shots
    80 m apart, 1024 receivers, nt = 3000, dt = 0.5 ms, 20 Hz."""
    h = 5.0
    z = np.arange(nz, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    zc, xc = 1280.0 * nz / 512.0, 2560.0 * nx / 1024.0
    sig = 200.0
    vel = 1500.0 + 2500.0 * z / (nz - 1) - 300.0 * np.exp(
        -(((z * h - zc) ** 2 + (x * h - xc) ** 2) / (2 * sig * sig)))
    m = faulted_reflectivity(nz, nx, rng(SEED_FAULTED2D_512, 0),
                             rng(SEED_FAULTED2D_512, 3))
    rec = _row_receivers(2, range(nx))
    spacing = 16
    shots = [Shot(i, (2, 0, 8 + spacing * i), rec.copy(), nt, 20.0)
             for i in range(nshots) if 8 + spacing * i < nx]
    return Workload("faulted2d-512x1024", SEED_FAULTED2D_512, 2, nz, 1, nx,
                    40, h, 0.5e-3, nt, 20.0,
                    vel[:, None, :].copy(), m[:, None, :].copy(), shots, Q=8,
                    S=4, niter=20, lam_rel=1e-3)


def layered3d_256x320x320(nz: int = 256, ny: int = 320, nx: int = 320,
                          nt: int = 2000, nrec_side: int = 128) -> Workload:
    """3-D, 256 x 320 x 320, h = 10 m, v(z) 1500 -> 3500 m/s, random layered
    reflectivity, 32 shots on an 8 x 4 grid, 128 x 128 receivers,
    nt = 2000, dt = 1 ms, 12 Hz."""
    h = 10.0
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    vel = np.broadcast_to(1500.0 + 2000.0 * z / (nz - 1), (nz, ny, nx)).copy()
    r = rng(SEED_LAYERED3D_256, 0)
    nl = 30
    depths = r.uniform(10, nz - 6, size=nl)
    dx = r.uniform(-0.03, 0.03, size=nl)
    dy = r.uniform(-0.03, 0.03, size=nl)
    amps = r.uniform(-0.1, 0.1, size=nl)
    m = np.zeros((nz, ny, nx))
    yy, xx = np.meshgrid(np.arange(ny) - (ny - 1) / 2.0,
                         np.arange(nx) - (nx - 1) / 2.0, indexing="ij")
    for i in range(nl):
        zi = np.rint(depths[i] + dx[i] * xx + dy[i] * yy).astype(int)
        ok = (zi >= 0) & (zi < nz)
        iy, ix = np.nonzero(ok)
        m[zi[ok], iy, ix] += amps[i]
    step = max(1, min((nx - 4) // nrec_side, (ny - 4) // nrec_side))
    off_x = (nx - step * (nrec_side - 1)) // 2
    off_y = (ny - step * (nrec_side - 1)) // 2
    ry, rx = np.meshgrid(off_y + step * np.arange(nrec_side),
                         off_x + step * np.arange(nrec_side), indexing="ij")
    rec = np.stack([np.full(rx.size, 2), ry.ravel(), rx.ravel()],
                   axis=1).astype(np.int32)
    sxs = [int(round((i + 0.5) * nx / 8)) for i in range(8)]
    sys_ = [int(round((j + 0.5) * ny / 4)) for j in range(4)]
    shots = []
    for j, sy in enumerate(sys_):
        for i, sx in enumerate(sxs):
            shots.append(Shot(len(shots), (2, sy, sx), rec.copy(), nt, 12.0))
    return Workload("layered3d-256x320x320", SEED_LAYERED3D_256, 3, nz, ny,
                    nx, 20, h, 1e-3, nt, 12.0,
                    vel, m, shots, Q=8, S=4, niter=20, lam_rel=1e-3)


def tiny2d(nz: int = 12, nx: int = 12, nb: int = 6, nt: int = 120,
           nshots: int = 2, nrec: int = 12, seed: int = 7,
           velocity: str = "gradient") -> Workload:
    """Small 2-D problem for dense-matrix checks and parity at a few tiles."""
    r = np.random.default_rng(seed)
    z = np.arange(nz, dtype=np.float64)[:, None]
    if velocity == "constant":
        vel = np.full((nz, nx), 2000.0)
    else:
        vel = 1800.0 + 600.0 * z / max(nz - 1, 1) + 100.0 * r.uniform(
            -1, 1, size=(nz, nx))
    m = r.uniform(-0.1, 0.1, size=(nz, nx))
    xs = np.linspace(1, nx - 2, nrec).round().astype(int)
    rec = _row_receivers(min(2, nz - 1), xs)
    sx = np.linspace(2, nx - 3, nshots).round().astype(int)
    shots = [Shot(i, (min(2, nz - 1), 0, int(x)), rec.copy(), nt, 25.0)
             for i, x in enumerate(sx)]
    return Workload("tiny2d", -1, 2, nz, 1, nx, nb, 10.0, 1e-3, nt, 25.0,
                    vel[:, None, :].copy(), m[:, None, :].copy(), shots,
                    Q=nshots, S=1, niter=10, lam_rel=0.01)


def tiny3d(nz: int = 8, ny: int = 8, nx: int = 8, nb: int = 4, nt: int = 80,
           nshots: int = 2, seed: int = 11) -> Workload:
    r = np.random.default_rng(seed)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    vel = np.broadcast_to(1800.0 + 500.0 * z / (nz - 1),
                          (nz, ny, nx)) + 80.0 * r.uniform(-1, 1,
                                                           (nz, ny, nx))
    m = r.uniform(-0.1, 0.1, size=(nz, ny, nx))
    ry, rx = np.meshgrid(np.arange(1, ny - 1, 2), np.arange(1, nx - 1, 2),
                         indexing="ij")
    rec = np.stack([np.full(rx.size, 1), ry.ravel(), rx.ravel()],
                   axis=1).astype(np.int32)
    shots = [Shot(i, (1, 2 + 3 * i % (ny - 2), 2 + 2 * i % (nx - 2)),
                  rec.copy(), nt, 30.0) for i in range(nshots)]
    return Workload("tiny3d", -1, 3, nz, ny, nx, nb, 10.0, 1e-3, nt, 30.0,
                    np.ascontiguousarray(vel), m, shots, Q=nshots, S=1,
                    niter=10, lam_rel=0.01)


def _smooth(a: np.ndarray, half: int) -> np.ndarray:
    """Moving average over 2 * half + 1 cells along each axis (edges
    replicated), applied twice."""
    out = a
    for _ in range(2):
        for ax in range(out.ndim):
            if out.shape[ax] == 1:
                continue
            pad = [(0, 0)] * out.ndim
            pad[ax] = (half, half)
            c = np.cumsum(np.pad(out, pad, mode="edge"), axis=ax)
            c = np.insert(c, 0, 0.0, axis=ax)
            n = out.shape[ax]
            hi = np.take(c, np.arange(2 * half + 1, 2 * half + 1 + n), axis=ax)
            lo = np.take(c, np.arange(0, n), axis=ax)
            out = (hi - lo) / (2 * half + 1)
    return out


def streaming(base: Workload, nshots: int, Q: int, apertures, nts,
              seed_group: int, positions=None, niter: int = 5,
              drift_per_64: float = 1e-3) -> Workload:
    """A stream of shots over `base`'s model: shot i sits at position
    i mod len(positions) (default: base's shot positions, in sweeps), with
    a contiguous receiver aperture of n_r ~ U{apertures} cells centred on
    the source (clipped to the model) on base's receiver row, and nt drawn
    from `nts`. The reflectivity drifts: shot i sees
        m_i = m_0 + (i / 64) * drift,  ||drift|| = drift_per_64 ||m_0||,
    with drift a seeded Gaussian field smoothed over 4 cells (base.extra
    keeps m_0 in m_true; `drift` goes to extra). Windows of Q shots slide
    by Q / 2."""
    r = rng(seed_group, 3)
    nx = base.nx
    zr = int(base.shots[0].rec[0, 0])
    pos = positions if positions is not None else [s.src for s in base.shots]
    lo_a, hi_a = apertures
    shots = []
    for i in range(nshots):
        src = pos[i % len(pos)]
        nr = int(min(r.integers(lo_a, hi_a + 1), nx))
        x0 = int(np.clip(src[2] - nr // 2, 0, nx - nr))
        rec = _row_receivers(zr, range(x0, x0 + nr))
        nt = int(r.choice(nts))
        shots.append(Shot(i, tuple(src), rec, nt, base.f0))
    d = _smooth(r.standard_normal(base.model_shape), 4)
    d *= drift_per_64 * np.linalg.norm(base.m_true) / np.linalg.norm(d)
    extra = dict(base.extra)
    extra["drift"] = d
    return Workload(base.name + "-stream", seed_group, base.ndim, base.nz,
                    base.ny, base.nx, base.nb, base.h, base.dt,
                    max(s.nt for s in shots), base.f0, base.vel, base.m_true,
                    shots, Q=Q, S=max(1, Q // 2), niter=niter,
                    lam_rel=base.lam_rel, extra=extra)


def stream2d_512x1024(nshots: int = 512, Q: int = 8) -> Workload:
    """Streaming form of the faulted 512 x 1024 workload: `nshots` shots in
    sweeps of its 64 positions, apertures U{256..1024} receivers, nt in
    {2000, 3000, 4000}, reflectivity drifting 0.1 % per 64 shots."""
    return streaming(faulted2d_512x1024(), nshots, Q, (256, 1024),
                     (2000, 3000, 4000), SEED_STREAM2D_512)


def model_at(w: Workload, i: int) -> np.ndarray:
    """The reflectivity shot i sees (streaming workloads drift)."""
    d = w.extra.get("drift")
    return w.m_true if d is None else w.m_true + (i / 64.0) * d


def noise_like(shape, seed_group: int) -> np.ndarray:
    return rng(seed_group, 1).standard_normal(shape)


def unit_random_like(shape, seed: int, norm: Optional[float] = None):
    v = gaussian(shape, seed)
    if norm is not None:
        v *= norm / np.linalg.norm(v)
    return v


# ---------------------------------------------------------------------------
# Split-step Fourier (shot-profile, one-way) workloads: 2-D models whose
# lateral size is a power of two (the lateral FFT length, taper included),
# sources and receivers on the top level.
# ---------------------------------------------------------------------------
@dataclass
class SsfShot:
    id: int
    xs: int          # source column
    rec: np.ndarray  # int32 [nrec] receiver columns
    f0: float

    @property
    def nrec(self) -> int:
        return int(self.rec.size)


@dataclass
class SsfWorkload:
    name: str
    seed_group: int
    nz: int
    nx: int
    dx: float
    dz: float
    nt: int
    dt: float
    fmin: float
    fmax: float
    ntap: int
    vel: np.ndarray     # float64 [nz, nx], m/s (the migration velocity)
    m_true: np.ndarray  # float64 [nz, nx]
    shots: List[SsfShot]
    Q: int
    S: int
    niter: int
    lam_rel: float
    noise_rel: float = 0.01
    extra: dict = field(default_factory=dict)

    @property
    def model_shape(self):
        return (self.nz, self.nx)

    windows = Workload.windows


def _smooth2(a: np.ndarray, half: int) -> np.ndarray:
    """Box average over (2 half + 1)^2 cells, edges replicated."""
    p = np.pad(a, half, mode="edge")
    c = np.cumsum(np.cumsum(p, 0), 1)
    c = np.pad(c, ((1, 0), (1, 0)))
    k = 2 * half + 1
    return (c[k:, k:] - c[:-k, k:] - c[k:, :-k] + c[:-k, :-k]) / (k * k)


def ssf_small(nz: int = 24, nx: int = 64, nt: int = 256, dt: float = 4e-3,
              fmin: float = 4.0, fmax: float = 40.0, ntap: int = 8,
              seed: int = 0) -> SsfWorkload:
    """Small split-step case for parity: v rising with depth plus a lateral
    sine and seeded noise, a random reflectivity, three shots with
    different receiver sets (a dense split spread, a scattered set with both
    edge columns and a repeated column, an off-end spread to the left)."""
    r = rng(SEED_SSF_SMALL, seed)
    z = np.arange(nz, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    vel = 1700.0 + 1200.0 * z / max(nz - 1, 1) + 180.0 * np.sin(
        2 * np.pi * x / nx + 2.0 * z / max(nz, 1))
    vel += 40.0 * r.standard_normal((nz, nx))
    m = 0.1 * r.standard_normal((nz, nx))
    xs = [nx // 3, nx // 2 + 1, (5 * nx) // 6]
    recs = [np.arange(nx // 8, nx - nx // 16, 2),
            np.array([0, 5, 5, nx // 4 + 1, nx - 1, (5 * nx) // 8]),
            np.array([xs[2] - 4 - 2 * k for k in range(12)])]
    shots = [SsfShot(i, xs[i], recs[i].astype(np.int32), 15.0)
             for i in range(3)]
    return SsfWorkload("ssf-small-%dx%d" % (nz, nx), SEED_SSF_SMALL, nz, nx,
                       10.0, 10.0, nt, dt, fmin, fmax, ntap, vel, m, shots,
                       Q=2, S=1, niter=5, lam_rel=1e-2)


def ssf2d_256x1024(nshots: int = 240) -> SsfWorkload:
    """Stand-in for the paper's Marmousi example (Examples section): 2-D,
    256 x 1024 at 12.5 m (3.2 x 12.8 km, 32-cell tapers at the sides), a
    200 m water layer over a faulted layered velocity 1500 -> 4500 m/s
    (smoothed over 9 cells: the migration velocity), faulted layered
    reflectivity (extra: the true velocity, and the high-passed squared-
    slowness perturbation it carries against the migration velocity); 240
    shots 25 m apart (the paper's count and spacing), each with 96
    receivers 25 m apart on an
    off-end spread to the left of the source (near offset 100 m), 20 Hz
    Ricker, 4096 samples at 1 ms, band 3-40 Hz (151 frequencies); windows of
    5 shots sliding by 3, 8 CG iterations (the paper's configuration)."""
    nz, nx, h = 256, 1024, 12.5
    b = faulted_blocks(nz, nx, rng(SEED_SSF2D_256, 0), rng(SEED_SSF2D_256, 3))
    z = np.arange(nz, dtype=np.float64)[:, None]
    vtrue = 1500.0 + 2600.0 * (z / (nz - 1)) ** 0.8 + 400.0 * b * (
        0.3 + 0.7 * z / (nz - 1))
    vtrue[:16] = 1500.0  # water layer (200 m), as on top of Marmousi
    vel = _smooth2(vtrue, 4)
    m = faulted_reflectivity(nz, nx, rng(SEED_SSF2D_256, 0),
                             rng(SEED_SSF2D_256, 3))
    shots = []
    for i in range(nshots):
        xs = 300 + 2 * i
        rec = np.array([xs - 8 - 2 * k for k in range(96)], dtype=np.int32)
        shots.append(SsfShot(i, xs, rec, 20.0))
    # the perturbation nonlinear data of vtrue carry against the migration
    # velocity: relative squared slowness, minus its 9-cell average
    pert = (vel / vtrue) ** 2 - 1.0
    return SsfWorkload("ssf2d-256x1024", SEED_SSF2D_256, nz, nx, h, h, 4096,
                       1e-3, 3.0, 40.0, 32, vel, m, shots, Q=5, S=3, niter=8,
                       lam_rel=1e-3,
                       extra={"vel_true": vtrue,
                              "m_nonlinear": pert - _smooth2(pert, 4)})
