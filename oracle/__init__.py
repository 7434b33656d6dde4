"""FP64 CPU oracle for block-row recursive least-squares migration.

TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct reference the
GPU library is checked against. Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it. It shares no code
with the GPU library.

What it computes (Kazemi & Sacchi, arXiv 1801.00819):
  * ``born`` / ``adjoint``: the de-migration operator A of eq. 1 and the
    migration operator A^T of eq. 2, as the finite-difference Born operator
    defined in ``orc.c`` (the paper's own operator is a split-step one-way
    operator with no formulas given, Examples section);
  * ``cgls``: the damped least-squares problem of eq. 3 (normal equations
    eq. 4) solved by conjugate gradients on the least-squares form, one A and
    one A^T per iteration, all vectors and scalars in FP64;
  * ``chain``: the block-row recursion of eqs. 10-11: windows of Q shots
    sliding by S (rank-S update and downdate), each window's CG warm-started
    from the previous window's image (the reading used for eq. 11 regularises
    the whole image, so each window solves eq. 10 exactly as posed);
  * ``illumination`` / ``illumination_minv``: the diagonal preconditioner the
    paper asks for in each window's CG (it names none; this build's reading:
    the source-side illumination sum over the window's shots and time levels
    of (D2 u0^n)^2, inverted with a stabiliser of 1 % of its mean), used by
    ``cgls(..., minv=...)``;
  * ``oracle.ssf``: the paper's own operator family, split-step Fourier
    shot-profile de-migration and migration (Examples section), whose
    problems plug into ``cgls`` and ``chain`` unchanged.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "orc.c")


def build(force: bool = False) -> str:
    """Compile orc.c into liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
            "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ci, cd = ctypes.c_int, ctypes.c_double
        dims = [ci, ci, ci, ci, ci, cd]
        L.orc_padded_size.argtypes = [ci, ci, ci, ci, ci, i64p]
        L.orc_medium.argtypes = dims + [cd, dp, dp, dp, dp]
        L.orc_ricker.argtypes = [ci, cd, cd, dp]
        L.orc_laplacian.argtypes = dims + [dp, dp]
        shot = [dp, dp, dp, ci, ci, ci, dp, ci, ci, ip]
        L.orc_background.argtypes = dims + [cd] + shot + [dp, dp]
        L.orc_born.argtypes = dims + [cd] + shot + [dp, dp]
        L.orc_adjoint.argtypes = dims + [cd] + shot + [dp, dp]
        for f in ("orc_padded_size", "orc_medium", "orc_ricker",
                  "orc_laplacian", "orc_background", "orc_born",
                  "orc_adjoint"):
            getattr(L, f).restype = ci
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def ricker(nt: int, dt: float, f0: float) -> np.ndarray:
    out = np.zeros(nt)
    _check(lib().orc_ricker(nt, dt, f0, _dp(out)), "ricker")
    return out


@dataclass
class Grid:
    ndim: int
    nz: int
    ny: int
    nx: int
    nb: int
    h: float
    dt: float

    @property
    def padded_shape(self):
        py = self.ny + 2 * self.nb if self.ndim == 3 else 1
        return (self.nz + 2 * self.nb, py, self.nx + 2 * self.nb)

    @property
    def model_shape(self):
        return (self.nz, self.ny if self.ndim == 3 else 1, self.nx)

    def args(self):
        return (self.ndim, self.nz, self.ny if self.ndim == 3 else 1, self.nx,
                self.nb, float(self.h))


def laplacian(grid: Grid, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(grid.padded_shape)
    out = np.zeros_like(u)
    _check(lib().orc_laplacian(*grid.args(), _dp(u), _dp(out)), "laplacian")
    return out


class Medium:
    """Padded W = v^2 dt^2, C1, C2 for a model-grid velocity."""

    def __init__(self, grid: Grid, vel: np.ndarray):
        self.grid = grid
        v = np.ascontiguousarray(vel, dtype=np.float64).reshape(
            grid.model_shape)
        shp = grid.padded_shape
        self.W = np.zeros(shp)
        self.C1 = np.zeros(shp)
        self.C2 = np.zeros(shp)
        _check(lib().orc_medium(*grid.args(), float(grid.dt), _dp(v),
                                _dp(self.W), _dp(self.C1), _dp(self.C2)),
               "medium")


@dataclass
class ShotGeom:
    src: tuple
    rec: np.ndarray  # int32 [nrec, 3]
    nt: int
    f0: float
    wavelet: Optional[np.ndarray] = None

    def __post_init__(self):
        self.rec = np.ascontiguousarray(self.rec, dtype=np.int32).reshape(-1, 3)
        if self.wavelet is not None:
            self.wavelet = np.ascontiguousarray(self.wavelet, np.float64)

    @property
    def nrec(self):
        return int(self.rec.shape[0])


class Problem:
    """Operator pair over shots on one medium (all FP64)."""

    def __init__(self, grid: Grid, vel: np.ndarray, shots: Sequence,
                 medium: Optional[Medium] = None):
        self.grid = grid
        self.medium = medium if medium is not None else Medium(grid, vel)
        self.shots: List[ShotGeom] = []
        for s in shots:
            g = s if isinstance(s, ShotGeom) else ShotGeom(
                tuple(s.src), s.rec, s.nt, s.f0)
            if g.wavelet is None:  # Ricker of the shot's peak frequency
                g.wavelet = ricker(g.nt, grid.dt, g.f0)
            self.shots.append(g)

    @classmethod
    def from_workload(cls, w, shots=None):
        grid = Grid(w.ndim, w.nz, w.ny, w.nx, w.nb, w.h, w.dt)
        return cls(grid, w.vel, w.shots if shots is None else shots)

    def _shot_args(self, s: ShotGeom, medium: Optional[Medium] = None):
        med = medium or self.medium
        z, y, x = s.src
        return (_dp(med.W), _dp(med.C1), _dp(med.C2), int(z), int(y), int(x),
                _dp(s.wavelet), int(s.nt), s.nrec, _ip(s.rec))

    def data_shape(self, i: int):
        s = self.shots[i]
        return (s.nt, s.nrec)

    # --- single shot -----------------------------------------------------
    def born_shot(self, i: int, m: np.ndarray) -> np.ndarray:
        s = self.shots[i]
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(
            self.grid.model_shape)
        d = np.zeros((s.nt, s.nrec))
        _check(lib().orc_born(*self.grid.args(), float(self.grid.dt),
                              *self._shot_args(s), _dp(m), _dp(d)), "born")
        return d

    def adjoint_shot(self, i: int, r: np.ndarray) -> np.ndarray:
        s = self.shots[i]
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(s.nt, s.nrec)
        g = np.zeros(self.grid.model_shape)
        _check(lib().orc_adjoint(*self.grid.args(), float(self.grid.dt),
                                 *self._shot_args(s), _dp(r), _dp(g)),
               "adjoint")
        return g

    def background_shot(self, i: int, want_d2u0=False, want_rec=True,
                        medium: Optional[Medium] = None):
        s = self.shots[i]
        M = int(np.prod(self.grid.model_shape))
        d2 = np.zeros((max(s.nt - 1, 0), M)) if want_d2u0 else None
        ur = np.zeros((s.nt, s.nrec)) if want_rec else None
        _check(lib().orc_background(*self.grid.args(), float(self.grid.dt),
                                    *self._shot_args(s, medium), _dp(d2),
                                    _dp(ur)), "background")
        return d2, ur

    # --- window ------------------------------------------------------------
    def born(self, m: np.ndarray, idx: Sequence[int]) -> List[np.ndarray]:
        return [self.born_shot(i, m) for i in idx]

    def adjoint(self, r: Sequence[np.ndarray], idx: Sequence[int]):
        g = np.zeros(self.grid.model_shape)
        for ri, i in zip(r, idx):  # fixed order: slot order
            g += self.adjoint_shot(i, ri)
        return g


def _dot(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    return float(sum(np.vdot(x, y) for x, y in zip(a, b)))


@dataclass
class CGLSResult:
    m: np.ndarray
    iters: int
    s0_norm: float
    s_norms: List[float]
    r_norms: List[float]
    alphas: List[float]
    betas: List[float]
    iterates: Optional[List[np.ndarray]] = None


def cgls(prob: Problem, idx: Sequence[int], d: Sequence[np.ndarray],
         lam: float, niter: int, m0: Optional[np.ndarray] = None,
         rtol: float = 0.0, keep_iterates: bool = False,
         minv: Optional[np.ndarray] = None,
         m_ref: Optional[np.ndarray] = None,
         weights: Optional[Sequence[float]] = None) -> CGLSResult:
    """CG on min ||A m - d||^2 + lam ||m||^2 (eq. 3 / eq. 10), least-squares
    form: one A and one A^T per iteration, all in FP64.

    With ``minv`` (the inverse of a positive diagonal preconditioner M, model
    shaped) this is preconditioned CG on the normal equations
    (A^T A + lam I) m = A^T d: the search direction follows M^{-1} s, with
    gamma = <s, M^{-1} s>.

    With ``m_ref`` the damping pulls towards m_ref instead of zero:
    min ||A m - d||^2 + lam ||m - m_ref||^2, i.e. s = A^T r - lam (m - m_ref)
    (the correction-regularised recursion when m_ref is the previous
    window's image).

    With ``weights`` (one per shot of ``idx``, >= 0) shot j's misfit counts
    w_j times: min sum_j w_j ||A_j m - d_j||^2 + lam ||m - m_ref||^2, CG on
    (A^T W A + lam I) m = A^T W d with W the per-shot weights; the
    exponentially weighted (forgetting-factor) window sets w_j = beta^age.
    The search runs on the unweighted residual r = d - A m, with
    s = A^T W r - lam (m - m_ref) and delta = <q, W q> + lam <p, p>.

    Stops after ``niter`` iterations, or earlier once
    ||A^T W r - lam m|| <= rtol * ||A^T W d|| (s unpreconditioned in
    both)."""
    m = np.zeros(prob.grid.model_shape) if m0 is None else np.array(
        m0, dtype=np.float64).reshape(prob.grid.model_shape)
    d = [np.asarray(x, dtype=np.float64) for x in d]
    w = None if minv is None else np.asarray(
        minv, dtype=np.float64).reshape(prob.grid.model_shape)
    mr = np.zeros(prob.grid.model_shape) if m_ref is None else np.array(
        m_ref, dtype=np.float64).reshape(prob.grid.model_shape)
    wts = np.ones(len(idx)) if weights is None else np.asarray(
        weights, dtype=np.float64)
    if wts.shape != (len(idx),) or not np.all(np.isfinite(wts)) or \
            np.any(wts < 0):
        raise ValueError("weights: one finite value >= 0 per shot")

    def wt(x):  # W x, per shot
        return [w * xi for w, xi in zip(wts, x)]
    Am = prob.born(m, idx)
    r = [di - ai for di, ai in zip(d, Am)]
    s = prob.adjoint(wt(r), idx) - lam * (m - mr)
    z = s if w is None else w * s
    p = z.copy()
    gamma = float(np.vdot(s, z))
    snorm = float(np.linalg.norm(s))
    ref = None
    if rtol > 0:
        ref = np.linalg.norm(prob.adjoint(wt(d), idx))
    res = CGLSResult(m, 0, snorm, [snorm], [np.sqrt(_dot(r, r))], [], [],
                     [m.copy()] if keep_iterates else None)
    for k in range(niter):
        if ref is not None and snorm <= rtol * ref:
            break
        if gamma == 0.0:
            break
        q = prob.born(p, idx)
        delta = _dot(q, wt(q)) + lam * float(np.vdot(p, p))
        if delta <= 0.0:
            raise ArithmeticError("CG breakdown: delta <= 0")
        alpha = gamma / delta
        m = m + alpha * p
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        s = prob.adjoint(wt(r), idx) - lam * (m - mr)
        z = s if w is None else w * s
        gamma_new = float(np.vdot(s, z))
        beta = gamma_new / gamma
        p = z + beta * p
        gamma = gamma_new
        snorm = float(np.linalg.norm(s))
        res.iters += 1
        res.alphas.append(alpha)
        res.betas.append(beta)
        res.s_norms.append(snorm)
        res.r_norms.append(np.sqrt(_dot(r, r)))
        if keep_iterates:
            res.iterates.append(m.copy())
    res.m = m
    return res


def illumination(prob: Problem, idx: Sequence[int]) -> np.ndarray:
    """Source-side illumination of a window: at each model point, the sum
    over the window's shots and over the time levels n = 0 .. nt-2 of the
    squared Born source (D2 u0^n)^2 (the stored frames of eq. F2)."""
    acc = np.zeros(int(np.prod(prob.grid.model_shape)))
    for i in idx:
        d2, _ = prob.background_shot(i, want_d2u0=True, want_rec=False)
        acc += np.sum(d2 * d2, axis=0)
    return acc.reshape(prob.grid.model_shape)


# stabiliser of the illumination preconditioner, relative to the mean
ILLUM_EPS = 0.01


def illumination_minv(illum: np.ndarray) -> np.ndarray:
    """Inverse diagonal preconditioner 1 / (I + ILLUM_EPS * mean(I))."""
    illum = np.asarray(illum, dtype=np.float64)
    return 1.0 / (illum + ILLUM_EPS * float(np.mean(illum)))


@dataclass
class ChainResult:
    m: np.ndarray
    windows: List[List[int]]
    images: List[np.ndarray]
    results: List[CGLSResult]


def chain(prob: Problem, data: Sequence[np.ndarray], windows, lam: float,
          niter: int, m0: Optional[np.ndarray] = None,
          correction: bool = False,
          forgetting: Optional[float] = None) -> ChainResult:
    """Block-row recursion (eqs. 10-11): solve each window's damped problem by
    CG, starting from the previous window's image (zero for the first).
    ``correction``: damp the correction to the previous image instead of the
    image (min ||A_w m - d_w||^2 + lam ||m - m_{w-1}||^2). ``forgetting``:
    a factor beta in (0, 1] weighting each shot's misfit by beta^age, age
    the number of earlier windows that held it (the exponentially weighted
    window of forgetting-factor RLS)."""
    m = m0
    images, results = [], []
    first = {}
    for k, w in enumerate(windows):
        for i in w:
            first.setdefault(i, k)
        wts = None if forgetting is None else \
            [float(forgetting) ** (k - first[i]) for i in w]
        res = cgls(prob, w, [data[i] for i in w], lam, niter, m0=m,
                   m_ref=m if correction else None, weights=wts)
        m = res.m
        images.append(m.copy())
        results.append(res)
    return ChainResult(m, [list(w) for w in windows], images, results)


def synthesize_data(prob: Problem, m_true: np.ndarray, noise_rel: float,
                    noise_std: Sequence[np.ndarray]) -> List[np.ndarray]:
    """d = A m_true + n with n = noise_rel * RMS(A m_true) * noise_std
    (eq. 1); ``noise_std`` are standard-normal arrays, one per shot."""
    clean = [prob.born_shot(i, m_true) for i in range(len(prob.shots))]
    allv = np.concatenate([c.ravel() for c in clean])
    sigma = noise_rel * np.sqrt(np.mean(allv * allv))
    return [c + sigma * n.reshape(c.shape) for c, n in zip(clean, noise_std)]


def power_norm(prob: Problem, idx: Sequence[int], iters: int, seed: int):
    """Estimate ||A_w^T A_w|| by power iteration from a seeded start."""
    x = np.random.default_rng(seed).standard_normal(prob.grid.model_shape)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = prob.adjoint(prob.born(x, idx), idx)
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam
