"""FP64 oracle of the split-step Fourier shot-profile operators: de-migration
A (Born modelling) and migration A^T, the operator family the paper's
examples use (Examples section: shot-profile wave-equation forward and
adjoint operators with a split-step correction, applied to finite-difference
data from a Ricker source).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it; it shares no code with
the GPU library.

The paper names the operator and gives no formulas; what follows is this
implementation's reading, written from standard one-way wave theory
(phase shift in the wavenumber domain with a reference slowness per depth
level, then a split-step phase in space for the lateral variation):

* 2-D grid of nz depth levels and nx columns (nx a power of two, the lateral
  FFT length), spacings dz and dx; slowness s = 1/v; the reference slowness
  of level j is the mean s0_j of s over the row; the split-step time
  theta_j(x) = (s_j(x) - s0_j) dz.
* Frequencies: the nt-point DFT grid df = 1/(nt dt) restricted to
  [fmin, fmax]: w_k = 2 pi (k0 + k) df, k0 = ceil(fmin/df),
  k = 0 .. nw-1 up to floor(fmax/df). Time series x_n become
  X(w) = sum_n x_n exp(-i w n dt) dt.
* One depth step through level j, E_j u: FFT over x (exp(-i kx x)), times
  exp(-i kz dz) with kz = sqrt(w^2 s0_j^2 - kx^2) where that is real and
  exp(-sqrt(kx^2 - w^2 s0_j^2) dz) where it is not, inverse FFT, times
  exp(-i w theta_j(x)), times a lateral taper tau(x) (cosine over ntap
  cells at each side, 1 inside). Time runs as exp(+i w t), so each step
  adds traveltime. E_j^H undoes the factors in reverse with conjugates.
* Source at column xs of level 0:
  S_0 = F(w) (-i / (2 w s(0, xs))) delta(x - xs), F the DFT of the Ricker
  wavelet of peak f0 delayed by 1.5/f0; S_{j+1} = E_j S_j. The factor
  -i/(2 w s) is the vertical-incidence one-way form of a 2-D point source:
  with it the field below the source is dx F G, G = (-i/4) H0^(2)(w s r)
  the outgoing Green's function of the Helmholtz equation, so the one-way
  source radiates like the two-way point source of the finite-difference
  operator.
* Born scattering at level j of a relative squared-slowness perturbation m
  (the same m as the finite-difference operator): the first-order change of
  the split-step phase when s becomes s (1 + m/2), injected as
  W_j m_j with W_j = -i (w dz / 2) s_j S_j.
* A (de-migration): R_{nz-1} = W_{nz-1} m_{nz-1}; R_j = W_j m_j + E_j R_{j+1}
  (the scattered field travels up, adding traveltime); data = R_0 at the
  receivers' columns (level 0).
* A^T (migration): Q_0 = receivers' data scattered into their columns;
  image_j = Re sum_w conj(W_j) Q_j; Q_{j+1} = E_j^H Q_j (the receiver field
  continued down with the adjoint step; the imaging condition is the
  zero-lag cross-correlation with the source field).
* Data of one shot are complex, nw x nrec; as real vectors they are stored
  as (re, im) pairs, shape (nw, nrec, 2), so that the CG solver of the
  window (``oracle.cgls``) works on them with the real inner product
  Re(a^H b) = sum a_re b_re + a_im b_im, under which A^T above is the exact
  adjoint of A.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

from . import ricker


def band(nt: int, dt: float, fmin: float, fmax: float):
    """The DFT frequency grid of nt samples at dt restricted to [fmin, fmax]:
    (df, k0, nw) with frequencies (k0 + k) df, k = 0 .. nw-1."""
    df = 1.0 / (nt * dt)
    k0 = int(np.ceil(fmin / df - 1e-9))
    k1 = int(np.floor(fmax / df + 1e-9))
    if k1 < k0:
        raise ValueError("empty frequency band")
    return df, k0, k1 - k0 + 1


def dft(x: np.ndarray, dt: float, omegas: np.ndarray) -> np.ndarray:
    """X(w) = sum_n x_n exp(-i w n dt) dt along axis 0 (the definition,
    written out as a matrix product)."""
    x = np.asarray(x, dtype=np.float64)
    n = np.arange(x.shape[0])
    kern = np.exp(-1j * np.outer(omegas, n * dt)) * dt
    return kern @ x.reshape(x.shape[0], -1)


def taper(nx: int, ntap: int) -> np.ndarray:
    """1 inside; 0.5 (1 - cos(pi (d + 1) / (ntap + 1))) at distance d < ntap
    from either lateral edge."""
    t = np.ones(nx)
    for d in range(min(ntap, nx)):
        v = 0.5 * (1.0 - np.cos(np.pi * (d + 1) / (ntap + 1)))
        t[d] = min(t[d], v)
        t[nx - 1 - d] = min(t[nx - 1 - d], v)
    return t


@dataclass
class SsfGrid:
    nz: int
    nx: int

    @property
    def model_shape(self):
        return (self.nz, self.nx)


@dataclass
class SsfShot:
    xs: int              # source column (level 0)
    rec: np.ndarray      # receiver columns (level 0), int
    f0: float            # Ricker peak frequency (Hz)


@dataclass
class SsfProblem:
    vel: np.ndarray      # (nz, nx) velocity, m/s
    dx: float
    dz: float
    nt: int
    dt: float
    fmin: float
    fmax: float
    ntap: int
    shots: List[SsfShot] = field(default_factory=list)

    def __post_init__(self):
        v = np.asarray(self.vel, dtype=np.float64)
        nz, nx = v.shape
        if nx & (nx - 1):
            raise ValueError("nx must be a power of two")
        self.grid = SsfGrid(nz, nx)
        self.s = 1.0 / v
        self.s0 = self.s.mean(axis=1)
        self.theta = (self.s - self.s0[:, None]) * self.dz
        self.tau = taper(nx, self.ntap)
        self.kx = 2.0 * np.pi * np.fft.fftfreq(nx, self.dx)
        self.df, self.k0, self.nw = band(self.nt, self.dt, self.fmin,
                                         self.fmax)
        self.omegas = 2.0 * np.pi * (self.k0 + np.arange(self.nw)) * self.df

    # --- one depth step --------------------------------------------------
    def phase(self, j: int) -> np.ndarray:
        """(nw, nx) wavenumber-domain factor of level j."""
        a = (self.omegas[:, None] * self.s0[j]) ** 2 - self.kx[None, :] ** 2
        kz = np.sqrt(np.abs(a))
        return np.where(a >= 0, np.exp(-1j * kz * self.dz),
                        np.exp(-kz * self.dz))

    def step(self, u: np.ndarray, j: int) -> np.ndarray:
        """E_j applied to u of shape (nw, nx)."""
        u = np.fft.ifft(np.fft.fft(u, axis=-1) * self.phase(j), axis=-1)
        return u * np.exp(-1j * np.outer(self.omegas, self.theta[j])) \
            * self.tau

    def step_adj(self, u: np.ndarray, j: int) -> np.ndarray:
        """E_j^H applied to u of shape (nw, nx)."""
        u = u * self.tau * np.exp(1j * np.outer(self.omegas, self.theta[j]))
        return np.fft.ifft(np.fft.fft(u, axis=-1) * np.conj(self.phase(j)),
                           axis=-1)

    # --- per-shot pieces -------------------------------------------------
    def wavelet(self, f0: float) -> np.ndarray:
        return dft(ricker(self.nt, self.dt, f0), self.dt, self.omegas)[:, 0]

    def weights(self, i: int) -> np.ndarray:
        """W_j = -i (w dz/2) s_j S_j for every level: (nz, nw, nx)."""
        sh = self.shots[i]
        nz, nx = self.grid.model_shape
        S = np.zeros((self.nw, nx), dtype=np.complex128)
        S[:, sh.xs] = self.wavelet(sh.f0) * (
            -0.5j / (self.omegas * self.s[0, sh.xs]))
        W = np.empty((nz, self.nw, nx), dtype=np.complex128)
        for j in range(nz):
            W[j] = -0.5j * self.dz * self.omegas[:, None] * self.s[j] * S
            if j + 1 < nz:
                S = self.step(S, j)
        return W

    def born_shot(self, i: int, m: np.ndarray, W=None) -> np.ndarray:
        """A_i m as complex (nw, nrec)."""
        W = self.weights(i) if W is None else W
        m = np.asarray(m, dtype=np.float64).reshape(self.grid.model_shape)
        nz = self.grid.nz
        R = W[nz - 1] * m[nz - 1]
        for j in range(nz - 2, -1, -1):
            R = W[j] * m[j] + self.step(R, j)
        return R[:, np.asarray(self.shots[i].rec)]

    def adjoint_shot(self, i: int, D: np.ndarray, W=None) -> np.ndarray:
        """A_i^T D for complex D of shape (nw, nrec): image (nz, nx)."""
        W = self.weights(i) if W is None else W
        nz, nx = self.grid.model_shape
        Q = np.zeros((self.nw, nx), dtype=np.complex128)
        np.add.at(Q, (slice(None), np.asarray(self.shots[i].rec)),
                  np.asarray(D, dtype=np.complex128))
        img = np.zeros((nz, nx))
        for j in range(nz):
            img[j] = np.sum(np.conj(W[j]) * Q, axis=0).real
            if j + 1 < nz:
                Q = self.step_adj(Q, j)
        return img

    # --- window operators on real (re, im) pairs -------------------------
    def born(self, m: np.ndarray, idx: Sequence[int]) -> List[np.ndarray]:
        out = []
        for i in idx:
            D = self.born_shot(i, m)
            out.append(np.stack([D.real, D.imag], axis=-1))
        return out

    def adjoint(self, r: Sequence[np.ndarray], idx: Sequence[int]):
        img = np.zeros(self.grid.model_shape)
        for i, x in zip(idx, r):
            x = np.asarray(x, dtype=np.float64)
            img += self.adjoint_shot(i, x[..., 0] + 1j * x[..., 1])
        return img

    def illumination(self, idx: Sequence[int]) -> np.ndarray:
        """Source-side illumination of a window: at each point, the sum over
        its shots and frequencies of |W_j(x)|^2 (the diagonal of A^T A when
        the receivers record every column of the level itself, with no
        propagation between scatterer and receiver)."""
        acc = np.zeros(self.grid.model_shape)
        for i in idx:
            acc += np.sum(np.abs(self.weights(i)) ** 2, axis=1)
        return acc

    def observed(self, d_time: np.ndarray) -> np.ndarray:
        """Time-domain data (nt, nrec) of one shot to the operator's data
        space: (nw, nrec, 2) pairs of its DFT over the band."""
        D = dft(d_time, self.dt, self.omegas)
        return np.stack([D.real, D.imag], axis=-1)
