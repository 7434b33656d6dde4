"""Python binding of the split-step Fourier context (C ABI in
``include/brrlsm_ssf.h``): the shot-profile de-migration / migration pair of
the paper's examples inside the same block-row recursion. The methods carry
the C names and only marshal arguments; every step runs in the library's
gfx950 kernels.

Host arrays are numpy float32 / int32; with ``device=True`` pass contiguous
float32 torch CUDA tensors and the library orders its work on torch's current
stream.
"""
from __future__ import annotations

import ctypes
from typing import List

import numpy as np

from . import _lib as L
from . import _ptr


class SsfContext:
    """One velocity model, one window of shots, one image."""

    def __init__(self, handle, nz, nx, nt, device):
        self._h = handle
        self.model_shape = (nz, nx)
        self.model_size = nz * nx
        self.nt = nt
        self.device = device
        # bumped by every update and downdate (see Context.generation)
        self.generation = 0

    def close(self):
        if self._h:
            L.lib().brls_ssf_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        return L.check_ssf(rc, self._h)

    def brls_ssf_band(self):
        """(k0, nw, df): the band's first DFT index, count and spacing."""
        k0, nw, df = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(L.lib().brls_ssf_band(self._h, ctypes.byref(k0),
                                          ctypes.byref(nw), ctypes.byref(df)))
        return k0.value, nw.value, df.value

    band = brls_ssf_band

    def brls_ssf_update(self, id: int, xs: int, rec, f0: float, data=None):
        rec = np.ascontiguousarray(rec, dtype=np.int32).ravel()
        sh = L.brls_ssf_shot()
        sh.id = int(id)
        sh.xs = int(xs)
        sh.nrec = int(rec.size)
        sh.f0 = float(f0)
        sh.rec = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if data is not None and not self.device:
            data = np.ascontiguousarray(data, dtype=np.float32)
        p = _ptr(data, self.device, self.nt * sh.nrec)
        sh.data = p.value if p is not None else None
        self._check(L.lib().brls_ssf_update(self._h, ctypes.byref(sh)))
        self.generation += 1

    update = brls_ssf_update

    def brls_ssf_downdate(self, id: int):
        self._check(L.lib().brls_ssf_downdate(self._h, int(id)))
        self.generation += 1

    downdate = brls_ssf_downdate

    def brls_ssf_window(self) -> List[int]:
        n = ctypes.c_int32()
        self._check(L.lib().brls_ssf_window(self._h, None, 0,
                                            ctypes.byref(n)))
        ids = (ctypes.c_int64 * max(n.value, 1))()
        self._check(L.lib().brls_ssf_window(self._h, ids, n.value,
                                            ctypes.byref(n)))
        return list(ids[:n.value])

    window = brls_ssf_window

    def brls_ssf_window_data_size(self) -> int:
        n = ctypes.c_int64()
        self._check(L.lib().brls_ssf_window_data_size(self._h,
                                                      ctypes.byref(n)))
        return n.value

    window_data_size = brls_ssf_window_data_size

    def _data_out(self, out):
        if out is not None:
            return out
        n = self.window_data_size()
        if self.device:
            import torch
            return torch.empty(n, dtype=torch.float32, device="cuda")
        return np.empty(n, dtype=np.float32)

    def _model_out(self, out):
        if out is not None:
            return out
        if self.device:
            import torch
            return torch.empty(self.model_shape, dtype=torch.float32,
                               device="cuda")
        return np.empty(self.model_shape, dtype=np.float32)

    def _in(self, a):
        return a if self.device else np.ascontiguousarray(a, dtype=np.float32)

    def brls_ssf_apply_born(self, m, out=None):
        m = self._in(m)
        out = self._data_out(out)
        self._check(L.lib().brls_ssf_apply_born(
            self._h, _ptr(m, self.device, self.model_size),
            _ptr(out, self.device, self.window_data_size())))
        return out

    apply_born = brls_ssf_apply_born

    def brls_ssf_apply_adjoint(self, d, out=None):
        d = self._in(d)
        out = self._model_out(out)
        self._check(L.lib().brls_ssf_apply_adjoint(
            self._h, _ptr(d, self.device, self.window_data_size()),
            _ptr(out, self.device, self.model_size)))
        return out

    apply_adjoint = brls_ssf_apply_adjoint

    def brls_ssf_observed(self, out=None):
        out = self._data_out(out)
        self._check(L.lib().brls_ssf_observed(
            self._h, _ptr(out, self.device, self.window_data_size())))
        return out

    observed = brls_ssf_observed

    def brls_ssf_solve_window(self, max_iter: int, rtol: float = 0.0) -> dict:
        st = L.brls_stats()
        self._check(L.lib().brls_ssf_solve_window(
            self._h, int(max_iter), float(rtol), ctypes.byref(st)))
        return {"iters": st.iters, "s0_norm": st.s0_norm,
                "s_norm": st.s_norm, "r_norm": st.r_norm,
                "seconds": st.seconds, "ref_norm": st.ref_norm}

    solve_window = brls_ssf_solve_window

    def brls_ssf_set_precond(self, mode: int):
        """0: plain CG; 1: diagonal illumination preconditioner."""
        self._check(L.lib().brls_ssf_set_precond(self._h, int(mode)))

    set_precond = brls_ssf_set_precond

    def brls_ssf_get_precond(self) -> int:
        v = ctypes.c_int32()
        self._check(L.lib().brls_ssf_get_precond(self._h, ctypes.byref(v)))
        return v.value

    get_precond = brls_ssf_get_precond

    def brls_ssf_illumination(self, out=None):
        out = self._model_out(out)
        self._check(L.lib().brls_ssf_illumination(
            self._h, _ptr(out, self.device, self.model_size)))
        return out

    illumination = brls_ssf_illumination

    def brls_ssf_set_regularization(self, mode: int):
        """0: damp the image; 1: damp the correction to the image the solve
        starts from (correction-regularised recursion)."""
        self._check(L.lib().brls_ssf_set_regularization(self._h, int(mode)))

    set_regularization = brls_ssf_set_regularization

    def brls_ssf_get_regularization(self) -> int:
        v = ctypes.c_int32()
        self._check(L.lib().brls_ssf_get_regularization(self._h,
                                                        ctypes.byref(v)))
        return v.value

    get_regularization = brls_ssf_get_regularization

    def brls_ssf_set_shot_weight(self, id: int, w: float):
        """Misfit weight of a window shot (1 by default)."""
        self._check(L.lib().brls_ssf_set_shot_weight(self._h, int(id),
                                                     float(w)))

    set_shot_weight = brls_ssf_set_shot_weight

    def brls_ssf_get_shot_weight(self, id: int) -> float:
        v = ctypes.c_double()
        self._check(L.lib().brls_ssf_get_shot_weight(self._h, int(id),
                                                     ctypes.byref(v)))
        return v.value

    get_shot_weight = brls_ssf_get_shot_weight

    def brls_ssf_image(self, out=None):
        out = self._model_out(out)
        self._check(L.lib().brls_ssf_image(
            self._h, _ptr(out, self.device, self.model_size)))
        return out

    image = brls_ssf_image

    def brls_ssf_set_image(self, m):
        m = self._in(m)
        self._check(L.lib().brls_ssf_set_image(
            self._h, _ptr(m, self.device, self.model_size)))

    set_image = brls_ssf_set_image

    def brls_ssf_kernel_timing(self, enable: bool = True):
        self._check(L.lib().brls_ssf_kernel_timing(self._h, int(enable)))

    kernel_timing = brls_ssf_kernel_timing

    def brls_ssf_kernel_stats(self) -> dict:
        arr = (L.brls_kstat * 16)()
        n = ctypes.c_int32()
        self._check(L.lib().brls_ssf_kernel_stats(self._h, arr, 16,
                                                  ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms)
                for i in range(min(n.value, 16))}

    kernel_stats = brls_ssf_kernel_stats

    def brls_ssf_memory_bytes(self) -> int:
        n = ctypes.c_int64()
        self._check(L.lib().brls_ssf_memory_bytes(self._h, ctypes.byref(n)))
        return n.value

    memory_bytes = brls_ssf_memory_bytes

    def brls_ssf_sync(self):
        self._check(L.lib().brls_ssf_sync(self._h))

    sync = brls_ssf_sync


def brls_ssf_open(nz: int, nx: int, dx: float, dz: float, nt: int,
                  dt: float, fmin: float, fmax: float, ntap: int,
                  nrec_max: int, q_max: int, lam: float, vel: np.ndarray,
                  device: bool = False, stream=None) -> SsfContext:
    """Open a split-step context for velocity ``vel`` [nz][nx] (m/s, host)."""
    g = L.brls_ssf_grid()
    g.nz, g.nx = int(nz), int(nx)
    g.dx, g.dz = float(dx), float(dz)
    g.nt, g.dt = int(nt), float(dt)
    g.fmin, g.fmax = float(fmin), float(fmax)
    g.ntap, g.nrec_max, g.q_max = int(ntap), int(nrec_max), int(q_max)
    g.lambda_ = float(lam)
    g.flags = L.BRLS_DEVICE_PTRS if device else 0
    if device and stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    v = np.ascontiguousarray(vel, dtype=np.float32)
    if v.size < nz * nx:
        raise ValueError(f"vel holds {v.size} values, the grid has "
                         f"{nz * nx} points")
    h = ctypes.c_void_p()
    rc = L.lib().brls_ssf_open(ctypes.byref(g), v.ctypes.data,
                               ctypes.c_void_p(stream) if stream else None,
                               ctypes.byref(h))
    L.check_ssf(rc, None)
    return SsfContext(h, nz, nx, nt, device)
