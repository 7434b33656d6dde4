"""Block-row recursive least-squares migration on MI355X.

Python binding of the HIP library ``libbrrlsm.so`` (C ABI in
``include/brrlsm.h``). The functions below carry the C names and only marshal
arguments; all computation runs in the library's gfx950 kernels.

Host arrays are numpy float32 / int32. With ``device=True`` the context
takes device pointers: pass torch CUDA tensors (float32, contiguous), and the
library orders its work on torch's current stream.

Method: Kazemi & Sacchi, "Block row recursive least squares migration"
(arXiv 1801.00819): eqs. 1-4 (Born de-migration A, migration A^T, damped
least squares) and eqs. 10-11 (sliding windows of shots with rank-K update,
downdate and warm-started CG).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional

import numpy as np

from . import _lib as L
from ._lib import (BRLS_EXEC_BATCHED, BRLS_EXEC_GRAPH,  # noqa: F401
                   BRLS_EXEC_PERSISTENT, BRLS_EXEC_PLAIN, BrlsError)

__all__ = [
    "Context", "brls_open", "BrlsError", "BRLS_EXEC_PLAIN",
    "BRLS_EXEC_BATCHED", "BRLS_EXEC_GRAPH", "BRLS_EXEC_PERSISTENT",
]


def _ptr(a, device: bool, n: Optional[int] = None, bits: int = 32):
    """Pointer to a float32 (``bits`` 64: float64) buffer the library reads
    or writes: a contiguous CUDA tensor (device context) or a C-contiguous
    ndarray (host context) holding at least ``n`` elements."""
    if a is None:
        return None
    if device:
        import torch
        want = torch.float32 if bits == 32 else torch.float64
        if not (isinstance(a, torch.Tensor) and a.is_cuda):
            raise TypeError("device context: pass a CUDA tensor")
        if a.dtype != want:
            raise TypeError(f"tensor must be {want}, got {a.dtype}")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        size = a.numel()
        ptr = a.data_ptr()
    else:
        want = np.float32 if bits == 32 else np.float64
        if not (isinstance(a, np.ndarray) and a.dtype == want
                and a.flags.c_contiguous):
            raise TypeError(f"host context: pass a C-contiguous "
                            f"{np.dtype(want).name} ndarray")
        size = a.size
        ptr = a.ctypes.data
    if n is not None and size < n:
        raise ValueError(f"buffer holds {size} floats, the call needs {n}")
    return ctypes.c_void_p(ptr)


class Context:
    """One velocity model, one window of shots, one image."""

    def __init__(self, handle, nz, ny, nx, device):
        self._h = handle
        self.model_shape = (nz, ny, nx)
        self.model_size = nz * ny * nx
        self.device = device
        self._keep = []
        self._data_size = {}  # shot id -> nt * nrec
        # bumped by every update and downdate: the window (and so the
        # operator) a result belongs to
        self.generation = 0

    # ------------------------------------------------------------------
    def close(self):
        if self._h:
            L.lib().brls_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        return L.check(rc, self._h)

    def brls_update(self, id: int, src, rec: np.ndarray, nt: int, f0: float,
                    data=None):
        rec = np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 3)
        sh = L.brls_shot()
        sh.id = int(id)
        sh.sz, sh.sy, sh.sx = (int(v) for v in src)
        sh.nt = int(nt)
        sh.nrec = int(rec.shape[0])
        sh.f0 = float(f0)
        sh.rec = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if data is not None and not self.device:
            data = np.ascontiguousarray(data, dtype=np.float32)
        p = _ptr(data, self.device, sh.nt * sh.nrec)
        sh.data = p.value if p is not None else None
        self._check(L.lib().brls_update(self._h, ctypes.byref(sh)))
        self._data_size[int(id)] = sh.nt * sh.nrec
        self.generation += 1

    update = brls_update

    def brls_downdate(self, id: int):
        self._check(L.lib().brls_downdate(self._h, int(id)))
        self._data_size.pop(int(id), None)
        self.generation += 1

    downdate = brls_downdate

    def brls_set_data(self, id: int, data):
        if not self.device:
            data = np.ascontiguousarray(data, dtype=np.float32)
        self._check(L.lib().brls_set_data(
            self._h, int(id),
            _ptr(data, self.device, self._data_size.get(int(id)))))

    set_data = brls_set_data

    def brls_window(self) -> List[int]:
        n = ctypes.c_int32()
        self._check(L.lib().brls_window(self._h, None, 0, ctypes.byref(n)))
        ids = (ctypes.c_int64 * max(n.value, 1))()
        self._check(L.lib().brls_window(self._h, ids, n.value,
                                        ctypes.byref(n)))
        return list(ids[:n.value])

    window = brls_window

    def brls_window_data_size(self) -> int:
        n = ctypes.c_int64()
        self._check(L.lib().brls_window_data_size(self._h, ctypes.byref(n)))
        return n.value

    window_data_size = brls_window_data_size

    def brls_solve_window(self, max_iter: int, rtol: float = 0.0) -> dict:
        st = L.brls_stats()
        self._check(L.lib().brls_solve_window(self._h, int(max_iter),
                                              float(rtol), ctypes.byref(st)))
        return dict(iters=st.iters, s0_norm=st.s0_norm, s_norm=st.s_norm,
                    r_norm=st.r_norm, seconds=st.seconds,
                    ref_norm=st.ref_norm)

    solve_window = brls_solve_window

    def brls_solve_history(self) -> dict:
        """alpha, beta and ||s|| per iteration of the last solve."""
        n = ctypes.c_int32()
        self._check(L.lib().brls_solve_history(self._h, 0, None, None, None,
                                               ctypes.byref(n)))
        k = n.value
        out = {x: np.zeros(k, np.float64) for x in ("alpha", "beta",
                                                     "s_norm")}
        if k:
            self._check(L.lib().brls_solve_history(
                self._h, k, out["alpha"].ctypes.data, out["beta"].ctypes.data,
                out["s_norm"].ctypes.data, ctypes.byref(n)))
        return out

    solve_history = brls_solve_history

    def _model_out(self, out):
        if out is not None:
            return out
        if self.device:
            import torch
            return torch.empty(self.model_shape, dtype=torch.float32,
                               device="cuda")
        return np.empty(self.model_shape, dtype=np.float32)

    def brls_image(self, out=None):
        out = self._model_out(out)
        self._check(L.lib().brls_image(self._h, _ptr(out, self.device,
                                                      self.model_size)))
        return out

    image = brls_image

    def brls_set_image(self, m):
        if not self.device:
            m = np.ascontiguousarray(m, dtype=np.float32)
        self._check(L.lib().brls_set_image(self._h, _ptr(m, self.device,
                                                          self.model_size)))

    set_image = brls_set_image

    def brls_image64(self, out=None):
        """The current image in float64 (the chain's full state with float64
        CG vectors)."""
        if out is None:
            if self.device:
                import torch
                out = torch.empty(self.model_shape, dtype=torch.float64,
                                  device="cuda")
            else:
                out = np.empty(self.model_shape, np.float64)
        self._check(L.lib().brls_image64(
            self._h, _ptr(out, self.device, self.model_size, 64)))
        return out

    image64 = brls_image64

    def brls_set_image64(self, m):
        if not self.device:
            m = np.ascontiguousarray(m, dtype=np.float64)
        self._check(L.lib().brls_set_image64(
            self._h, _ptr(m, self.device, self.model_size, 64)))

    set_image64 = brls_set_image64

    def brls_set_precond(self, mode: int):
        """0: plain CG; 1: diagonal illumination preconditioner."""
        self._check(L.lib().brls_set_precond(self._h, int(mode)))

    set_precond = brls_set_precond

    def brls_set_regularization(self, mode: int):
        """0: damp the image; 1: damp the correction to the image the solve
        starts from (correction-regularised recursion)."""
        self._check(L.lib().brls_set_regularization(self._h, int(mode)))

    set_regularization = brls_set_regularization

    def brls_set_precision(self, background: int = 64, vectors: int = 64):
        """Bits of the background wavefield of new shots (64 needs stored
        Born sources) and of the CG vectors: 32 or 64 each."""
        self._check(L.lib().brls_set_precision(self._h, int(background),
                                               int(vectors)))

    set_precision = brls_set_precision

    def brls_get_precision(self):
        b, v = ctypes.c_int32(), ctypes.c_int32()
        self._check(L.lib().brls_get_precision(self._h, ctypes.byref(b),
                                               ctypes.byref(v)))
        return b.value, v.value

    get_precision = brls_get_precision

    def brls_set_shot_weight(self, id: int, w: float):
        """Misfit weight of a window shot (1 by default; beta^age gives the
        exponentially weighted window)."""
        self._check(L.lib().brls_set_shot_weight(self._h, int(id), float(w)))

    set_shot_weight = brls_set_shot_weight

    def brls_get_shot_weight(self, id: int) -> float:
        v = ctypes.c_double()
        self._check(L.lib().brls_get_shot_weight(self._h, int(id),
                                                 ctypes.byref(v)))
        return v.value

    get_shot_weight = brls_get_shot_weight

    def brls_get_regularization(self) -> int:
        v = ctypes.c_int32()
        self._check(L.lib().brls_get_regularization(self._h,
                                                    ctypes.byref(v)))
        return v.value

    get_regularization = brls_get_regularization

    def brls_get_precond(self) -> int:
        v = ctypes.c_int32()
        self._check(L.lib().brls_get_precond(self._h, ctypes.byref(v)))
        return v.value

    get_precond = brls_get_precond

    def brls_illumination(self, out=None):
        out = self._model_out(out)
        self._check(L.lib().brls_illumination(
            self._h, _ptr(out, self.device, self.model_size)))
        return out

    illumination = brls_illumination

    def brls_apply_born(self, m, out=None):
        if not self.device:
            m = np.ascontiguousarray(m, dtype=np.float32)
        n = self.window_data_size()
        if out is None:
            if self.device:
                import torch
                out = torch.empty(n, dtype=torch.float32, device="cuda")
            else:
                out = np.empty(n, dtype=np.float32)
        self._check(L.lib().brls_apply_born(
            self._h, _ptr(m, self.device, self.model_size),
            _ptr(out, self.device, n)))
        return out

    apply_born = brls_apply_born

    def brls_apply_adjoint(self, d, out=None):
        if not self.device:
            d = np.ascontiguousarray(d, dtype=np.float32)
        out = self._model_out(out)
        self._check(L.lib().brls_apply_adjoint(
            self._h, _ptr(d, self.device, self.window_data_size()),
            _ptr(out, self.device, self.model_size)))
        return out

    apply_adjoint = brls_apply_adjoint

    def brls_apply_adjoint_static(self, d, out=None):
        """brls_apply_adjoint with the image accumulators in the library's
        static device scratch (no device allocation in the call)."""
        if not self.device:
            d = np.ascontiguousarray(d, dtype=np.float32)
        out = self._model_out(out)
        self._check(L.lib().brls_apply_adjoint_static(
            self._h, _ptr(d, self.device, self.window_data_size()),
            _ptr(out, self.device, self.model_size)))
        return out

    apply_adjoint_static = brls_apply_adjoint_static

    def brls_background_window(self, out=None):
        """Finite-difference modelling in the context's velocity: each
        window shot's background wavefield at its receivers, [nt][nrec] per
        shot in window order."""
        n = self.window_data_size()
        if out is None:
            if self.device:
                import torch
                out = torch.empty(n, dtype=torch.float32, device="cuda")
            else:
                out = np.empty(n, dtype=np.float32)
        self._check(L.lib().brls_background_window(
            self._h, _ptr(out, self.device, n)))
        return out

    background_window = brls_background_window

    def brls_set_exec(self, mode: int):
        self._check(L.lib().brls_set_exec(self._h, int(mode)))

    set_exec = brls_set_exec

    def brls_set_chains(self, n: int):
        """Concurrent launch chains of the batched and graph modes (1, 2)."""
        self._check(L.lib().brls_set_chains(self._h, int(n)))

    set_chains = brls_set_chains

    def brls_get_chains(self) -> int:
        n = ctypes.c_int32()
        self._check(L.lib().brls_get_chains(self._h, ctypes.byref(n)))
        return n.value

    get_chains = brls_get_chains

    def brls_set_spin_limit(self, polls: int):
        """Polls before a persistent launch's barrier wait gives up."""
        self._check(L.lib().brls_set_spin_limit(self._h, int(polls)))

    set_spin_limit = brls_set_spin_limit

    def brls_set_zchunk(self, planes: int):
        """3-D: z planes per work item of the 3-D kernels."""
        self._check(L.lib().brls_set_zchunk(self._h, int(planes)))

    set_zchunk = brls_set_zchunk

    def brls_get_zchunk(self) -> int:
        v = ctypes.c_int32()
        self._check(L.lib().brls_get_zchunk(self._h, ctypes.byref(v)))
        return v.value

    get_zchunk = brls_get_zchunk

    def brls_set_tile(self, variant: int, shots_per_block: Optional[int] = None):
        self._check(L.lib().brls_set_tile(self._h, int(variant)))
        if shots_per_block is not None:
            self._check(L.lib().brls_set_shots_per_block(
                self._h, int(shots_per_block)))

    set_tile = brls_set_tile

    def brls_get_tile(self):
        v, pb = ctypes.c_int32(), ctypes.c_int32()
        self._check(L.lib().brls_get_tile(self._h, ctypes.byref(v),
                                          ctypes.byref(pb)))
        return v.value, pb.value

    get_tile = brls_get_tile

    def brls_set_resident_grid(self, enable: bool):
        self._check(L.lib().brls_set_resident_grid(self._h, int(bool(enable))))

    set_resident_grid = brls_set_resident_grid

    def brls_get_resident_grid(self) -> bool:
        v = ctypes.c_int32()
        self._check(L.lib().brls_get_resident_grid(self._h, ctypes.byref(v)))
        return bool(v.value)

    get_resident_grid = brls_get_resident_grid

    def brls_set_tuning(self, variant: int, born_per_block: int,
                        born_resident_grid: int, adj_per_block: int,
                        adj_resident_grid: int):
        self._check(L.lib().brls_set_tuning(
            self._h, int(variant), int(born_per_block),
            int(born_resident_grid), int(adj_per_block),
            int(adj_resident_grid)))

    set_tuning = brls_set_tuning

    def brls_get_tuning(self) -> dict:
        v = [ctypes.c_int32() for _ in range(5)]
        self._check(L.lib().brls_get_tuning(self._h,
                                            *[ctypes.byref(x) for x in v]))
        return dict(variant=v[0].value, born_per_block=v[1].value,
                    born_resident_grid=v[2].value, adj_per_block=v[3].value,
                    adj_resident_grid=v[4].value)

    get_tuning = brls_get_tuning

    def brls_autotune(self) -> int:
        best = ctypes.c_int32()
        self._check(L.lib().brls_autotune(self._h, ctypes.byref(best)))
        return best.value

    autotune = brls_autotune

    def brls_kernel_timing(self, enable: bool):
        self._check(L.lib().brls_kernel_timing(self._h, int(bool(enable))))

    kernel_timing = brls_kernel_timing

    def brls_kernel_stats(self) -> dict:
        arr = (L.brls_kstat * 16)()
        n = ctypes.c_int32()
        self._check(L.lib().brls_kernel_stats(self._h, arr, 16,
                                              ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms)
                for i in range(min(n.value, 16))}

    kernel_stats = brls_kernel_stats

    def brls_memory_bytes(self) -> int:
        n = ctypes.c_int64()
        self._check(L.lib().brls_memory_bytes(self._h, ctypes.byref(n)))
        return n.value

    memory_bytes = brls_memory_bytes

    def brls_sync(self):
        self._check(L.lib().brls_sync(self._h))

    sync = brls_sync


def brls_open(ndim: int, nz: int, ny: int, nx: int, nb: int, nt_max: int,
              nrec_max: int, q_max: int, h: float, dt: float, lam: float,
              vel: np.ndarray, device: bool = False, stream=None,
              ckpt_interval: int = 0) -> Context:
    """Open a context (velocity ``vel`` [nz][ny][nx], m/s, host array).

    ``stream``: a hipStream_t as int; with ``device=True`` and no stream given,
    torch's current stream is used. ``ckpt_interval``: 0 stores the Born
    source of every step, k > 0 checkpoints the background every k steps and
    recomputes it, -1 picks k = ceil(sqrt(nt_max))."""
    g = L.brls_grid()
    g.ndim, g.nz, g.ny, g.nx, g.nb = ndim, nz, ny, nx, nb
    g.nt_max, g.nrec_max, g.q_max = nt_max, nrec_max, q_max
    g.h, g.dt, g.lambda_ = float(h), float(dt), float(lam)
    g.ckpt_interval = int(ckpt_interval)
    g.flags = L.BRLS_DEVICE_PTRS if device else 0
    if device and stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    v = np.ascontiguousarray(vel, dtype=np.float32)
    if v.size < nz * (ny if ndim == 3 else 1) * nx:
        raise ValueError(f"vel holds {v.size} values, the grid has "
                         f"{nz * (ny if ndim == 3 else 1) * nx} points")
    h_ = ctypes.c_void_p()
    rc = L.lib().brls_open(ctypes.byref(g), v.ctypes.data,
                           ctypes.c_void_p(stream) if stream else None,
                           ctypes.byref(h_))
    L.check(rc, None)
    return Context(h_, nz, ny if ndim == 3 else 1, nx, device)


def tile_variants():
    n = ctypes.c_int32()
    L.check(L.lib().brls_tile_count(ctypes.byref(n)))
    out = []
    for v in range(n.value):
        tx, tz, r, pp = (ctypes.c_int32() for _ in range(4))
        L.check(L.lib().brls_tile_info(v, ctypes.byref(tx), ctypes.byref(tz),
                                       ctypes.byref(r), ctypes.byref(pp)))
        out.append((tx.value, tz.value, r.value, pp.value))
    return out


def tile3_variants():
    n = ctypes.c_int32()
    L.check(L.lib().brls_tile3_count(ctypes.byref(n)))
    out = []
    for v in range(n.value):
        tx, ty, sb = (ctypes.c_int32() for _ in range(3))
        L.check(L.lib().brls_tile3_info(v, ctypes.byref(tx), ctypes.byref(ty),
                                        ctypes.byref(sb)))
        out.append((tx.value, ty.value, sb.value))
    return out
