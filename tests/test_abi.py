"""The C-ABI library loads and exports every symbol include/*.h declare (no
compute: this runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    inc = os.path.join(ROOT, "include")
    names = set()
    for f in sorted(os.listdir(inc)):
        if not f.endswith(".h"):
            continue
        src = open(os.path.join(inc, f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(brls_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_verbs():
    names = _declared()
    for verb in ("brls_open", "brls_update", "brls_downdate",
                 "brls_solve_window", "brls_image", "brls_close",
                 "brls_apply_born", "brls_apply_adjoint", "brls_last_error"):
        assert verb in names


def test_library_exports_every_declared_symbol():
    from paper_1801_00819_amd import _lib
    L = _lib.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing
    assert sorted(n for n, _, _ in _lib.SIGNATURES) == _declared()


def test_open_rejects_bad_grid_without_touching_the_device():
    import numpy as np
    import paper_1801_00819_amd as P
    with pytest.raises(P.BrlsError) as e:
        P.brls_open(2, 0, 1, 8, 4, 10, 4, 1, 10.0, 1e-3, 0.0,
                    np.ones((1, 8), np.float32))
    assert e.value.code == -1 and "invalid grid" in str(e.value)
    with pytest.raises(P.BrlsError) as e:
        P.brls_open(4, 8, 8, 8, 4, 10, 4, 1, 10.0, 1e-3, 0.0,
                    np.ones((8, 8, 8), np.float32))
    assert e.value.code == -1 and "ndim" in str(e.value)


def _open_raw(**kw):
    """brls_open through the C ABI with a one-value velocity buffer: every
    case here must be rejected before the library reads the velocity."""
    import ctypes
    import numpy as np
    from paper_1801_00819_amd import _lib
    g = _lib.brls_grid()
    g.ndim, g.nz, g.ny, g.nx, g.nb = 2, 64, 1, 64, 20
    g.nt_max, g.nrec_max, g.q_max = 100, 16, 2
    g.h, g.dt, g.lambda_ = 10.0, 1e-3, 0.0
    for k, v in kw.items():
        setattr(g, k, v)
    vel = np.ones(1, np.float32)
    h = ctypes.c_void_p()
    rc = _lib.lib().brls_open(ctypes.byref(g), vel.ctypes.data, None,
                              ctypes.byref(h))
    return rc, _lib.lib().brls_last_error(None).decode()


def test_open_rejects_grids_past_the_kernels_offsets():
    """The kernels address a wavefield with 32-bit byte offsets: a padded
    2-D grid of 2^29 points or more (3-D: 2^30) is refused, as is a shot
    segment of more than 2^30 samples, before the device is touched."""
    # 2-D model just under 2^29 points whose padded grid is over it
    rc, msg = _open_raw(nz=16384, nx=32760, nb=40)
    assert rc == -1 and "padded grid" in msg
    rc, msg = _open_raw(ndim=3, nz=1024, ny=1024, nx=1000, nb=20)
    assert rc == -1 and "padded grid" in msg
    rc, msg = _open_raw(nt_max=1 << 16, nrec_max=(1 << 14) + 1)
    assert rc == -1 and "2^30" in msg


def test_bindings_check_buffer_sizes():
    """Host-side guards of the Python binding: a velocity array smaller than
    the grid, and buffers smaller than a call needs or of another dtype,
    are refused before the library sees them."""
    import numpy as np
    import paper_1801_00819_amd as P
    from paper_1801_00819_amd import _ptr
    from paper_1801_00819_amd.ssf import brls_ssf_open
    with pytest.raises(ValueError, match="vel holds"):
        P.brls_open(2, 64, 1, 64, 20, 100, 16, 2, 10.0, 1e-3, 0.0,
                    np.ones((64, 63), np.float32))
    with pytest.raises(ValueError, match="vel holds"):
        brls_ssf_open(24, 64, 10.0, 10.0, 256, 1e-3, 5.0, 40.0, 8, 8, 2,
                      0.0, np.ones((24, 32), np.float32))
    a = np.zeros(10, np.float32)
    assert _ptr(a, False, 10).value == a.ctypes.data
    with pytest.raises(ValueError, match="needs 11"):
        _ptr(a, False, 11)
    with pytest.raises(TypeError):
        _ptr(np.zeros(10, np.float64), False, 10)


def test_missing_library_fails_loudly(tmp_path):
    from paper_1801_00819_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.lib(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def test_split_step_header_declares_its_verbs():
    names = _declared()
    for verb in ("brls_ssf_open", "brls_ssf_update", "brls_ssf_downdate",
                 "brls_ssf_solve_window", "brls_ssf_apply_born",
                 "brls_ssf_apply_adjoint", "brls_ssf_image",
                 "brls_ssf_close", "brls_ssf_last_error"):
        assert verb in names


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=96), "power of two"),
    (dict(nx=4096), "power of two"),
    (dict(ntap=32), "ntap"),
    (dict(fmin=60.0, fmax=50.0), "band"),
    (dict(fmax=200.0), "band"),
    (dict(fmin=20.1, fmax=20.2), "no DFT frequency"),
    (dict(q_max=0), "q_max"),
    (dict(nt=1 << 27, nrec_max=9), "2^30"),
])
def test_split_step_open_rejects_bad_grids(kw, msg):
    import numpy as np
    from paper_1801_00819_amd import BrlsError
    from paper_1801_00819_amd.ssf import brls_ssf_open
    a = dict(nz=8, nx=64, dx=10.0, dz=10.0, nt=256, dt=4e-3, fmin=4.0,
             fmax=40.0, ntap=8, nrec_max=8, q_max=2, lam=0.0)
    a.update(kw)
    with pytest.raises(BrlsError) as e:
        brls_ssf_open(**a, vel=np.full((a["nz"], a["nx"]), 2000.0,
                                       np.float32))
    assert e.value.code == -1 and msg in str(e.value)
