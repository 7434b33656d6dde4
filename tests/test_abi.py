"""The C-ABI library loads and exports every symbol include/brrlsm.h declares
(no compute: this runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "brrlsm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(brls_[a-z_0-9]+)\s*\(", src)))


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


def test_missing_library_fails_loudly(tmp_path):
    from paper_1801_00819_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.lib(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved
