"""The 512 x 1024 faulted workload at full size against the oracle, through
the C ABI, in the launch configuration the benchmark times (graph mode, the
default launch choice): the operators over the whole first window (8 shots,
nt = 3000, 1024 receivers each) and the chain's first two windows (20 CG
iterations each, warm-started; the paper's block-row recursion, eqs. 10-11,
Fig. 2d).

The oracle's images of the chain are stored in
``tests/golden/faulted2d_512x1024_chain2.npz`` by
``tests/golden/make_faulted2d_chain.py`` (hours of oracle work); the data
both sides use are regenerated here by the same oracle calls and checked
against the hash stored with the images.

Truncated damped CG is sensitive to rounding at this size: the oracle's own
20th iterate moves by 5.5 % when only its operator operands and results
are rounded to float32 (the stored ``images_r32``), from about the 8th
iteration on. So the chain is checked three ways: the 7th iterate of the
first window, before that sensitivity sets in, to 1e-4; the first window's
20th iterate against the oracle's float32-interface run, to 1e-4; and the
20-iteration images and data misfits of both windows against the FP64 run
within twice its distance from the float32-interface run.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

from gpu_helpers import f32, open_ctx, rel, split

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
IMG_TOL = 1e-4
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "faulted2d_512x1024_chain2.npz")


def _recipe():
    spec = importlib.util.spec_from_file_location(
        "make_faulted2d_chain",
        os.path.join(HERE, "golden", "make_faulted2d_chain.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def inputs():
    """Workload, oracle problem over shots 0-11, their clean oracle data,
    the float32 data with noise and its hash (about a minute of oracle
    work on the host)."""
    mk = _recipe()
    w, prob = mk.problem()
    print("oracle: data of shots 0-11 at full size", flush=True)
    clean, data, digest = mk.window_inputs(prob, w.m_true.astype(np.float32))
    return mk, w, prob, clean, data, digest


def _bench_tuning():
    import bench
    return bench.DEFAULT_TUNING


def _window_ctx(w, lam=0.0):
    ctx = open_ctx(w, lam=lam, q_max=8)
    ctx.set_tuning(*_bench_tuning())
    return ctx


@pytest.mark.timeout(900)
def test_full_size_born_every_shot_matches_oracle(inputs):
    """A m_true over the whole first window: each of the 8 shots' data
    against the oracle's."""
    mk, w, prob, clean, data, _ = inputs
    idx = mk.WINDOWS[0]
    print("512x1024 born, 8-shot window, graph mode, bench launch choice",
          flush=True)
    ctx = _window_ctx(w)
    for i in idx:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
    got = split(w, idx, ctx.apply_born(f32(w.m_true)))
    ctx.close()
    errs = [rel(got[k], clean[i]) for k, i in enumerate(idx)]
    print("born per shot: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= OP_TOL


@pytest.mark.timeout(900)
def test_full_size_adjoint_of_window_matches_oracle(inputs):
    """A^T d over the whole first window, d the observed data of all 8
    shots (nonzero everywhere): the library's image, summed over the shot
    groups in float64, against the oracle's 8-shot sum."""
    mk, w, prob, clean, data, _ = inputs
    idx = mk.WINDOWS[0]
    print("512x1024 adjoint, 8-shot window, graph mode, bench launch choice",
          flush=True)
    ctx = _window_ctx(w)
    for i in idx:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
    got = ctx.apply_adjoint(np.concatenate([data[i].ravel() for i in idx]))
    ctx.close()
    print("oracle: adjoint of 8 shots", flush=True)
    want = prob.adjoint([data[i].astype(np.float64) for i in idx], idx)
    e = rel(got, want)
    print(f"adjoint of the window: {e:.2e}")
    assert e <= OP_TOL


def _golden(digest):
    if not os.path.exists(GOLDEN):
        pytest.skip("oracle images not generated "
                    "(tests/golden/make_faulted2d_chain.py)")
    g = np.load(GOLDEN, allow_pickle=False)
    assert str(g["data_sha256"]) == digest, \
        "regenerated data differ from the ones the oracle images used"
    return g


def _load_window(ctx, w, data, win, held):
    for i in list(held):
        if i not in win:
            ctx.downdate(i)
            held.remove(i)
    for i in win:
        if i not in held:
            s = w.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
            held.append(i)


@pytest.mark.timeout(900)
def test_full_size_early_iterate_matches_oracle(inputs):
    """The first window from a zero image, 7 CG iterations: the image
    against the oracle's 7th iterate and ||A^T r - lambda m|| at every
    iteration against the oracle's, 1e-4."""
    mk, w, prob, clean, data, digest = inputs
    g = _golden(digest)
    if "early" not in g.files:
        pytest.skip("oracle's early iterate not stored")
    k = int(g["early_k"])
    want = np.array(json.loads(str(g["early_stats"]))["s_norms"])
    ctx = _window_ctx(w, float(g["lam"]))
    _load_window(ctx, w, data, mk.WINDOWS[0], [])
    st = ctx.solve_window(k)
    assert st["iters"] == k
    e = rel(ctx.image(), g["early"])
    got = np.concatenate([[st["s0_norm"]], ctx.solve_history()["s_norm"]])
    ctx.close()
    es = np.abs(got / want - 1)
    print(f"iterate {k}: image vs oracle {e:.2e}; ||s|| per iteration vs "
          "oracle: " + " ".join(f"{x:.1e}" for x in es))
    assert e <= IMG_TOL and es.max() <= IMG_TOL


@pytest.mark.timeout(900)
def test_full_size_chain_matches_oracle(inputs):
    """The chain's first windows (8 shots sliding by 4, 20 iterations each,
    the second warm-started from the first's image) against the oracle.
    Window 0 against the oracle's run with float32 operator operands and
    results (the library's interface precision): image and data misfit
    ||d_w - A_w m|| to 1e-4. Every window against the FP64 run: image and
    misfit within max(1e-4, 2 x the distance between the oracle's FP64 and
    float32-interface runs of window 0), the truncated solve's measured
    sensitivity to that rounding."""
    mk, w, prob, clean, data, digest = inputs
    g = _golden(digest)
    if "images_r32" not in g.files:
        pytest.skip("oracle's float32-interface chain not stored")
    lam = float(g["lam"])
    images, im32 = g["images"], g["images_r32"]
    st64 = json.loads(str(g["stats"]))
    st32 = json.loads(str(g["stats_r32"]))
    img_bound = max(IMG_TOL, 2.0 * rel(im32[0], images[0]))
    r64, r32 = st64[0]["r_norms"][-1], st32[0]["r_norms"][-1]
    mis_bound = max(IMG_TOL, 2.0 * abs(r32 - r64) / r64)
    ctx = _window_ctx(w, lam)
    held = []
    fails = []
    for k in range(images.shape[0]):
        _load_window(ctx, w, data, mk.WINDOWS[k], held)
        st = ctx.solve_window(mk.NITER)
        assert st["iters"] == mk.NITER
        img = ctx.image()
        e = rel(img, images[k])
        want_r = st64[k]["r_norms"][-1]
        er = abs(st["r_norm"] - want_r) / want_r
        print(f"window {k}: vs FP64 oracle image {e:.2e} (bound "
              f"{img_bound:.2e}), misfit {st['r_norm']:.6e} vs {want_r:.6e}"
              f" {er:.2e} (bound {mis_bound:.2e})", flush=True)
        if e > img_bound or er > mis_bound:
            fails.append(k)
        if k < im32.shape[0]:
            e32 = rel(img, im32[k])
            w32 = st32[k]["r_norms"][-1]
            er32 = abs(st["r_norm"] - w32) / w32
            print(f"window {k}: vs float32-interface oracle image {e32:.2e}, "
                  f"misfit {er32:.2e}", flush=True)
            if e32 > IMG_TOL or er32 > IMG_TOL:
                fails.append(k)
    ctx.close()
    assert not fails, f"windows {fails} outside the bounds"


STREAM_GOLDEN = os.path.join(HERE, "golden", "stream2d_512x1024_q4_chain2.npz")


@pytest.mark.timeout(900)
def test_full_size_stream_chain_matches_oracle():
    """The 512-shot streaming form at full size, windows of 4 sliding by 2
    (shots 0-3, then 2-5: ragged nt 2000 / 3000 and 304 .. 1022 receivers,
    each shot's data from its own drifted model), 5 iterations per window
    warm-started, in the bench's launch choice: both images against the
    oracle's stored ones (``tests/golden/make_stream2d_chain.py``), 1e-4."""
    spec = importlib.util.spec_from_file_location(
        "make_stream2d_chain",
        os.path.join(HERE, "golden", "make_stream2d_chain.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    w, prob = mk.problem()
    print("oracle: data of the stream's shots 0-5 at full size", flush=True)
    data, digest = mk.stream_inputs(w, prob)
    g = np.load(STREAM_GOLDEN, allow_pickle=False)
    assert str(g["data_sha256"]) == digest, \
        "regenerated data differ from the ones the oracle images used"
    ctx = open_ctx(w, lam=float(g["lam"]), q_max=mk.Q)
    ctx.set_tuning(*_bench_tuning())
    held, errs = [], []
    for k, win in enumerate(mk.WINDOWS):
        _load_window(ctx, w, data, win, held)
        st = ctx.solve_window(mk.NITER)
        assert st["iters"] == mk.NITER
        errs.append(rel(ctx.image(), g["images"][k]))
        print(f"stream window {k} (shots {win}): image vs oracle "
              f"{errs[-1]:.2e}", flush=True)
    ctx.close()
    assert max(errs) <= IMG_TOL
