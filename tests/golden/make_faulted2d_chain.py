"""Writes the oracle's first two windows of the 512 x 1024 faulted chain to
``faulted2d_512x1024_chain2.npz`` (test infrastructure: calls only
``oracle`` and the seeded inputs of ``synth``).

The chain is the block-row recursion of the paper (block-row section,
eqs. 10-11): windows of 8 shots sliding by 4 (shots 0-7, then 4-11), each
window solved by 20 iterations of damped CG (eq. 10, the windowed eq. 3),
the second warm-started from the first window's image (eq. 11).

Inputs (all seeded, all rounded to float32 before either side sees them):
  * the 512 x 1024 faulted model's velocity and reflectivity;
  * data d_i = A_i m_true + n_i for shots 0-11, n_i Gaussian with standard
    deviation 1 % of the RMS of the clean data of these 12 shots, drawn
    shot after shot from ``numpy.random.default_rng(1001)``;
  * lambda = 1e-3 (the workload's relative damping) times a 3-step power
    estimate of ||A_w0^T A_w0|| from a seeded start (seed 2002).

Stored arrays:
  * ``images`` [windows][nz][nx]: the oracle's image after each window
    (FP64 CG, rounded to float32 for storage), ``stats`` its norms;
  * ``early`` [nz][nx], ``early_k``, ``early_stats``: window 0's iterate
    after EARLY = 7 iterations, before the truncated CG becomes sensitive
    to rounding (below);
  * ``images_r32``, ``stats_r32``: the same chain with every operator
    operand and result rounded to float32 (the library's interface
    precision; the window's adjoint summed in FP64 and rounded once). At
    this size the 20-iteration iterate of damped CG moves by percents
    under that rounding alone: a search direction with a small component
    along the largest-curvature directions (the source footprint) is
    amplified by hundreds per iteration from about the 8th iteration on.
    The spread between ``images`` and ``images_r32`` measures that
    sensitivity, which bounds how closely any float32-interface solver can
    follow the FP64 iterate.

The GPU test regenerates the data with ``window_inputs`` (the same oracle
calls, bitwise) and checks the stored hash before comparing images.

Run from the repository root: ``python tests/golden/make_faulted2d_chain.py
[--windows N] [--round32 N] [--early] [--partials DIR]`` (hours of oracle
work on 8 cores per window). Each finished piece is kept as a partial file
(``.w<k>.npy``, ``.r32.w<k>.npy``, ``.early<K>.npy``, each with a ``.json``
of norms) in the partials folder (default: next to the output), so an
interrupted run resumes; the output is rewritten from every partial found.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "faulted2d_512x1024_chain2.npz")
SHOTS = list(range(12))
WINDOWS = [list(range(0, 8)), list(range(4, 12))]
NITER = 20
EARLY = 7
NOISE_REL = 0.01
NOISE_SEED = 1001
POWER_ITERS = 3
POWER_SEED = 2002


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def problem():
    import oracle
    import synth
    w = synth.faulted2d_512x1024()
    grid = oracle.Grid(2, w.nz, 1, w.nx, w.nb, w.h, w.dt)
    vel = w.vel.astype(np.float32).astype(np.float64)
    prob = oracle.Problem(grid, vel, [w.shots[i] for i in SHOTS])
    return w, prob


def window_inputs(prob, m_true32):
    """Clean float64 data A_i m_true of shots 0-11, the float32 data with
    noise (lists of [nt][nrec] arrays) and the sha256 of the latter's
    bytes."""
    clean = [prob.born_shot(i, m_true32.astype(np.float64))
             for i in range(len(SHOTS))]
    allv = np.concatenate([c.ravel() for c in clean])
    sigma = NOISE_REL * float(np.sqrt(np.mean(allv * allv)))
    r = np.random.default_rng(NOISE_SEED)
    data = [np.ascontiguousarray(
        (c + sigma * r.standard_normal(c.shape)).astype(np.float32))
        for c in clean]
    h = hashlib.sha256()
    for d in data:
        h.update(d.tobytes())
    return clean, data, h.hexdigest()


def _r32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(
        np.float64)


class Round32:
    """The oracle's window operators with operands and results rounded to
    float32: A m of each shot from float32 m, rounded; A^T r summed over
    the window's shots (slot order, FP64) from float32 r, rounded once."""

    def __init__(self, prob):
        self.prob = prob
        self.grid = prob.grid

    def born(self, m, idx):
        m32 = _r32(m)
        return [_r32(self.prob.born_shot(i, m32)) for i in idx]

    def adjoint(self, r, idx):
        g = np.zeros(self.grid.model_shape)
        for ri, i in zip(r, idx):
            g += self.prob.adjoint_shot(i, _r32(ri))
        return _r32(g)


class Progress:
    """Operators ``ops`` that log each window product they compute."""

    def __init__(self, ops, name):
        self.ops, self.name, self.calls = ops, name, 0
        self.grid = ops.grid

    def born(self, m, idx):
        self.calls += 1
        log(f"{self.name}: product {self.calls} (A)")
        return self.ops.born(m, idx)

    def adjoint(self, r, idx):
        log(f"{self.name}: product {self.calls} (A^T)")
        return self.ops.adjoint(r, idx)


def _stats(res):
    return {"iters": res.iters, "s0_norm": res.s0_norm,
            "s_norms": res.s_norms, "r_norms": res.r_norms}


def _save(path, m, st):
    np.save(path, m)
    with open(path + ".json", "w") as f:
        json.dump(st, f)


def _load(path):
    with open(path + ".json") as f:
        return np.load(path), json.load(f)


def _meta(part_dir, digest, prob):
    """lambda and the power estimate: from the partials folder, else from
    an output written with the same data, else computed."""
    import oracle
    import synth
    path = os.path.join(part_dir, os.path.basename(OUT) + ".meta.json")
    if os.path.exists(path):
        with open(path) as f:
            meta = json.load(f)
        if meta.get("data_sha256") != digest:
            raise SystemExit("stored partial run used other data")
        return meta
    meta = None
    if os.path.exists(OUT):
        g = np.load(OUT, allow_pickle=False)
        if str(g["data_sha256"]) == digest:
            meta = {"data_sha256": digest, "norm": float(g["norm"]),
                    "lambda": float(g["lam"])}
    if meta is None:
        t = time.time()
        nrm = oracle.power_norm(prob, WINDOWS[0], POWER_ITERS,
                                seed=POWER_SEED)
        meta = {"data_sha256": digest, "norm": nrm,
                "lambda": synth.faulted2d_512x1024().lam_rel * nrm}
        log(f"power estimate {nrm:.6e} in {time.time() - t:.0f}s")
    with open(path, "w") as f:
        json.dump(meta, f)
    return meta


def _chain(ops, d64, lam, nwin, prefix):
    """Windows 0 .. nwin-1 of the chain with operators ``ops``, each kept
    as a partial file ``prefix + w<k>.npy``."""
    import oracle
    m = None
    for k, win in enumerate(WINDOWS[:nwin]):
        part = f"{prefix}w{k}.npy"
        if os.path.exists(part):
            m, _ = _load(part)
            log(f"{os.path.basename(part)}: resumed")
            continue
        t = time.time()
        res = oracle.cgls(Progress(ops, os.path.basename(part)), win,
                          [d64[i] for i in win], lam, NITER, m0=m)
        m = res.m
        _save(part, m, _stats(res))
        log(f"{os.path.basename(part)}: {res.iters} iterations in "
            f"{time.time() - t:.0f}s, ||s|| {res.s0_norm:.4e} -> "
            f"{res.s_norms[-1]:.4e}")


def _collect(prefix, nwin):
    images, stats = [], []
    for k in range(nwin):
        part = f"{prefix}w{k}.npy"
        if not os.path.exists(part):
            break
        m, st = _load(part)
        images.append(m.astype(np.float32))
        stats.append(st)
    return images, stats


def main(argv=None):
    import oracle
    ap = argparse.ArgumentParser()
    ap.add_argument("--windows", type=int, default=len(WINDOWS),
                    help="FP64 chain windows to compute")
    ap.add_argument("--round32", type=int, default=0,
                    help="float32-interface chain windows to compute")
    ap.add_argument("--early", action="store_true",
                    help=f"window 0's iterate after {EARLY} iterations")
    ap.add_argument("--partials", default=HERE)
    a = ap.parse_args(argv)
    os.makedirs(a.partials, exist_ok=True)
    base = os.path.join(a.partials, os.path.basename(OUT))
    w, prob = problem()
    t = time.time()
    _, data, digest = window_inputs(prob, w.m_true.astype(np.float32))
    log(f"data of {len(SHOTS)} shots in {time.time() - t:.0f}s, sha256 "
        f"{digest[:16]}")
    d64 = [d.astype(np.float64) for d in data]
    meta = _meta(a.partials, digest, prob)
    lam = meta["lambda"]
    if a.early and not os.path.exists(f"{base}.early{EARLY}.npy"):
        t = time.time()
        win = WINDOWS[0]
        res = oracle.cgls(Progress(prob, f"early{EARLY}"), win,
                           [d64[i] for i in win], lam, EARLY)
        _save(f"{base}.early{EARLY}.npy", res.m, _stats(res))
        log(f"window 0 after {EARLY} iterations in {time.time() - t:.0f}s")
    _chain(prob, d64, lam, a.windows, f"{base}.")
    if a.round32:
        _chain(Round32(prob), d64, lam, a.round32, f"{base}.r32.")
    images, stats = _collect(f"{base}.", len(WINDOWS))
    if not images:
        log("no finished window: output not written")
        return
    out = {"images": np.stack(images), "lam": np.float64(lam),
           "norm": np.float64(meta["norm"]),
           "data_sha256": np.array(digest),
           "stats": np.array(json.dumps(stats))}
    r32, st32 = _collect(f"{base}.r32.", len(WINDOWS))
    if r32:
        out["images_r32"] = np.stack(r32)
        out["stats_r32"] = np.array(json.dumps(st32))
    if os.path.exists(f"{base}.early{EARLY}.npy"):
        m, st = _load(f"{base}.early{EARLY}.npy")
        out["early"] = m.astype(np.float32)
        out["early_k"] = np.int64(EARLY)
        out["early_stats"] = np.array(json.dumps(st))
    target = OUT if a.partials == HERE else base
    np.savez(target, **out)
    log(f"wrote {target}: {len(images)} window(s), {len(r32)} float32-"
        f"interface window(s), early iterate "
        f"{'yes' if 'early' in out else 'no'}")


if __name__ == "__main__":
    main()
