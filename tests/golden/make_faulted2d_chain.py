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

The GPU test regenerates the data with ``window_inputs`` (the same oracle
calls, bitwise) and checks the stored hash before comparing images.

Run from the repository root: ``python tests/golden/make_faulted2d_chain.py
[nwindows]`` (about 4 hours on 8 cores for both windows). It keeps the float64 image of each finished
window next to the output (``.w<k>.npy``), so an interrupted run resumes
after the last finished window.
"""
from __future__ import annotations

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


def main(nwin=len(WINDOWS)):
    import oracle
    w, prob = problem()
    m_true32 = w.m_true.astype(np.float32)
    t = time.time()
    _, data, digest = window_inputs(prob, m_true32)
    log(f"data of {len(SHOTS)} shots in {time.time() - t:.0f}s, sha256 "
        f"{digest[:16]}")
    d64 = [d.astype(np.float64) for d in data]
    meta_path = OUT + ".meta.json"
    meta = {}
    if os.path.exists(meta_path):
        with open(meta_path) as f:
            meta = json.load(f)
        if meta.get("data_sha256") != digest:
            raise SystemExit("stored partial run used other data")
    if "lambda" not in meta:
        t = time.time()
        nrm = oracle.power_norm(prob, WINDOWS[0], POWER_ITERS,
                                seed=POWER_SEED)
        meta = {"data_sha256": digest, "norm": nrm,
                "lambda": w.lam_rel * nrm}
        with open(meta_path, "w") as f:
            json.dump(meta, f)
        log(f"power estimate {nrm:.6e} in {time.time() - t:.0f}s")
    lam = meta["lambda"]
    m = None
    images, stats = [], []
    for k, win in enumerate(WINDOWS[:nwin]):
        part = f"{OUT}.w{k}.npy"
        if os.path.exists(part):
            m = np.load(part)
            with open(part + ".json") as f:
                stats.append(json.load(f))
            images.append(m.astype(np.float32))
            log(f"window {k}: resumed")
            continue
        t = time.time()
        res = oracle.cgls(prob, win, [d64[i] for i in win], lam, NITER,
                          m0=m)
        m = res.m
        np.save(part, m)
        st = {"iters": res.iters, "s0_norm": res.s0_norm,
              "s_norms": res.s_norms, "r_norms": res.r_norms}
        with open(part + ".json", "w") as f:
            json.dump(st, f)
        stats.append(st)
        images.append(m.astype(np.float32))
        log(f"window {k}: {res.iters} iterations in {time.time() - t:.0f}s, "
            f"||s|| {res.s0_norm:.4e} -> {res.s_norms[-1]:.4e}")
    np.savez(OUT, images=np.stack(images), lam=np.float64(lam),
             norm=np.float64(meta["norm"]),
             data_sha256=np.array(digest),
             stats=np.array(json.dumps(stats)))
    log(f"wrote {OUT}")


if __name__ == "__main__":
    # an optional argument stops after that many windows (the output then
    # holds only their images)
    main(int(sys.argv[1]) if len(sys.argv) > 1 else len(WINDOWS))
