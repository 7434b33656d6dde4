"""Writes the oracle's first two windows of the 512 x 1024 streaming chain
(Q = 4) to ``stream2d_512x1024_q4_chain2.npz`` (test infrastructure: calls
only ``oracle`` and the seeded inputs of ``synth``).

The stream is the block-row recursion of the paper (block-row section,
eqs. 10-11) on uneven shots: the 512-shot streaming form of the faulted
512 x 1024 workload (apertures U{256..1024} receivers, nt in {2000, 3000,
4000}, reflectivity drifting 0.1 % per 64 shots), windows of 4 shots
sliding by 2 (shots 0-3, then 2-5: a rank-2 downdate and update), 5 damped
CG iterations per window (eq. 10), the second warm-started from the first
window's image (eq. 11).

Inputs (all seeded, all rounded to float32 before either side sees them):
  * the model, and shot i's drifted reflectivity m_i (``synth.model_at``);
  * data d_i = A_i m_i + n_i for shots 0-5, n_i Gaussian with standard
    deviation 1 % of the RMS of the clean data of these 6 shots, drawn
    shot after shot from ``numpy.random.default_rng(1101)``;
  * lambda = 1e-3 (the workload's relative damping) times a 3-step power
    estimate of ||A_w0^T A_w0|| from a seeded start (seed 2102).

The GPU test regenerates the data with ``stream_inputs`` (the same oracle
calls, bitwise) and checks the stored hash before comparing images.

Run from the repository root: ``python tests/golden/make_stream2d_chain.py
[--out PATH]`` (about 8 minutes on 16 cores, an hour on 8 busy ones).
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

OUT = os.path.join(HERE, "stream2d_512x1024_q4_chain2.npz")
NSHOTS = 512
Q = 4
SHOTS = list(range(6))
WINDOWS = [list(range(0, 4)), list(range(2, 6))]
NITER = 5
NOISE_REL = 0.01
NOISE_SEED = 1101
POWER_ITERS = 3
POWER_SEED = 2102


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def problem():
    """The 512-shot stream (its drift field depends on the shot count) and
    the oracle problem over its first six shots."""
    import oracle
    import synth
    w = synth.stream2d_512x1024(nshots=NSHOTS, Q=Q)
    grid = oracle.Grid(2, w.nz, 1, w.nx, w.nb, w.h, w.dt)
    vel = w.vel.astype(np.float32).astype(np.float64)
    prob = oracle.Problem(grid, vel, [w.shots[i] for i in SHOTS])
    return w, prob


def stream_inputs(w, prob):
    """Float32 data with noise of shots 0-5 ([nt_i][nrec_i] arrays, each
    from its own drifted model) and the sha256 of their bytes."""
    import synth
    clean = [prob.born_shot(k, synth.model_at(w, i).astype(np.float32)
                            .astype(np.float64))
             for k, i in enumerate(SHOTS)]
    allv = np.concatenate([c.ravel() for c in clean])
    sigma = NOISE_REL * float(np.sqrt(np.mean(allv * allv)))
    r = np.random.default_rng(NOISE_SEED)
    data = [np.ascontiguousarray(
        (c + sigma * r.standard_normal(c.shape)).astype(np.float32))
        for c in clean]
    h = hashlib.sha256()
    for d in data:
        h.update(d.tobytes())
    return data, h.hexdigest()


class Progress:
    """The oracle problem, logging each window product it computes."""

    def __init__(self, prob, name):
        self.prob, self.name, self.calls = prob, name, 0
        self.grid = prob.grid

    def born(self, m, idx):
        self.calls += 1
        log(f"{self.name}: product {self.calls} (A)")
        return self.prob.born(m, idx)

    def adjoint(self, r, idx):
        log(f"{self.name}: product {self.calls} (A^T)")
        return self.prob.adjoint(r, idx)


def main(argv=None):
    import oracle
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args(argv)
    w, prob = problem()
    t = time.time()
    data, digest = stream_inputs(w, prob)
    log(f"data of shots {SHOTS} (nt {[w.shots[i].nt for i in SHOTS]}, "
        f"receivers {[w.shots[i].nrec for i in SHOTS]}) in "
        f"{time.time() - t:.0f}s, sha256 {digest[:16]}")
    d64 = [d.astype(np.float64) for d in data]
    t = time.time()
    # the oracle problem's shot k is the stream's shot SHOTS[k] = k
    nrm = oracle.power_norm(Progress(prob, "power"), WINDOWS[0], POWER_ITERS,
                            seed=POWER_SEED)
    lam = w.lam_rel * nrm
    log(f"power estimate {nrm:.6e} in {time.time() - t:.0f}s")
    m = None
    images, stats = [], []
    for k, win in enumerate(WINDOWS):
        t = time.time()
        res = oracle.cgls(Progress(prob, f"window {k}"), win,
                          [d64[i] for i in win], lam, NITER, m0=m)
        m = res.m
        images.append(m.astype(np.float32))
        stats.append({"iters": res.iters, "s0_norm": res.s0_norm,
                      "s_norms": res.s_norms, "r_norms": res.r_norms})
        log(f"window {k}: {res.iters} iterations in {time.time() - t:.0f}s, "
            f"||s|| {res.s0_norm:.4e} -> {res.s_norms[-1]:.4e}")
    np.savez(a.out, images=np.stack(images), lam=np.float64(lam),
             norm=np.float64(nrm), data_sha256=np.array(digest),
             stats=np.array(json.dumps(stats)))
    log(f"wrote {a.out}")


if __name__ == "__main__":
    main()
