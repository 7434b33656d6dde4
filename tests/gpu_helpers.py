"""Helpers shared by the GPU tests: open a library context for a synthetic
workload and run the oracle on exactly the same (float32-rounded) inputs."""
import numpy as np

import oracle
import synth


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


def vel32(w):
    return f32(w.vel)


def oracle_problem(w, shots=None):
    """Oracle on the velocity the library sees (rounded to float32)."""
    grid = oracle.Grid(w.ndim, w.nz, w.ny, w.nx, w.nb, w.h, w.dt)
    v = vel32(w).astype(np.float64)
    return oracle.Problem(grid, v, w.shots if shots is None else shots)


def open_ctx(w, lam=0.0, q_max=None, nt_max=None, nrec_max=None,
             device=False, ckpt_interval=0):
    import paper_1801_00819_amd as P
    q_max = q_max or len(w.shots)
    nt_max = nt_max or max(s.nt for s in w.shots)
    nrec_max = nrec_max or max(s.nrec for s in w.shots)
    return P.brls_open(w.ndim, w.nz, w.ny, w.nx, w.nb, nt_max, nrec_max,
                       q_max, w.h, w.dt, lam, vel32(w), device=device,
                       ckpt_interval=ckpt_interval)


def add_shot(ctx, w, i, data=None, sid=None):
    s = w.shots[i]
    ctx.update(i if sid is None else sid, s.src, s.rec, s.nt, s.f0,
               None if data is None else f32(data))


def split(w, idx, packed):
    out, off = [], 0
    for i in idx:
        s = w.shots[i]
        n = s.nt * s.nrec
        out.append(np.asarray(packed[off:off + n]).reshape(s.nt, s.nrec))
        off += n
    return out


def ragged2d():
    """A model spanning several tiles with ragged edges, a sponge width not
    a multiple of 32, shots of different length and receiver sets (one
    receiver position repeated)."""
    nz, nx, nb = 77, 133, 13
    r = np.random.default_rng(21)
    z = np.arange(nz, dtype=np.float64)[:, None]
    vel = 1700.0 + 900.0 * z / (nz - 1) + 80.0 * r.uniform(-1, 1, (nz, nx))
    m = r.uniform(-0.1, 0.1, (nz, nx)) * (r.uniform(size=(nz, nx)) < 0.3)
    shots = []
    specs = [((2, 0, 10), 300, 25.0), ((5, 0, 70), 260, 22.0),
             ((3, 0, 131), 311, 28.0)]
    for i, (src, nt, f0) in enumerate(specs):
        xs = np.sort(r.choice(nx, size=40 + 7 * i, replace=False))
        rec = np.stack([np.full(xs.size, 1 + i), np.zeros(xs.size, int), xs],
                       1).astype(np.int32)
        if i == 1:  # a repeated receiver position
            rec = np.concatenate([rec, rec[3:4]], 0)
        deep = np.array([[nz - 1, 0, 5], [40, 0, nx - 1]], dtype=np.int32)
        rec = np.concatenate([rec, deep], 0)
        shots.append(synth.Shot(i, src, rec, nt, f0))
    return synth.Workload("ragged2d", -1, 2, nz, 1, nx, nb, 10.0, 1e-3, 311,
                          25.0, vel[:, None, :].copy(), m[:, None, :].copy(),
                          shots, Q=3, S=1, niter=6, lam_rel=0.01)
