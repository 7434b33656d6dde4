"""Benchmark: block-row recursive least-squares migration, one MI355X.

Workload (the paper's method on the faulted 2-D model): 512 x 1024 grid,
h = 5 m, 40-cell sponge (592 x 1104 padded), 64 shots 80 m apart with 1024
receivers each, nt = 3000 at dt = 0.5 ms, 20 Hz Ricker; windows of Q = 8
shots sliding by S = 4; 20 CG iterations per window; lambda = 1e-3 relative
to ||A_w^T A_w|| of the first window.

One step = one window of the chain: downdate the S oldest shots, update the
S new ones (data already resident in device memory), build their background
wavefields, run the warm-started CG solve, copy the image out.

value = Born + adjoint grid-point updates per second over the timed steps
(every propagated Born-field and adjoint-field point per time step and shot,
background propagation not counted, time of everything in the step counted).

Prints one JSON line. Also reports the roofline of the dominant kernel
(event-timed in a separate pass), the seconds per window solved to a fixed
CG residual (batched graph launches and plain per-shot launches at the same
residual), and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# launch choice used unless --autotune is given (and by the counter runs):
# tile variant, Born shots per block and grid shape, adjoint shots per block
# and grid shape -- the fastest in a sweep of all choices on this workload
# (segment-marching wavefronts taking two time steps per launch over
# 16-row segments, blocks of four wavefronts marching the four shots of a
# group on one segment -- the adjoint's summing their image contributions
# in LDS -- on a grid of resident blocks whose work items run strips
# fastest)
DEFAULT_TUNING = (24, 4, 5, 4, 5)
# with checkpointed backgrounds (no stored Born sources): the fastest
# one-step choice
DEFAULT_TUNING_CKPT = (16, 1, 0, 4, 2)
# kernel behind each tile kind (the fourth number of a tile variant)
KERNEL_NAME = {0: "k_step2d", 1: "k_step2d", 2: "k_march2d", 3: "k_march2t",
               4: "k_march2s"}
DEFAULT_TILE3 = 0

# HBM bytes per launch of the 2-D step kernel under DEFAULT_TUNING, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs of `bench.py --ops-only`, scaled
# by the same counters on a 512 MiB copy (fetch x 2.000, write x 1.000).
# Valid only for the kernel sources they were taken on: reported as null
# once the 2-D kernel sources hash differently.
TRAFFIC_2D = {
    "sources_sha256_16": "4538816f1336829a",
    "born": 2 * 61555.1 * 1024 + 45267.7 * 1024,
    "adjoint": 2 * 58025.3 * 1024 + 52137.5 * 1024,
}


# Counter-measured HBM bytes per launch of the split-step kernels on the
# 5-shot window of the 256 x 1024 workload (rocprofv3 FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000, the factors a 512 MiB device copy reads in the same
# program), valid for the kernel sources of that hash.
TRAFFIC_SSF = {
    "sources_sha256_16": "9b68de91c98c97be",
    "born": 2 * 1133856.9 * 1024 + 566.2 * 1024,
    "adjoint": 2 * 1538643.5 * 1024 + 773120.0 * 1024,
}


def kernel_sources_hash(files=("stencil2d.hip", "march2d.hip", "march2t.hip",
                               "march2s.hip",
                               "march_common.h", "devutil.h", "layout.h")):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1801_00819_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, tuning):
    """Counter-measured HBM bytes per launch, or None when the kernel or
    the launch choice differs from the one the counters were taken on."""
    t = (tuning["variant"], tuning["born_per_block"],
         tuning["born_resident_grid"], tuning["adj_per_block"],
         tuning["adj_resident_grid"])
    if t != DEFAULT_TUNING or \
            kernel_sources_hash() != TRAFFIC_2D["sources_sha256_16"]:
        return None
    return int(TRAFFIC_2D[kind])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--stream-shots", type=int, default=128,
                    help="stream workload: shots taken from the 512")
    ap.add_argument("--stream-iters", type=int, default=5,
                    help="stream workload: CG iterations per window")
    ap.add_argument("--stream-forgetting", type=float, default=0.8,
                    help="stream workload: forgetting factor of the "
                         "weighted-window run (shot weights beta^age)")
    ap.add_argument("--no-stream-options", action="store_true",
                    help="stream workload: skip the correction-regularised "
                         "and weighted-window runs")
    ap.add_argument("--stream-plain-windows", type=int, default=4,
                    help="stream workload: windows run with plain launches")
    ap.add_argument("--fr-windows", type=int, default=3,
                    help="windows solved to a fixed residual (0: skip)")
    ap.add_argument("--no-small-chain", action="store_true",
                    help="skip the 64 x 64 chain in every execution mode")
    ap.add_argument("--no-host-window", action="store_true",
                    help="skip the window solved through host pointers "
                         "(PCIe-inclusive rate)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch choice by timing (else the "
                         "built-in default)")
    ap.add_argument("--cpu-sample-nt", type=int, default=3000)
    ap.add_argument("--cpu-sample-shots", type=int, default=2)
    ap.add_argument("--cpu-sample-nt3d", type=int, default=100,
                    help="3d workload: time steps of the oracle sample")
    ap.add_argument("--chain3d-windows", type=int, default=0,
                    help="3d workload: windows of the chain solved to a "
                         "fixed residual (0: skip)")
    ap.add_argument("--chain3d-iters", type=int, default=5,
                    help="3d workload: CG iterations that set the fixed "
                         "residual on window 0")
    ap.add_argument("--only-steps", action="store_true",
                    help="time the steps only (for profiler runs)")
    ap.add_argument("--workload", default="2d",
                    choices=["2d", "3d", "autograd", "stream", "ssf"],
                    help="2d: the window chain (default); 3d: the batched "
                         "3-D operator pair; autograd: differentiable Born "
                         "with checkpointed backgrounds; stream: ragged "
                         "streaming windows, latency p50/p99; ssf: the "
                         "split-step Fourier operator pair in the paper's "
                         "window configuration")
    ap.add_argument("--ssf-windows", type=int, default=0,
                    help="ssf workload: windows of the chain to run (0: all)")
    ap.add_argument("--ssf-precond", type=int, default=0, choices=[0, 1],
                    help="ssf workload: 1 = illumination-preconditioned CG")
    ap.add_argument("--ssf-regularize", type=int, default=0, choices=[0, 1],
                    help="ssf workload: 1 = damp the correction to the "
                         "previous window's image")
    ap.add_argument("--ssf-data", default="nonlinear",
                    choices=["nonlinear", "born"],
                    help="ssf workload: finite-difference modelling in the "
                         "true velocity minus that in the migration velocity "
                         "(nonlinear), or two-way FD Born data of the "
                         "reflectivity")
    ap.add_argument("--ops-only", action="store_true",
                    help="after setup run one 512 MiB device copy (the "
                         "counter calibration kernel) and one batched Born "
                         "and adjoint application on the first window, "
                         "then exit (for hardware-counter runs)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kind, Q, ngroups, npad, nint, nrec, steps=1):
    """Bytes one batched launch must move at minimum (float32), the launch
    advancing every shot by `steps` time steps (1, or 2 for the two-step
    kernels): per shot and padded point u read, v read, v write, u write
    (16 B, once per launch) and per step the Born-source frame on the model
    region (4 B) and the receiver samples (4 B each); per block group the
    medium W' (4 B/point) and the model vector (Born: 4 B) or the float64
    image accumulator read and written (adjoint: 16 B) on the model
    region."""
    per_shot = 16 * npad + steps * (4 * nint + 4 * nrec)
    if kind == "born":
        shared = 4 * npad + 4 * nint
    else:
        shared = 4 * npad + 16 * nint
    return Q * per_shot + ngroups * shared


def point_step_bytes(kind, B):
    """Algorithmic float32 bytes per (padded point, time step, shot) of one
    operator with stored Born sources, B shots sharing a work item, as a
    one-step-per-launch kernel moves them: the propagated field's u and v
    each read and written (16 B), plus per work item the medium W' (4 B)
    and, for Born, the model vector (4 B): Born 16 + 8 / B, adjoint
    16 + 4 / B (the image accumulator held on chip; the Born-source frame
    counted in neither, as in the per-step count of the design)."""
    return 16.0 + (8.0 if kind == "born" else 4.0) / B


def point_step_bytes_3d(kind, B):
    """Algorithmic float32 bytes per (padded point, time step, shot) of one
    3-D operator with checkpointed backgrounds, B shots sharing a work item:
    Born advances the background and the Born field together (two fields
    each read twice and written once, 24 B) plus the medium and the model
    vector per work item (8 / B); the adjoint step is the background
    recompute over a segment (12 B), its Born-source frame written and read
    back (8 B) and the adjoint field (12 B), plus the medium read by both
    launches (8 / B): Born 24 + 8 / B, adjoint 32 + 8 / B."""
    return (24.0 if kind == "born" else 32.0) + 8.0 / B


def small_chain(P, synth, torch, reps=5):
    """The launch-bound 64 x 64 chain (4 shots, windows of 2 sliding by 1,
    10 CG iterations each, lambda 0.01 relative to a power estimate of the
    first window): seconds for the whole chain from a zero image (updates,
    downdates, backgrounds, solves, image out) in each execution mode, the
    data synthesised by the library's Born + 1 % noise. Also the largest
    relative distance between the modes' final images."""
    w = synth.layers2d_64x64()
    vel = w.vel.astype(np.float32)
    nrec = w.shots[0].nrec
    m_true = torch.from_numpy(w.m_true.astype(np.float32)).cuda()
    n = len(w.shots)
    ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, w.nt, nrec, n, w.h, w.dt, 0.0,
                      vel, device=True)
    ctx.set_tuning(*DEFAULT_TUNING)
    for s in w.shots:
        ctx.update(s.id, s.src, s.rec, s.nt, s.f0, None)
    data = ctx.apply_born(m_true).view(n, w.nt, nrec).clone()
    ctx.close()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    rms = float(torch.sqrt(torch.mean(data.double() ** 2)))
    data += w.noise_rel * rms * torch.randn(data.shape, generator=gen,
                                            device="cuda")
    windows = w.windows()
    ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, w.nt, nrec, w.Q, w.h, w.dt,
                      0.0, vel, device=True)
    ctx.set_tuning(*DEFAULT_TUNING)
    for i in windows[0]:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
    x = torch.from_numpy(synth.gaussian(w.model_shape, 2002).astype(
        np.float32)).cuda()
    x /= torch.linalg.vector_norm(x)
    norm = 0.0
    for _ in range(8):
        y = ctx.apply_adjoint(ctx.apply_born(x))
        norm = float(torch.linalg.vector_norm(y.double()))
        x = y / norm
    ctx.close()
    lam = w.lam_rel * norm
    zero = torch.zeros(w.model_shape, dtype=torch.float32, device="cuda")
    image = torch.empty_like(zero)
    out, images = {}, {}
    for mode, name in ((P.BRLS_EXEC_PLAIN, "plain"),
                       (P.BRLS_EXEC_BATCHED, "batched"),
                       (P.BRLS_EXEC_GRAPH, "graph"),
                       (P.BRLS_EXEC_PERSISTENT, "persistent")):
        ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, w.nt, nrec, w.Q, w.h,
                          w.dt, lam, vel, device=True)
        ctx.set_tuning(*DEFAULT_TUNING)
        ctx.set_exec(mode)

        def chain():
            held = []
            ctx.set_image(zero)
            for win in windows:
                for i in list(held):
                    if i not in win:
                        ctx.downdate(i)
                        held.remove(i)
                for i in win:
                    if i not in held:
                        s = w.shots[i]
                        ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
                        held.append(i)
                ctx.solve_window(w.niter)
            ctx.image(image)
            for i in held:
                ctx.downdate(i)

        chain()  # graph capture and first-touch outside the timing
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            chain()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / reps
        images[name] = image.clone()
        ctx.close()
        out[name] = {"s_per_chain": round(sec, 5),
                     "ms_per_window": round(sec / len(windows) * 1e3, 3)}
        log(f"64x64 chain, {name}: {out[name]}")
    ref = images["graph"]
    out["max_rel_diff_between_modes"] = float(max(
        torch.linalg.vector_norm((v - ref).double()) /
        torch.linalg.vector_norm(ref.double()) for v in images.values()))
    out["windows"] = len(windows)
    out["cg_iters"] = w.niter
    out["lam"] = lam
    return out


def oracle_small_chain(synth):
    """The FP64 oracle on the same 64 x 64 chain, on its own inputs (oracle
    Born of the model + 1 % seeded noise, lambda from an 8-step power
    estimate): seconds for the whole chain, and for those inputs."""
    import oracle
    w = synth.layers2d_64x64()
    prob = oracle.Problem.from_workload(w)
    t = time.perf_counter()
    r = np.random.default_rng(7)
    noise = [r.standard_normal(prob.data_shape(i))
             for i in range(len(w.shots))]
    data = oracle.synthesize_data(prob, w.m_true, w.noise_rel, noise)
    lam = w.lam_rel * oracle.power_norm(prob, w.windows()[0], 8, seed=2002)
    t_in = time.perf_counter() - t
    t = time.perf_counter()
    oracle.chain(prob, data, w.windows(), lam, w.niter)
    return {"s_per_chain": round(time.perf_counter() - t, 3),
            "inputs_s": round(t_in, 3)}


def fixed_residual(args, P, w, data, lam, vel, torch):
    """Seconds per window solve at a fixed CG residual. The stop test is
    ||A^T r - lambda m|| <= tau ||A^T d||, with tau the ratio the first
    window (cold start) reaches after the configured iteration count. The
    chain's first windows are solved to tau with the batched graph launches
    (plain CG, and CG preconditioned by the window's illumination) and, the
    first of them, with plain per-shot launches."""
    nrec = w.shots[0].nrec
    windows = w.windows()

    def chain(exec_mode, nwin, rtol, max_iter, precond=0):
        ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, w.nt, nrec, w.Q, w.h, w.dt,
                          lam, vel, device=True)
        ctx.set_tuning(*DEFAULT_TUNING)
        ctx.set_exec(exec_mode)
        ctx.set_precond(precond)
        held, stats = [], []
        for k in range(nwin):
            win = windows[k]
            for i in list(held):
                if i not in win:
                    ctx.downdate(i)
                    held.remove(i)
            for i in win:
                if i not in held:
                    s = w.shots[i]
                    ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
                    held.append(i)
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = ctx.solve_window(max_iter, rtol)
            torch.cuda.synchronize()
            st["wall"] = time.perf_counter() - t
            stats.append(st)
            log(f"fixed residual ({'plain' if exec_mode == P.BRLS_EXEC_PLAIN else 'graph'}"
                f"{', preconditioned' if precond else ''}) "
                f"window {k}: iters={st['iters']} s={st['wall']:.3f}")
        ctx.close()
        return stats

    # tau from window 0 after the configured iterations (rtol tiny: the
    # stop test never fires, but the solve reports ||A^T d||)
    st0 = chain(P.BRLS_EXEC_GRAPH, 1, 1e-30, args.iters)[0]
    tau = st0["s_norm"] / st0["ref_norm"]
    g = chain(P.BRLS_EXEC_GRAPH, args.fr_windows, tau, 10 * args.iters)
    p = chain(P.BRLS_EXEC_PLAIN, 1, tau, 10 * args.iters)
    pc = chain(P.BRLS_EXEC_GRAPH, args.fr_windows, tau, 10 * args.iters,
               precond=1)

    def summary(stats):
        secs = [x["wall"] for x in stats]
        return {"windows": len(stats),
                "s_per_window_mean": round(float(np.mean(secs)), 4),
                "s_per_window_max": round(float(np.max(secs)), 4),
                "iters": [x["iters"] for x in stats]}
    return {"tau": tau, "graph": summary(g), "plain": summary(p),
            "plain_over_graph_first_window":
                round(p[0]["wall"] / g[0]["wall"], 3),
            "graph_illumination_preconditioned": summary(pc)}


def host_window(args, P, w, data, lam, vel, torch):
    """The first window solved by a context that takes host pointers: the
    window's data leave host memory inside brls_update (one copy per shot)
    and the image returns to host memory. Timed from the first update to
    the image on the host, against the same window through device
    pointers."""
    nrec = w.shots[0].nrec
    win = w.windows()[0]
    host = {i: data[i].cpu().numpy() for i in win}
    npad = (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb)
    res = {}
    for device in (False, True):
        ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, w.nt, nrec, w.Q, w.h, w.dt,
                          lam, vel, device=device)
        ctx.set_tuning(*DEFAULT_TUNING)
        ctx.set_exec(P.BRLS_EXEC_GRAPH)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in win:
            s = w.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0,
                       data[i] if device else host[i])
        st = ctx.solve_window(args.iters)
        img = ctx.image()
        if device:
            torch.cuda.synchronize()
        sec = time.perf_counter() - t
        ctx.close()
        ups = 2 * (1 + st["iters"]) * len(win) * npad * (w.nt - 1)
        res["host" if not device else "device"] = {
            "seconds": round(sec, 4),
            "Gpt_updates_per_s": round(ups / sec / 1e9, 2)}
        del img
    res["host_over_device"] = round(res["host"]["seconds"]
                                    / res["device"]["seconds"], 4)
    res["h2d_bytes"] = int(sum(host[i].nbytes for i in win))
    return res


def ops_only(P, w, vel, m_true):
    """One 512 MiB device copy (calibrates the memory counters), then one
    batched Born and one adjoint application over the first window (the
    kernels the timed steps run, one launch chain), for hardware-counter
    runs."""
    import torch
    src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    nrec = w.shots[0].nrec
    ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, w.nt, nrec, w.Q, w.h, w.dt,
                      1.0, vel, device=True)
    for i in w.windows()[0]:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
    ctx.set_tuning(*DEFAULT_TUNING)
    ctx.set_exec(P.BRLS_EXEC_BATCHED)
    # one chain: each launch covers the whole window, as in the per-launch
    # roofline figures the counters are paired with
    ctx.set_chains(1)
    ctx.apply_adjoint(ctx.apply_born(m_true))
    torch.cuda.synchronize()
    ctx.close()
    log("ops-only: done")


def bytes3d(kind, Q, ngroups, npad, nint, nrec):
    """Algorithmic bytes of one batched 3-D step launch (float32), with the
    background checkpointed and recomputed: the fused Born step advances two
    fields (32 B per shot and padded point); the background recompute
    advances one and writes its Born source on the model region; the
    adjoint advances one and reads that source; per block group the medium
    and the model vector (Born) or the float64 image accumulator (adjoint)."""
    if kind == "born":
        return Q * (32 * npad + 4 * nrec) + ngroups * (4 * npad + 4 * nint)
    if kind == "background":
        return Q * (16 * npad + 4 * nint) + ngroups * 4 * npad
    return Q * (16 * npad + 4 * nint + 4 * nrec) + ngroups * (
        4 * npad + 16 * nint)


def bench_3d(args, P, synth, torch):
    """3-D batching form: 256 x 320 x 320 model (296 x 360 x 360 padded),
    one 8-shot window, 128 x 128 receivers, nt = 2000, background
    checkpointed every ceil(sqrt(nt)) steps. Times one Born + adjoint pair
    replayed from a graph against the plain per-shot launches."""
    w = synth.layered3d_256x320x320()
    Q = w.Q
    nt, nrec = w.nt, w.shots[0].nrec
    pz, py, px = (w.nz + 2 * w.nb, w.ny + 2 * w.nb, w.nx + 2 * w.nb)
    npad, nint = pz * py * px, w.nz * w.ny * w.nx
    vel = w.vel.astype(np.float32)
    m = torch.from_numpy(w.m_true.astype(np.float32)).cuda()
    ctx = P.brls_open(3, w.nz, w.ny, w.nx, w.nb, nt, nrec, Q, w.h, w.dt, 1.0,
                      vel, device=True, ckpt_interval=-1)
    for i in w.windows()[0]:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
    t = time.perf_counter()
    if args.autotune:
        ctx.autotune()
    else:
        ctx.set_tile(DEFAULT_TILE3)
        ctx.apply_born(m)  # builds the background checkpoints
    torch.cuda.synchronize()
    log(f"3d: checkpoints + tuning {time.perf_counter() - t:.1f}s, tile "
        f"{ctx.get_tuning()} {P.tile3_variants()[ctx.get_tile()[0]]}")
    res = {}
    modes = [(P.BRLS_EXEC_GRAPH, "graph")]
    if not args.no_plain:
        modes.append((P.BRLS_EXEC_PLAIN, "plain"))
    d = None
    for mode, name in modes:
        ctx.set_exec(mode)
        if mode == P.BRLS_EXEC_GRAPH:
            d = ctx.apply_born(m)
            ctx.apply_adjoint(d)  # graph capture outside the timing
        torch.cuda.synchronize()
        t = time.perf_counter()
        d = ctx.apply_born(m)
        ctx.apply_adjoint(d)
        torch.cuda.synchronize()
        res[name] = time.perf_counter() - t
        log(f"3d {name}: {res[name]:.2f}s")
    ctx.set_exec(P.BRLS_EXEC_BATCHED)
    ctx.kernel_timing(True)
    ctx.apply_adjoint(ctx.apply_born(m))
    ks = ctx.kernel_stats()
    ctx.kernel_timing(False)
    var, pb = ctx.get_tile()
    ngroups = (Q + pb - 1) // pb
    roof = {}
    for kind, name in (("born", "born_step"), ("adjoint", "adjoint_step"),
                       ("background", "background_step")):
        n, ms = ks[name]
        avg = ms / n / 1e3
        b = bytes3d(kind, Q, ngroups, npad, nint, nrec)
        roof[kind] = dict(avg_us=avg * 1e6, bytes=b, gbs=b / avg / 1e9)
    # per operator and time step on the per-unit bytes: Born one launch,
    # the adjoint two (background recompute + adjoint field)
    units = Q * npad
    op_us = {"born": roof["born"]["avg_us"],
             "adjoint": roof["adjoint"]["avg_us"] +
             roof["background"]["avg_us"]}
    op = {k: dict(us=v, bytes=int(point_step_bytes_3d(k, pb) * units))
          for k, v in op_us.items()}
    mem = ctx.memory_bytes()
    ctx.close()
    chain = window_chain_3d(args, P, w, m, vel, torch) \
        if args.chain3d_windows > 0 else None
    pair = 2 * Q * npad * (nt - 1)
    dop = max(op, key=lambda k: op[k]["us"])
    out = {
        "metric": "Born+adjoint Gpt-updates/s",
        "value": round(pair / res["graph"] / 1e9, 3),
        "unit": "Gpt-updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(res["graph"] * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "layered3d-256x320x320: one window of 8 "
                               "shots, 128x128 receivers, nt=2000, one Born "
                               "+ adjoint pair, background checkpointed "
                               "(45 steps)",
                   "padded_grid": [pz, py, px], "tile": [var, pb]},
        "device_bytes": mem,
        "roofline": {
            "bound": "hbm",
            "kernel": (f"{dop} time step (k_step3d"
                       + (", background recompute + adjoint launches)"
                          if dop == "adjoint" else ")")),
            "achieved": round(op[dop]["bytes"] / op[dop]["us"] / 1e3, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(op[dop]["bytes"] / op[dop]["us"] / 1e3
                          / HBM_PEAK_GBS, 4),
            "traffic": None,
            "avg_step_us": round(op[dop]["us"], 1),
            "algorithmic_bytes_per_step": op[dop]["bytes"],
            "bytes_basis": f"{point_step_bytes_3d(dop, pb):g} B per padded "
                           f"point, step and shot x {units} point-step-"
                           "shots per step",
            "other": {k: {"avg_step_us": round(v["us"], 1),
                          "achieved_GBs": round(v["bytes"] / v["us"] / 1e3,
                                                1)}
                      for k, v in op.items() if k != dop},
            # the launches on the tighter count (difference-form fields,
            # model-region sources, the image accumulator)
            "launches": {k: {"avg_launch_us": round(v["avg_us"], 1),
                             "bytes": v["bytes"],
                             "achieved_GBs": round(v["gbs"], 1)}
                         for k, v in roof.items()},
        },
        "plain_per_shot": ({"seconds": round(res["plain"], 3),
                            "Gpt_updates_per_s":
                                round(pair / res["plain"] / 1e9, 3)}
                           if "plain" in res else None),
        "window_chain": chain,
    }
    if not args.no_cpu_baseline:
        # the oracle on one shot at a bounded length (one Born and one
        # adjoint application, FP64, OpenMP over the host cores)
        import oracle
        ns = args.cpu_sample_nt3d
        s0 = w.shots[0]
        shots = [synth.Shot(0, s0.src, s0.rec, ns, s0.f0)]
        grid = oracle.Grid(3, w.nz, w.ny, w.nx, w.nb, w.h, w.dt)
        prob = oracle.Problem(grid, vel.astype(np.float64), shots)
        t = time.perf_counter()
        d = prob.born_shot(0, w.m_true.astype(np.float32).astype(np.float64))
        prob.adjoint_shot(0, d)
        tc = time.perf_counter() - t
        cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
        out["cpu_baseline"] = {
            "value": round(2 * npad * (ns - 1) / tc / 1e9, 4),
            "unit": "Gpt-updates/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"1 shot, nt={ns} (of {nt}), one Born + one adjoint "
                      f"application, FP64, {tc:.1f}s",
        }
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def window_chain_3d(args, P, w, m, vel, torch):
    """The 3-D block-row chain: windows of 8 shots sliding by 4, data
    A m_true + 1 % noise synthesised on the GPU, lambda 1e-3 of a 2-step
    power estimate of ||A_w0^T A_w0||. Window 0 runs --chain3d-iters CG
    iterations with graph launches; the ratio ||s|| / ||A^T d|| it reaches
    is the fixed residual tau. The next windows (warm-started, graph) and
    window 0 again with plain per-shot launches are solved to tau; seconds
    per window and iterations are reported."""
    Q, S = w.Q, w.S
    nt, nrec = w.nt, w.shots[0].nrec
    nwin = args.chain3d_windows
    wins = w.windows()[:nwin]
    shots = sorted({i for win in wins for i in win})
    t0 = time.perf_counter()
    ctx = P.brls_open(3, w.nz, w.ny, w.nx, w.nb, nt, nrec, Q, w.h, w.dt, 0.0,
                      vel, device=True, ckpt_interval=-1)
    ctx.set_tile(DEFAULT_TILE3)
    data = {}
    for b in range(0, len(shots), Q):
        ids = shots[b:b + Q]
        for i in ids:
            s = w.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
        d = ctx.apply_born(m)
        off = 0
        for i in ctx.window():
            s = w.shots[i]
            n = s.nt * s.nrec
            data[i] = d[off:off + n].clone()
            off += n
        for i in ids:
            ctx.downdate(i)
    rms = float(np.sqrt(sum(float((x.double() ** 2).sum())
                            for x in data.values())
                        / sum(x.numel() for x in data.values())))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3001)
    for i in shots:
        data[i] += 0.01 * rms * torch.randn(data[i].shape, generator=gen,
                                            device="cuda")
    for i in wins[0]:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
    x = torch.from_numpy(synth_gaussian(w.model_shape, 2002)).cuda()
    x /= torch.linalg.vector_norm(x)
    nrm = 0.0
    for _ in range(2):
        y = ctx.apply_adjoint(ctx.apply_born(x))
        nrm = float(torch.linalg.vector_norm(y.double()))
        x = y / nrm
    ctx.close()
    torch.cuda.synchronize()
    log(f"3d chain: data of {len(shots)} shots and lambda in "
        f"{time.perf_counter() - t0:.1f}s")
    lam = w.lam_rel * nrm

    def solve(exec_mode, ks, rtol, iters):
        c = P.brls_open(3, w.nz, w.ny, w.nx, w.nb, nt, nrec, Q, w.h, w.dt,
                        lam, vel, device=True, ckpt_interval=-1)
        c.set_tile(DEFAULT_TILE3)
        c.set_exec(exec_mode)
        held, out = [], []
        for k in ks:
            torch.cuda.synchronize()
            t = time.perf_counter()
            for i in list(held):
                if i not in wins[k]:
                    c.downdate(i)
                    held.remove(i)
            for i in wins[k]:
                if i not in held:
                    s = w.shots[i]
                    c.update(i, s.src, s.rec, s.nt, s.f0, data[i])
                    held.append(i)
            st = c.solve_window(iters, rtol=rtol)
            torch.cuda.synchronize()
            out.append(dict(window=k, seconds=round(time.perf_counter() - t,
                                                    2),
                            iters=st["iters"],
                            s_over_ref=(st["s_norm"] / st["ref_norm"]
                                        if st["ref_norm"] > 0 else None)))
            log(f"3d chain {exec_mode} window {k}: {out[-1]}")
        c.close()
        return out

    first = solve(P.BRLS_EXEC_GRAPH, [0], 1e-12, args.chain3d_iters)
    tau = first[0]["s_over_ref"]
    graph = solve(P.BRLS_EXEC_GRAPH, list(range(nwin)), tau, 1000)
    plain = solve(P.BRLS_EXEC_PLAIN, [0], tau, 1000) \
        if not args.no_plain else None
    return {
        "windows": [list(x) for x in wins],
        "lambda": lam,
        "tau": tau,
        "tau_from": f"window 0 after {args.chain3d_iters} iterations",
        "graph": graph,
        "graph_s_per_window_mean": round(
            float(np.mean([x["seconds"] for x in graph])), 2),
        "plain_window0": plain,
        "note": "each window's seconds include the new shots' background "
                "checkpoints; plain = one launch per shot and time step",
    }


def synth_gaussian(shape, seed):
    import synth
    return synth.gaussian(shape, seed).astype(np.float32)


def bench_autograd(args, P, synth, torch):
    """Differentiation form on the 512 x 1024 model: one forward + backward
    of 0.5 ||A m - d||^2 through BornFn over an 8-shot window, background
    checkpointed every ceil(sqrt(nt)) steps vs stored for every step; device
    memory and recompute cost, and the finite-difference check along 4
    smoothed seeded directions."""
    from scipy.ndimage import gaussian_filter

    from paper_1801_00819_amd.autograd import misfit
    w = synth.faulted2d_512x1024()
    nt, nrec = w.nt, w.shots[0].nrec
    vel = w.vel.astype(np.float32)
    mt = torch.from_numpy(w.m_true.astype(np.float32)).cuda()
    res = {}
    for ck, name in ((-1, "checkpointed"), (0, "stored")):
        ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, nt, nrec, 8, w.h, w.dt, 1.0,
                          vel, device=True, ckpt_interval=ck)
        for i in w.windows()[0]:
            s = w.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
        ctx.set_tuning(*(DEFAULT_TUNING_CKPT if ck else DEFAULT_TUNING))
        d = ctx.apply_born(mt)
        m = (0.5 * mt).requires_grad_(True)
        misfit(m, d, ctx).backward()  # warm-up: graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        m.grad = None
        loss = misfit(m, d, ctx)
        loss.backward()
        torch.cuda.synchronize()
        res[name] = dict(seconds=round(time.perf_counter() - t, 4),
                         device_bytes=ctx.memory_bytes())
        if ck == -1:
            g = m.grad.double()
            m0 = (0.5 * mt).detach()
            fds, ans = [], []
            for k in range(4):
                p = gaussian_filter(synth.gaussian(w.model_shape, 2000 + k)
                                    [:, 0, :], 4.0)[:, None, :]
                p = torch.from_numpy(np.ascontiguousarray(p)).cuda()
                p *= torch.linalg.vector_norm(m0.double()) / \
                    torch.linalg.vector_norm(p)
                mp = (m0.double() + 1e-3 * p).float()
                mm = (m0.double() - 1e-3 * p).float()
                pe = (mp.double() - mm.double()) / 2e-3
                with torch.no_grad():
                    fds.append(float((misfit(mp, d, ctx) - misfit(mm, d, ctx))
                                     / 2e-3))
                ans.append(float(torch.sum(g * pe)))
            fds, ans = np.array(fds), np.array(ans)
            res[name]["fd_rel_l2"] = float(np.linalg.norm(fds - ans) /
                                           np.linalg.norm(ans))
        ctx.close()
        log(f"autograd {name}: {res[name]}")
    pair = 2 * 8 * (w.nz + 2 * w.nb) * (w.nx + 2 * w.nb) * (nt - 1)
    tc = res["checkpointed"]["seconds"]
    out = {
        "metric": "Born+adjoint Gpt-updates/s",
        "value": round(pair / tc / 1e9, 3),
        "unit": "Gpt-updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(tc * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "faulted2d-512x1024 autograd: BornFn forward "
                               "+ backward, 8 shots, nt=3000, checkpoints "
                               "every 55 steps"},
        "checkpointed": res["checkpointed"],
        "stored": res["stored"],
        "recompute_time_ratio": round(tc / res["stored"]["seconds"], 3),
        "memory_ratio": round(res["checkpointed"]["device_bytes"] /
                              res["stored"]["device_bytes"], 4),
    }
    print(json.dumps(out), flush=True)


def bench_stream(args, P, synth, torch):
    """Streaming uneven batching on the 512 x 1024 model: shots arrive in
    sweeps of the 64 positions with apertures U{256..1024} receivers and nt
    in {2000, 3000, 4000}, the reflectivity drifting 0.1 % per 64 shots.
    For each window size Q in {4, 8, 16} (slide Q / 2) the warm-started
    chain runs --stream-iters CG iterations per window over the first
    --stream-shots shots; reported: per-window latency (downdate + update +
    solve + image out) p50 / p99 with the batched graph launches, and with
    plain per-shot launches on the first windows."""
    nsh = args.stream_shots
    base = synth.stream2d_512x1024(nshots=nsh, Q=8)
    vel = base.vel.astype(np.float32)
    nrec_max = max(s.nrec for s in base.shots)
    nt_max = max(s.nt for s in base.shots)
    # data d_i = A_i m_i + 1 % noise, m_i the drifting model; shots in
    # batches of 8 that share the model of the batch's middle shot (the
    # drift within a batch, 0.0125 %, is far below the noise)
    t0 = time.perf_counter()
    ctx = P.brls_open(2, base.nz, 1, base.nx, base.nb, nt_max, nrec_max, 8,
                      base.h, base.dt, 0.0, vel, device=True)
    ctx.set_tuning(*DEFAULT_TUNING)
    data = []
    for b in range(0, nsh, 8):
        ids = list(range(b, min(b + 8, nsh)))
        for i in ids:
            s = base.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
        mb = torch.from_numpy(synth.model_at(base, ids[len(ids) // 2])
                              .astype(np.float32)).cuda()
        d = ctx.apply_born(mb)
        off = 0
        for i in ctx.window():
            s = base.shots[i]
            n = s.nt * s.nrec
            data.append((i, d[off:off + n].view(s.nt, s.nrec).clone()))
            off += n
        for i in ids:
            ctx.downdate(i)
    ctx.close()
    data = [x for _, x in sorted(data, key=lambda t: t[0])]
    rms = float(np.sqrt(sum(float((x.double() ** 2).sum()) for x in data)
                        / sum(x.numel() for x in data)))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4001)
    for x in data:
        x += 0.01 * rms * torch.randn(x.shape, generator=gen, device="cuda")
    log(f"stream: data for {nsh} shots in {time.perf_counter() - t0:.1f}s")

    def run(Q, exec_mode, nwin, regularize=0, forgetting=None):
        w = synth.stream2d_512x1024(nshots=nsh, Q=Q)
        wins = w.windows()[:nwin]
        c = P.brls_open(2, w.nz, 1, w.nx, w.nb, nt_max, nrec_max, Q, w.h,
                        w.dt, 0.0, vel, device=True)
        c.set_tuning(*DEFAULT_TUNING)
        # lambda: relative 1e-3 of ||A^T A|| on the first window (power
        # iteration, 4 steps)
        for i in wins[0]:
            s = w.shots[i]
            c.update(i, s.src, s.rec, s.nt, s.f0, data[i])
        x = torch.from_numpy(synth.gaussian(w.model_shape, 2002)
                             .astype(np.float32)).cuda()
        x /= torch.linalg.vector_norm(x)
        nrm = 0.0
        for _ in range(4):
            y = c.apply_adjoint(c.apply_born(x))
            nrm = float(torch.linalg.vector_norm(y.double()))
            x = y / nrm
        c.close()
        c = P.brls_open(2, w.nz, 1, w.nx, w.nb, nt_max, nrec_max, Q, w.h,
                        w.dt, w.lam_rel * nrm, vel, device=True)
        c.set_tuning(*DEFAULT_TUNING)
        c.set_exec(exec_mode)
        c.set_regularization(regularize)
        image = torch.empty(w.model_shape, dtype=torch.float32, device="cuda")
        prev = torch.zeros_like(image)
        m0 = torch.from_numpy(w.m_true).cuda()
        drift = torch.from_numpy(w.extra["drift"]).cuda()
        held, lat, its, err, chg = [], [], [], [], []
        first = {}
        for k, win in enumerate(wins):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for i in list(held):
                if i not in win:
                    c.downdate(i)
                    held.remove(i)
            for i in win:
                if i not in held:
                    s = w.shots[i]
                    c.update(i, s.src, s.rec, s.nt, s.f0, data[i])
                    held.append(i)
                first.setdefault(i, k)
                if forgetting is not None:  # exponentially weighted window
                    c.set_shot_weight(i, forgetting ** (k - first[i]))
            st = c.solve_window(args.stream_iters)
            c.image(image)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t)
            its.append(st["iters"])
            # image quality, outside the timed latency: relative error
            # against the model the window's middle shot sees, and the
            # relative change from the previous window's image
            truth = m0 + (win[len(win) // 2] / 64.0) * drift
            img = image.double()
            err.append(float(torch.linalg.vector_norm(img - truth)
                             / torch.linalg.vector_norm(truth)))
            chg.append(float(torch.linalg.vector_norm(img - prev)
                             / torch.linalg.vector_norm(img)))
            prev.copy_(image)
            if k % 16 == 15:
                log(f"stream Q={Q} exec {exec_mode}: window {k + 1}/"
                    f"{len(wins)}, latency {lat[-1]:.3f}s")
        c.close()
        return lat, len(w.windows()), err, chg

    def summary(lat, err, chg):
        # the first window of each run includes graph capture and the
        # backgrounds of all Q shots; latencies are over the later windows
        steady = lat[1:] if len(lat) > 1 else lat
        half = len(err) // 2
        return {
            "windows": len(lat),
            "p50_s": round(float(np.percentile(steady, 50)), 4),
            "p99_s": round(float(np.percentile(steady, 99)), 4),
            "mean_s": round(float(np.mean(steady)), 4),
            "first_window_s": round(lat[0], 4),
            "image_rel_err_last": round(err[-1], 4),
            "image_rel_err_mean_second_half": round(
                float(np.mean(err[half:])), 4),
            "image_rel_change_mean_second_half": round(
                float(np.mean(chg[half:])), 4),
        }

    per_q = {}
    for Q in (4, 8, 16):
        lat, total, err, chg = run(Q, P.BRLS_EXEC_GRAPH, 10 ** 9)
        plain, _, _, _ = run(Q, P.BRLS_EXEC_PLAIN, args.stream_plain_windows)
        per_q[Q] = summary(lat, err, chg)
        per_q[Q]["plain_windows"] = len(plain)
        per_q[Q]["plain_p50_s"] = round(
            float(np.percentile(plain[1:] or plain, 50)), 4)
        log(f"stream Q={Q}: {per_q[Q]}")
    corr = forget = None
    if not args.no_stream_options:
        # the correction-regularised recursion (damping towards the
        # previous window's image instead of towards zero) on the same
        # Q = 8 stream
        lat, _, err, chg = run(8, P.BRLS_EXEC_GRAPH, 10 ** 9, regularize=1)
        corr = summary(lat, err, chg)
        log(f"stream Q=8 correction-regularised: {corr}")
        # and with each shot's misfit weighted by beta^age (forgetting
        # factor)
        lat, _, err, chg = run(8, P.BRLS_EXEC_GRAPH, 10 ** 9, regularize=1,
                               forgetting=args.stream_forgetting)
        forget = summary(lat, err, chg)
        forget["beta"] = args.stream_forgetting
        log(f"stream Q=8 correction-regularised, weighted window: {forget}")
    out = {
        "metric": "window solve latency p50 (Q=8)",
        "value": per_q[8]["p50_s"],
        "unit": "s",
        "n_gpus": 1, "steps": per_q[8]["windows"], "warmup": 0,
        "ms_per_step": round(per_q[8]["mean_s"] * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"stream2d-512x1024: first {nsh} of 512 "
                               "shots, apertures 256-1024, nt 2000/3000/"
                               f"4000, slide Q/2, {args.stream_iters} CG "
                               "iterations per window, drift 0.1 % per 64 "
                               "shots"},
        "per_window_size": {str(k): v for k, v in per_q.items()},
        "correction_regularised_q8": corr,
        "correction_regularised_weighted_q8": forget,
    }
    print(json.dumps(out), flush=True)


def ssf_flops_per_step(n):
    """Algorithmic float operations of one depth step of one (shot,
    frequency) field of n points: an n-point FFT and its inverse at
    5 n log2 n each (the standard count), the wavenumber-domain phase and
    the split-step phase with the taper (a complex multiply and a real
    scale each: 8 per point), and the Born injection or imaging term (4 per
    point). The phase angles' sine, cosine and square root are not
    counted."""
    return 10 * n * int(round(np.log2(n))) + 20 * n


def ssf_bytes(kind, items, nz, n, nrec_items):
    """Minimum HBM bytes of one launch over `items` (shot, frequency) pairs:
    the Born weights of every item and level (8 B per point); Born: the
    model once (4 B per point) and the receiver samples written (8 B per
    complex sample); adjoint: the receiver samples read and every item's
    image contribution written (4 B per point and level)."""
    wb = items * nz * n * 8
    if kind == "born":
        return wb + nz * n * 4 + 8 * nrec_items
    return wb + 8 * nrec_items + items * nz * n * 4


def bench_ssf(args, P, synth, torch):
    """Split-step Fourier shot-profile operator pair (the paper's own
    operator family) in the paper's window configuration on the 256 x 1024
    Marmousi stand-in: 240 shots, windows of 5 sliding by 3, 8 CG
    iterations per window, warm-started. The observed data come from the
    library's two-way 8th-order finite-difference modelling on a grid two
    rows taller (sources and receivers 2 cells down): by default the
    modelling in the true (faulted, blocky) velocity minus that in the
    migration velocity (nonlinear data, the paper's kind), or with
    --ssf-data born the FD Born data of the reflectivity; plus 1 % noise.
    The one-way operator never sees its own modelling. Reports the chain's
    throughput, seconds per window, per-kernel timing and the roofline of
    the dominant kernel."""
    from paper_1801_00819_amd.ssf import brls_ssf_open
    w = synth.ssf2d_256x1024()
    nz, nx, Q = w.nz, w.nx, w.Q
    nrec = w.shots[0].nrec
    if args.ops_only:
        # one 512 MiB device copy (calibrates the memory counters), then one
        # Born and one adjoint application over the first window
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        c = brls_ssf_open(nz, nx, w.dx, w.dz, w.nt, w.dt, w.fmin, w.fmax,
                          w.ntap, nrec, Q, 1.0, w.vel.astype(np.float32),
                          device=True)
        for i in w.windows()[0]:
            s = w.shots[i]
            c.update(i, s.xs, s.rec, s.f0)
        m = torch.from_numpy(w.m_true.astype(np.float32)).cuda()
        c.apply_adjoint(c.apply_born(m))
        torch.cuda.synchronize()
        c.close()
        log("ssf ops-only: done")
        return
    windows = w.windows()
    if args.ssf_windows > 0:
        windows = windows[:args.ssf_windows]
    need = sorted({i for win in windows for i in win})
    # ---- FD data (untimed) ---------------------------------------------
    t0 = time.perf_counter()

    # the FD grid: two rows above the model (sources and receivers 2 cells
    # down), and one row below at the larger of the two models' largest
    # velocities, so that both modellings get the same sponge (its damping
    # scales with the model's largest velocity) and the common wavefield,
    # direct wave included, cancels in their difference
    vcap = max(float(w.extra["vel_true"].max()), float(w.vel.max()))

    def fd_grid(v):
        return np.concatenate([np.repeat(v[:1], 2, 0), v,
                               np.full((1, nx), vcap)], 0)[:, None, :] \
            .astype(np.float32)
    nzf = nz + 3
    nonlinear = args.ssf_data == "nonlinear"
    if nonlinear:
        # modelling only: checkpointed backgrounds keep memory small
        fds = [P.brls_open(2, nzf, 1, nx, 40, w.nt, nrec, 8, w.dx, w.dt,
                           0.0, fd_grid(v), device=True, ckpt_interval=-1)
               for v in (w.extra["vel_true"], w.vel)]
        m_ref = w.extra["m_nonlinear"]
    else:
        fds = [P.brls_open(2, nzf, 1, nx, 40, w.nt, nrec, 8, w.dx, w.dt,
                           0.0, fd_grid(w.vel), device=True)]
        fds[0].set_tuning(*DEFAULT_TUNING)
        m_fd = np.concatenate([np.zeros((2, nx)), w.m_true,
                               np.zeros((1, nx))], 0)
        m_fd_t = torch.from_numpy(m_fd[:, None, :].astype(np.float32)).cuda()
        m_ref = w.m_true
    data = {}
    for b in range(0, len(need), 8):
        ids = need[b:b + 8]
        for fd in fds:
            for i in ids:
                s = w.shots[i]
                rec = np.stack([np.full(nrec, 2), np.zeros(nrec, int),
                                s.rec], 1).astype(np.int32)
                fd.update(i, (2, 0, s.xs), rec, w.nt, s.f0, None)
        if nonlinear:
            d = fds[0].background_window() - fds[1].background_window()
        else:
            d = fds[0].apply_born(m_fd_t)
        d = d.view(len(ids), w.nt, nrec)
        if nonlinear:
            # top mute: the true-minus-background difference also holds the
            # head and diving waves of the blocky shallow section and the
            # water-bottom reflection, which one-way continuation does not
            # model; keep each trace from just below the water-bottom
            # reflection time t0 + sqrt(x^2 + (2 z_w)^2) / v_w + 2 / f0
            # (40 ms cosine ramp)
            for k, i in enumerate(fds[0].window()):
                s = w.shots[i]
                off = torch.from_numpy(np.abs(s.rec - s.xs) * w.dx).cuda()
                tm = 1.5 / s.f0 + torch.sqrt(off ** 2 + 400.0 ** 2) / 1500.0 \
                    + 2.0 / s.f0
                t = torch.arange(w.nt, device="cuda",
                                 dtype=torch.float64)[:, None] * w.dt
                ramp = torch.clamp((t - tm[None, :]) / 0.04, 0.0, 1.0)
                d[k] *= (0.5 - 0.5 * torch.cos(np.pi * ramp)).float()
        for k, i in enumerate(fds[0].window()):
            data[i] = d[k].clone()
        for fd in fds:
            for i in ids:
                fd.downdate(i)
    for fd in fds:
        fd.close()
    rms = float(np.sqrt(sum(float((x.double() ** 2).sum())
                            for x in data.values())
                        / sum(x.numel() for x in data.values())))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5001)
    for i in need:
        data[i] += 0.01 * rms * torch.randn(data[i].shape, generator=gen,
                                            device="cuda")
    log(f"ssf: FD {args.ssf_data} data for {len(need)} shots in "
        f"{time.perf_counter() - t0:.1f}s")

    def open_ctx(lam):
        return brls_ssf_open(nz, nx, w.dx, w.dz, w.nt, w.dt, w.fmin, w.fmax,
                             w.ntap, nrec, Q, lam, w.vel.astype(np.float32),
                             device=True)

    # ---- lambda: 1e-3 of ||A^T A|| on the first window (4 power steps) ----
    c = open_ctx(0.0)
    for i in windows[0]:
        s = w.shots[i]
        c.update(i, s.xs, s.rec, s.f0, data[i])
    x = torch.from_numpy(synth.gaussian(w.model_shape, 5002)
                         .astype(np.float32)).cuda()
    x /= torch.linalg.vector_norm(x)
    nrm = 0.0
    for _ in range(4):
        y = c.apply_adjoint(c.apply_born(x))
        nrm = float(torch.linalg.vector_norm(y.double()))
        x = y / nrm
    k0, nw, df = c.band()
    c.close()
    lam = w.lam_rel * nrm
    # ---- the chain (timed) ---------------------------------------------
    c = open_ctx(lam)
    c.set_precond(args.ssf_precond)
    c.set_regularization(args.ssf_regularize)
    image = torch.empty(w.model_shape, dtype=torch.float32, device="cuda")
    held, lat, its = [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for win in windows:
        t = time.perf_counter()
        for i in list(held):
            if i not in win:
                c.downdate(i)
                held.remove(i)
        for i in win:
            if i not in held:
                s = w.shots[i]
                c.update(i, s.xs, s.rec, s.f0, data[i])
                held.append(i)
        st = c.solve_window(w.niter)
        c.image(image)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
        its.append(st["iters"])
    total = time.perf_counter() - t_all
    last = st
    # migration image of the last window (A^T d), for the quality figure
    mig = c.apply_adjoint(c.observed())
    # ---- per-kernel timing on the last window ---------------------------
    c.kernel_timing(True)
    c.solve_window(2)
    ks = c.kernel_stats()
    c.kernel_timing(False)
    mem = c.memory_bytes()
    c.close()
    items = Q * nw
    nrec_items = items * nrec
    roof = {}
    for kind, name in (("born", "ssf_born"), ("adjoint", "ssf_adjoint")):
        n, ms = ks[name]
        avg = ms / n / 1e3
        fl = items * (nz - 1) * ssf_flops_per_step(nx)
        by = ssf_bytes(kind, items, nz, nx, nrec_items)
        roof[kind] = dict(avg_us=avg * 1e6, flops=fl, bytes=by,
                          tflops=fl / avg / 1e12, gbs=by / avg / 1e9)
    n, ms = ks["ssf_image_sum"]
    sum_us = ms / n * 1e3
    sum_bytes = items * nz * nx * 4 + nz * nx * 4
    dom = max(roof, key=lambda k: roof[k]["avg_us"])
    # operator point-steps of the chain: every window runs niter + 1 Born
    # and niter + 1 adjoint applications over its items x nz x nx points
    pts = sum((it + 1) * 2 for it in its) * items * nz * nx
    # quality: normalised correlation with the reflectivity in the zone the
    # last window illuminates (from its leftmost receiver to its rightmost
    # source), the chain's image against that window's migration image
    lw = [w.shots[i] for i in windows[-1]]
    zs = slice(24, nz - 16)  # below the water bottom
    xs_ = slice(int(min(s.rec.min() for s in lw)),
                int(max(s.xs for s in lw)) + 1)
    mt = torch.from_numpy(m_ref).cuda()

    def corr(a):
        a = a[zs, xs_].double()
        b = mt[zs, xs_]
        return float(torch.sum(a * b) / torch.linalg.vector_norm(a)
                     / torch.linalg.vector_norm(b))
    out = {
        "metric": "split-step Born+adjoint Gpt-steps/s",
        "value": round(pts / total / 1e9, 3),
        "unit": "Gpt-steps/s",
        "n_gpus": 1,
        "steps": len(windows),
        "warmup": 0,
        "ms_per_step": round(float(np.mean(lat)) * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ssf2d-256x1024 (Marmousi stand-in): "
                               f"{len(windows)} windows of 5 shots sliding "
                               f"by 3 over {len(need)} shots, 96 receivers, "
                               f"{nw} frequencies {w.fmin}-{w.fmax} Hz, 8 CG "
                               "iterations, "
                               + ("nonlinear FD data (true minus migration "
                                  "velocity, top-muted)" if nonlinear else
                                  "two-way FD Born data")
                               + " + 1 % noise"
                               + (", illumination preconditioner"
                                  if args.ssf_precond else "")
                               + (", correction-regularised recursion"
                                  if args.ssf_regularize else ""),
                   "model": [nz, nx]},
        "s_per_window": {"mean": round(float(np.mean(lat)), 4),
                         "p50": round(float(np.percentile(lat, 50)), 4),
                         "max": round(float(np.max(lat)), 4),
                         "chain_total_s": round(total, 3)},
        "roofline": {
            "bound": "alu",
            "kernel": f"{dom} (k_ssf_{dom})",
            "achieved": round(roof[dom]["tflops"], 2),
            "peak": 157.3,
            "unit": "TFLOP/s",
            "frac": round(roof[dom]["tflops"] / 157.3, 4),
            "traffic": (int(TRAFFIC_SSF[dom])
                        if kernel_sources_hash(("ssf.hip", "ssf_kernels.h"))
                        == TRAFFIC_SSF["sources_sha256_16"] else None),
            "avg_launch_us": round(roof[dom]["avg_us"], 1),
            "algorithmic_flops_per_launch": roof[dom]["flops"],
            "hbm": {"algorithmic_bytes_per_launch": roof[dom]["bytes"],
                    "achieved_GBs": round(roof[dom]["gbs"], 1)},
            "other": {k: {"avg_launch_us": round(v["avg_us"], 1),
                          "achieved_TFLOPs": round(v["tflops"], 2),
                          "achieved_GBs": round(v["gbs"], 1)}
                      for k, v in roof.items() if k != dom},
            "image_sum": {"avg_launch_us": round(sum_us, 1),
                          "achieved_GBs": round(sum_bytes / sum_us / 1e3,
                                                1)},
        },
        "kernels": {k: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3,
                                                          1)}
                    for k, v in ks.items()},
        "quality": {"final_s_over_s0": round(last["s_norm"]
                                             / last["s0_norm"], 4),
                    "final_r_norm": last["r_norm"],
                    "corr_chain_image": round(corr(image), 4),
                    "corr_last_window_migration": round(corr(mig), 4),
                    "zone_columns": [xs_.start, xs_.stop]},
        "device_bytes": mem,
    }
    log(f"ssf: {len(windows)} windows in {total:.2f}s; kernels {ks}")
    if not args.no_cpu_baseline:
        from oracle.ssf import SsfProblem, SsfShot
        # the first window's shots over the whole band: 10-30 s of FP64
        # work on current host cores (each shot's Born weights untimed)
        nf = nw
        sample = [w.shots[i] for i in windows[0]]
        prob = SsfProblem(w.vel.astype(np.float32).astype(np.float64), w.dx,
                          w.dz, w.nt, w.dt, (k0 - 0.25) * df,
                          (k0 + nf - 0.75) * df, w.ntap,
                          [SsfShot(s.xs, s.rec, s.f0) for s in sample])
        m64 = w.m_true.astype(np.float32).astype(np.float64)
        tc = 0.0
        for i in range(len(sample)):
            W = prob.weights(i)
            t = time.perf_counter()
            D = prob.born_shot(i, m64, W)
            prob.adjoint_shot(i, D, W)
            tc += time.perf_counter() - t
            del W, D
        out["cpu_baseline"] = {
            "value": round(2 * len(sample) * nf * nz * nx / tc / 1e9, 5),
            "unit": "Gpt-steps/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the first window's {len(sample)} shots, all {nf} "
                      f"frequencies: one Born and one adjoint application "
                      f"each (source march untimed), FP64 numpy (FFTs and "
                      f"elementwise work on one thread), {tc:.1f}s",
        }
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                          "--gpus must be 1 (multi-GPU sharding by shot is "
                          "a design note, not implemented)"}))
        sys.exit(2)
    import torch

    import paper_1801_00819_amd as P
    import synth

    torch.cuda.set_device(0)
    if args.workload == "3d":
        return bench_3d(args, P, synth, torch)
    if args.workload == "autograd":
        return bench_autograd(args, P, synth, torch)
    if args.workload == "stream":
        return bench_stream(args, P, synth, torch)
    if args.workload == "ssf":
        return bench_ssf(args, P, synth, torch)
    w = synth.faulted2d_512x1024()
    Q, S = w.Q, w.S
    nshots = len(w.shots)
    nrec = w.shots[0].nrec
    nt = w.nt
    pz, px = w.nz + 2 * w.nb, w.nx + 2 * w.nb
    npad, nint = pz * px, w.nz * w.nx
    vel = w.vel.astype(np.float32)
    m_true = torch.from_numpy(w.m_true.astype(np.float32)).cuda()

    if args.ops_only:
        ops_only(P, w, vel, m_true)
        return

    # ---- setup (untimed): data d = A m_true + 1% noise, lambda ----------
    t_setup = time.perf_counter()
    ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, nt, nrec, Q, w.h, w.dt, 0.0,
                      vel, device=True)
    ctx.set_tuning(*DEFAULT_TUNING)
    data = torch.empty((nshots, nt, nrec), dtype=torch.float32, device="cuda")
    for b in range(0, nshots, Q):
        ids = list(range(b, min(b + Q, nshots)))
        for i in ids:
            s = w.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
        d = ctx.apply_born(m_true)
        data[ids[0]:ids[-1] + 1] = d.view(len(ids), nt, nrec)
        for i in ids:
            ctx.downdate(i)
    rms = float(torch.sqrt(torch.mean(data.double() ** 2)))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1001)
    data += 0.01 * rms * torch.randn(data.shape, generator=gen,
                                     device="cuda")
    win0 = w.windows()[0]
    for i in win0:
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
    x = torch.from_numpy(synth.gaussian(w.model_shape, 2002).astype(
        np.float32)).cuda()
    x /= torch.linalg.vector_norm(x)
    norm = 0.0
    for _ in range(8):
        y = ctx.apply_adjoint(ctx.apply_born(x))
        norm = float(torch.linalg.vector_norm(y.double()))
        x = y / norm
    lam = w.lam_rel * norm
    ctx.close()
    torch.cuda.synchronize()
    log(f"setup: data + lambda {time.perf_counter() - t_setup:.1f}s "
        f"(||A^T A|| ~ {norm:.4e}, lambda = {lam:.4e})")

    # ---- the chain ---------------------------------------------------------
    ctx = P.brls_open(2, w.nz, 1, w.nx, w.nb, nt, nrec, Q, w.h, w.dt, lam,
                      vel, device=True)
    ctx.set_exec(P.BRLS_EXEC_GRAPH)
    windows = w.windows()
    held = []
    image = torch.empty(w.model_shape, dtype=torch.float32, device="cuda")

    def step(k):
        win = windows[k % len(windows)]
        for i in list(held):  # rank-S downdate
            if i not in win:
                ctx.downdate(i)
                held.remove(i)
        for i in win:  # rank-S update
            if i not in held:
                s = w.shots[i]
                ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
                held.append(i)
        st = ctx.solve_window(args.iters)
        ctx.image(image)
        return st

    ctx.set_tuning(*DEFAULT_TUNING)
    if args.autotune:
        for i in win0:
            s = w.shots[i]
            ctx.update(i, s.src, s.rec, s.nt, s.f0, data[i])
            held.append(i)
        t = time.perf_counter()
        best = ctx.autotune()
        log(f"autotune: {ctx.get_tuning()} ({P.tile_variants()[best]}) in "
            f"{time.perf_counter() - t:.1f}s")
    tuning = ctx.get_tuning()

    nwin = args.warmup + args.steps
    if nwin > len(windows):
        log(f"note: {nwin} steps > {len(windows)} windows; the chain wraps")
    for k in range(args.warmup):
        st = step(k)
        log(f"warmup step {k}: {st}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.warmup, nwin):
        stats.append(step(k))
        log(f"step {k}: iters={stats[-1]['iters']} "
            f"s={stats[-1]['seconds']:.3f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ops = sum(2 * (1 + s["iters"]) for s in stats)
    updates = ops * Q * npad * (nt - 1)
    value = updates / elapsed / 1e9
    ms_per_step = elapsed / args.steps * 1e3

    out = {
        "metric": "Born+adjoint Gpt-updates/s",
        "value": round(value, 3),
        "unit": "Gpt-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "faulted2d-512x1024: 64 shots x 1024 receivers, "
                        "nt=3000, window 8 shots sliding by 4, 20 CG iters",
            "padded_grid": [pz, px],
            "window_shots": Q,
            "slide": S,
            "cg_iters": args.iters,
            "exec": "graph",
            "launch": tuning,
        },
        "s_per_window": round(elapsed / args.steps, 4),
        "cg_scalars": "f64",
    }
    if args.only_steps:
        print(json.dumps(out), flush=True)
        ctx.close()
        return

    # ---- roofline of the dominant kernel (event-timed launches) ----------
    ctx.set_exec(P.BRLS_EXEC_BATCHED)
    ctx.kernel_timing(True)
    dwin = ctx.apply_born(m_true)
    ctx.apply_adjoint(dwin)
    ks = ctx.kernel_stats()
    ctx.kernel_timing(False)
    # the same applications replayed from their graphs (two concurrent
    # launch chains), each timed as a whole with events on the stream
    ctx.set_exec(P.BRLS_EXEC_GRAPH)
    ctx.apply_born(m_true)
    ctx.apply_adjoint(dwin)  # capture outside the timing
    ctx.kernel_timing(True)
    ctx.apply_born(m_true)
    ctx.apply_adjoint(dwin)
    kg = ctx.kernel_stats()
    ctx.kernel_timing(False)
    var = tuning["variant"]
    steps = 2 if P.tile_variants()[var][3] >= 3 else 1  # steps per launch
    roof = {}
    for kind, name in (("born", "born_step"), ("adjoint", "adjoint_step")):
        n, ms = ks[name]
        avg_s = ms / n / 1e3
        pb = tuning["born_per_block" if kind == "born" else "adj_per_block"]
        ngroups = (Q + pb - 1) // pb
        units = Q * npad * steps  # padded point-steps of one launch
        byt = int(round(point_step_bytes(kind, pb) * units))
        least = algorithmic_bytes(kind, Q, ngroups, npad, nint, nrec, steps)
        roof[kind] = dict(avg_us=avg_s * 1e6, bytes=byt, units=units,
                          gbs=byt / avg_s / 1e9, least=least,
                          least_gbs=least / avg_s / 1e9)
    dom = max(roof, key=lambda k: roof[k]["avg_us"])
    r = roof[dom]
    kname = KERNEL_NAME[P.tile_variants()[var][3]]
    pb_dom = tuning["born_per_block" if dom == "born" else "adj_per_block"]
    how = f"{pb_dom} shots per work item"
    if dom == "adjoint" and kname == "k_march2t" and pb_dom in (4, 8):
        kname = "k_march2t_coop"
        how = (f"cooperative blocks of {pb_dom} wavefronts, one shot each, "
               "image contributions summed in LDS")
    elif kname == "k_march2s" and pb_dom > 1:
        how = (f"blocks of {pb_dom} wavefronts marching one segment, one "
               "shot each" + (", image contributions summed in LDS"
                              if dom == "adjoint" else ""))
    traffic = measured_traffic(dom, tuning)
    out["roofline"] = {
        "bound": "hbm",
        "kernel": f"{dom} launch ({kname}, tile {P.tile_variants()[var]}, "
                  f"{how}, {steps} time step(s) per launch)",
        "achieved": round(r["gbs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(r["gbs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_GBs": (round(traffic / (r["avg_us"] * 1e-6) / 1e9, 1)
                        if traffic else None),
        "avg_launch_us": round(r["avg_us"], 2),
        "algorithmic_bytes_per_launch": r["bytes"],
        "bytes_basis": f"{point_step_bytes(dom, pb_dom):g} B per padded "
                       f"point, step and shot x {r['units']} point-step-"
                       "shots per launch",
        # what a launch must move at minimum when it takes `steps` steps
        # (fields read and written once per launch): the tighter count
        "least_bytes_per_launch": r["least"],
        "least_frac": round(r["least_gbs"] / HBM_PEAK_GBS, 4),
        "other": {k: {"avg_launch_us": round(v["avg_us"], 2),
                      "achieved_GBs": round(v["gbs"], 1),
                      "frac": round(v["gbs"] / HBM_PEAK_GBS, 4)}
                  for k, v in roof.items() if k != dom},
    }
    # whole applications in the timed configuration: graph replay with
    # the window's shot groups in two concurrent chains of launches; the
    # same bytes per two-step level over the application's time per level
    levels = (nt - 1 + steps - 1) // steps
    eff = {}
    for kind, name in (("born", "born_graph"), ("adjoint", "adjoint_graph")):
        n, ms = kg[name]
        per_level = ms / n / 1e3 / levels
        eff[kind] = {"application_ms": round(ms / n, 2),
                     "us_per_level": round(per_level * 1e6, 2),
                     "achieved_GBs": round(roof[kind]["bytes"] / per_level
                                           / 1e9, 1),
                     "frac": round(roof[kind]["bytes"] / per_level / 1e9
                                   / HBM_PEAK_GBS, 4)}
    out["roofline"]["effective"] = {
        "chains": ctx.get_chains(), "levels_per_application": levels,
        "note": "graph-replayed applications, event-timed whole; the "
                "per-launch figures above run one chain with per-launch "
                "events",
        **eff}
    log(f"roofline: {roof}; effective {eff}")

    # ---- plain per-shot launches, same operator pair ------------------
    if not args.no_plain:
        res = {}
        for mode, name in ((P.BRLS_EXEC_PLAIN, "plain"),
                           (P.BRLS_EXEC_GRAPH, "graph")):
            ctx.set_exec(mode)
            ctx.apply_born(m_true)  # graph capture outside the timing
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.apply_born(m_true)
            ctx.apply_adjoint(dwin)
            torch.cuda.synchronize()
            res[name] = time.perf_counter() - t
        pair_updates = 2 * Q * npad * (nt - 1)
        out["operator_pair"] = {
            k: {"seconds": round(v, 4),
                "Gpt_updates_per_s": round(pair_updates / v / 1e9, 2)}
            for k, v in res.items()}
        log(f"operator pair: {out['operator_pair']}")
    ctx.close()

    # ---- s per window at a fixed CG residual ----------------------------
    if args.fr_windows > 0:
        out["fixed_residual"] = fixed_residual(args, P, w, data, lam, vel,
                                               torch)
        log(f"fixed residual: {out['fixed_residual']}")

    # ---- one window through host pointers (PCIe-inclusive) --------------
    if not args.no_host_window:
        out["host_pointers"] = host_window(args, P, w, data, lam, vel,
                                           torch)
        log(f"host pointers: {out['host_pointers']}")

    # ---- the launch-bound 64 x 64 chain in every execution mode ---------
    if not args.no_small_chain:
        out["small_chain"] = small_chain(P, synth, torch)
        log(f"64x64 chain: {out['small_chain']}")

    # ---- CPU baseline: the FP64 oracle on a bounded sample -------------
    if not args.no_cpu_baseline:
        import oracle
        ns, nsh = args.cpu_sample_nt, args.cpu_sample_shots
        shots = [synth.Shot(i, w.shots[i].src, w.shots[i].rec, ns,
                            w.shots[i].f0) for i in range(nsh)]
        grid = oracle.Grid(2, w.nz, 1, w.nx, w.nb, w.h, w.dt)
        prob = oracle.Problem(grid, vel.astype(np.float64), shots)
        m64 = w.m_true.astype(np.float64)
        t = time.perf_counter()
        for i in range(nsh):
            d = prob.born_shot(i, m64)
            prob.adjoint_shot(i, d)
        tc = time.perf_counter() - t
        cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
        out["cpu_baseline"] = {
            "value": round(2 * nsh * npad * (ns - 1) / tc / 1e9, 4),
            "unit": "Gpt-updates/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"{nsh} shots, nt={ns} (of {nt}), one Born + one "
                      f"adjoint application each, FP64, {tc:.1f}s",
        }
        if "small_chain" in out:
            out["cpu_baseline"]["small_chain"] = oracle_small_chain(synth)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
