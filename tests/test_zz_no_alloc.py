"""brls_apply_adjoint_static (no device allocation in the call) against
brls_apply_adjoint through the C ABI: two calls in a row on one context,
the second on a smaller window, each equal to the existing entry point's
result (bitwise with the same batched launches; within the operator bar of
the oracle). A window whose accumulators exceed the static scratch is
refused."""
import numpy as np
import pytest

import synth
from gpu_helpers import add_shot, f32, open_ctx, oracle_problem, rel

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5


def _residual(w, idx, seed):
    return np.concatenate([
        f32(synth.gaussian((w.shots[i].nt, w.shots[i].nrec), seed + i))
        .ravel() for i in idx])


def test_static_adjoint_matches_adjoint_twice():
    import bench
    import paper_1801_00819_amd as P
    w = synth.layers2d_64x64()
    prob = oracle_problem(w)
    ctx = open_ctx(w, q_max=4)
    ctx.set_tuning(*bench.DEFAULT_TUNING)
    ctx.set_exec(P.BRLS_EXEC_BATCHED)
    for idx, seed in (([0, 1, 2, 3], 500), ([1, 2], 600)):
        for i in list(ctx.window()):
            if i not in idx:
                ctx.downdate(i)
        for i in idx:
            if i not in ctx.window():
                add_shot(ctx, w, i)
        r = _residual(w, idx, seed)
        want = ctx.apply_adjoint(r)
        got = ctx.apply_adjoint_static(r)
        print(f"window {idx}: static vs adjoint max |diff| "
              f"{np.max(np.abs(got - want)):.3e}", flush=True)
        assert np.array_equal(got, want)
        parts, off = [], 0
        for i in idx:
            n = w.shots[i].nt * w.shots[i].nrec
            parts.append(r[off:off + n].reshape(w.shots[i].nt,
                                                w.shots[i].nrec)
                         .astype(np.float64))
            off += n
        assert rel(got, prob.adjoint(parts, idx)) <= OP_TOL
    ctx.close()


def test_static_adjoint_refuses_oversized_window():
    import paper_1801_00819_amd as P
    w = synth.faulted2d_512x1024()
    ctx = open_ctx(w, q_max=8)
    # one shot per adjoint work item: 8 groups x 524288 doubles = 32 MiB
    ctx.set_tuning(18, 1, 0, 1, 0)
    for i in range(8):
        s = w.shots[i]
        ctx.update(i, s.src, s.rec, s.nt, s.f0, None)
    r = np.zeros(ctx.window_data_size(), np.float32)
    with pytest.raises(P.BrlsError) as e:
        ctx.apply_adjoint_static(r)
    assert e.value.code == -1 and "static scratch" in str(e.value)
    ctx.close()
