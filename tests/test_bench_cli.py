"""Host-side parts of the benchmark: the one-GPU refusal and the
algorithmic-bytes arithmetic behind the roofline line (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_adjoint_algorithmic_bytes_of_the_headline_launch():
    """One two-step adjoint launch over the 8-shot window of the 512 x 1024
    model (592 x 1104 padded, 1024 receivers, two groups of 4 shots): per
    shot u, v read and written (16 B per padded point) and per step its
    Born-source frame (4 B per model point) and receiver samples (4 B); per
    group the medium (4 B per padded point) and the float64 image
    accumulator read and written (16 B per model point)."""
    sys.path.insert(0, ROOT)
    import bench
    npad, nint, nrec = 592 * 1104, 512 * 1024, 1024
    per_shot = 16 * npad + 2 * (4 * nint + 4 * nrec)
    per_group = 4 * npad + 16 * nint
    want = 8 * per_shot + 2 * per_group
    assert want == 139282432
    assert bench.algorithmic_bytes("adjoint", 8, 2, npad, nint, nrec,
                                   steps=2) == want
    # Born: the model vector (4 B per model point) instead of the
    # accumulator, one group per shot
    born = 8 * per_shot + 8 * (4 * npad + 4 * nint)
    assert bench.algorithmic_bytes("born", 8, 8, npad, nint, nrec,
                                   steps=2) == born


def test_point_step_bytes_of_the_headline_launches():
    """The roofline's byte basis: per padded point, time step and shot,
    Born 16 + 8/B and adjoint 16 + 4/B bytes; one two-step launch over the
    8-shot window of the 592 x 1104 padded grid is 10 457 088 point-steps,
    i.e. 177.8 MB for the adjoint in groups of 4 shots and 251.0 MB for
    Born with one shot per work item."""
    sys.path.insert(0, ROOT)
    import bench
    units = 8 * 592 * 1104 * 2
    assert units == 10457088
    assert bench.point_step_bytes("adjoint", 4) == 17.0
    assert bench.point_step_bytes("born", 1) == 24.0
    assert round(bench.point_step_bytes("adjoint", 4) * units) == 177770496
    assert round(bench.point_step_bytes("born", 1) * units) == 250970112
