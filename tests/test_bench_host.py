"""Host-side checks of bench.py (no GPU): the one-GPU guard, the oracle
sample spread over the frequency range, and the counter-traffic lookup that
is only trusted for the kernel source it was measured on."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_oracle_sample_spans_the_frequency_range():
    """The sampled frequencies include the lowest (slowest inner solves) and
    the highest, and the sampled diagonals are the oracle's own."""
    w = synth.rect((12, 10), K=8, seed=5)
    cpu, ref = bench.cpu_baseline(w, 4)
    assert sorted(ref) == [0, 2, 5, 7]
    assert "k = [0, 2, 5, 7]" in cpu["sample"] and cpu["kind"] == "oracle"
    V, om, sig = synth.make_inputs(w)
    d = oracle.assemble_diag(V, om, sig, w.mu)
    for k, g in ref.items():
        dense = oracle.diag_inv_dense(w.dims, d[k], w.t)
        assert oracle.rel_err(g, dense) < 1e-12


@pytest.mark.parametrize("form", ["interface", "x"])
def test_traffic_is_reported_only_for_the_profiled_source(monkeypatch, form):
    t = bench.traffic_for("k_cocg_update", "square256", "mixed16", form)
    path = os.path.join(ROOT, "profiles", f"k_cocg_update_square256_mixed16_{form}.txt")
    fields = dict(ln.split(":", 1) for ln in open(path) if ":" in ln and not ln.startswith("#"))
    if fields["source_hash"].strip() == bench.kernel_source_hash():
        assert t == float(fields["traffic_bytes_per_launch"])
    else:
        assert t is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "not-the-profiled-source")
    assert bench.traffic_for("k_cocg_update", "square256", "mixed16", form) is None
    assert bench.traffic_for("k_cocg_update", "no-such-workload", "mixed16", form) is None
    assert np.isfinite(float(fields["traffic_bytes_per_launch"]))


def test_kernel_source_hash_ignores_comments_only():
    """The profiles are keyed by the kernels' code: a comment edit keeps them
    valid, a code edit does not."""
    src = 'int a = 1;  // note\n/* block\n   comment */\nconst char* s = "x // y";\n'
    assert bench.code_only(src) == 'int a = 1;\nconst char* s = "x // y";'
    assert bench.code_only(src.replace("note", "other").replace("block", "b")) == bench.code_only(src)
    assert bench.code_only(src.replace("= 1", "= 2")) != bench.code_only(src)
