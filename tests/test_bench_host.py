"""Host-side pieces of bench.py (no GPU): the one-GPU guard, the
algorithmic operation count per interaction over the benchmark geometries'
element mix, the source hash that ties the stored counter figures to the
evaluation kernel's code (a comment edit keeps it, a code edit changes it),
the pointwise relative difference reported for the mixed path, and the
paper's own figures carried on the line as context."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_flops_of_the_benchmark_mixes():
    from synth import gem_cell, thgem_double
    for g, n_rect, n_tri, f_want in ((thgem_double(), 2688, 38912, 101.55076923076923),
                                     (gem_cell(), 128, 7936, 100.38095238095238)):
        kind = np.asarray(g.kind)
        assert (int((kind == 0).sum()), int((kind == 1).sum())) == (n_rect, n_tri)
        f = (n_rect * bench.ALG_FLOPS_RECT + n_tri * bench.ALG_FLOPS_TRI) / g.n
        assert abs(f - f_want) < 1e-9


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2606_24154_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.EVAL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2606_24154_amd", "csrc", name), csrc / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.eval_source_sha16()
    f = csrc / "panel_fp64.hpp"
    text = f.read_text()
    f.write_text("// a new comment line\n/* and a block\n   comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.eval_source_sha16() == h0
    f.write_text(text.replace("constexpr double kFarDiam = 5.0;", "constexpr double kFarDiam = 6.0;"))
    assert bench.eval_source_sha16() != h0


def test_rel_diff():
    ref = [np.array([1.0, -2.0, 1e-9]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 2.0, 0.0]),
           np.array([0.0, 0.0, 1e-12])]
    got = [ref[0] * (1 + np.array([1e-7, -3e-7, 0.5])), ref[1] + np.array([0.0, 4e-7, 0.0]), ref[2].copy(),
           ref[3].copy()]
    ephi, eE = bench.rel_diff(got, ref)
    # the third point lies below 1e-3 of the largest magnitude and is not counted
    assert abs(ephi - 3e-7) < 1e-15
    assert abs(eE - 2e-7) < 1e-15


def test_paper_context_serialises():
    ctx = json.loads(json.dumps(bench.PAPER_CONTEXT))
    assert "T1000" in ctx["hardware"] and "Xeon" in ctx["hardware"]
    t = ctx["total_solve_min"]
    assert abs(t["cpu_1_thread"] / t["hybrid_16_threads_gpu"] - t["speedup_vs_serial"]) < 0.01


def test_point_charge_reference_matches_oracle():
    """The host point-charge sum that serves as the line-charge benchmark's
    accuracy reference agrees with the oracle's Coulomb sum (self pairs and
    coincident charges skipped in both)."""
    import oracle
    from synth import charge_cloud
    xyz, q = charge_cloud([0.0, 0.0, 0.0], 20e-6, 3000, seed=8)
    xyz[7] = xyz[3]  # a coincident pair
    idx = np.array([0, 3, 7, 11, 2999])
    got = bench.point_charge_field(xyz, q, idx, chunk=2)
    want = oracle.coulomb(xyz[idx], xyz, q, idx)[:, 1:]
    scale = np.linalg.norm(want, axis=1)
    assert np.all(np.linalg.norm(got - want, axis=1) <= 1e-12 * scale)
