"""Writes the stored expected values of the full-size parity tests.  Calls
only the oracle (and the seeded input generators); no value comes from the
GPU path.  Run from the repository root:

    python tests/golden/make_golden.py gem       # ~30 min on 8 threads
    python tests/golden/make_golden.py traj      # ~25 min on 8 threads

gem:  the single-GEM cell (8064 elements, copies +-5): the oracle's full
      influence matrix (Eq. Matrix), its solution sigma (LU with two steps
      of FP64 refinement), and phi, E at 256 of the cell's seeded
      evaluation points (Eqs. Potential/Field).
traj: the reduced space-charge trajectory: the same cell with copies +-1,
      4096 charges (+-e alternating) from the seeded 20 um Gaussian at the
      hole centre, 20 steps of the dynamic loop (Algorithm 4 with point
      charges, Algorithm 2's sum; re-solve at steps 0 and 10, dt = 1 ps,
      mobility 1e-4 m^2/Vs): for 1024 sampled charges, positions and the
      field at the charges after steps 0, 9, 10 and 19 (around each
      re-solve and at the end), at every step the field's magnitude and the
      sum of the magnitudes of the charge-charge terms (the scale of the
      FP32 pair terms' error), and sigma after each re-solve.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import charge_cloud, gem_cell, gem_eval_points  # noqa: E402

GEM_POINTS = 256
TRAJ_CHARGES = 4096
TRAJ_STEPS = 20
TRAJ_KEEP_STEPS = (0, 9, 10, 19)
TRAJ_SAMPLE = 1024


def log(msg):
    print(f"[golden] {msg}", flush=True)


def make_gem():
    g = gem_cell()
    t0 = time.time()
    A = oracle.assemble(g)
    log(f"gem: assembly {g.n} x {g.n} x {g.images.count} copies in {time.time() - t0:.0f} s")
    b = g.rhs()
    sigma = oracle.solve_refined(A, b)
    resid = np.linalg.norm(A @ sigma - b) / np.linalg.norm(b)
    pts = gem_eval_points(g, 1_000_000, seed=1)
    idx = np.random.default_rng(11).choice(len(pts), GEM_POINTS, replace=False)
    idx.sort()
    t0 = time.time()
    f = oracle.eval_points(g, sigma, pts[idx])
    log(f"gem: {GEM_POINTS} points in {time.time() - t0:.0f} s; relative residual {resid:.2e}")
    np.savez(os.path.join(HERE, "gem_cell_fp64.npz"), sigma=sigma, point_index=idx, points=pts[idx],
             fields=f, rel_residual=resid)


def make_traj():
    g = gem_cell(n_images=1)
    t0 = time.time()
    A = oracle.assemble(g)
    log(f"traj: assembly {g.n} x {g.n} x {g.images.count} copies in {time.time() - t0:.0f} s")
    b0 = g.rhs()
    centre = [0.5 * (g.images.a1[0] + g.images.a2[0]), 0.5 * g.images.a2[1], 0.0]
    xyz, q = charge_cloud(centre, 20e-6, TRAJ_CHARGES, seed=3)
    params = oracle.SpaceChargeParams(dt=1e-12, mobility=1e-4, resolve_every=10)
    pos, E, sig, pair_abs = [], [], [], []
    sigma = None
    x = xyz.copy()
    sample = np.sort(np.random.default_rng(17).choice(TRAJ_CHARGES, TRAJ_SAMPLE, replace=False))
    for k in range(TRAJ_STEPS):
        t0 = time.time()
        # the charge-charge terms' magnitudes at the start-of-step positions
        _, ab = oracle.coulomb(x[sample], x, q, sample, with_abs=True)
        pair_abs.append(ab)
        x, sigma, e = oracle.spacecharge_step(g, A, b0, sigma, x, q, k, params)
        pos.append(x)
        E.append(e)
        if k % params.resolve_every == 0:
            sig.append(sigma)
        log(f"traj: step {k} in {time.time() - t0:.0f} s")
    keep = np.array(TRAJ_KEEP_STEPS)
    np.savez(os.path.join(HERE, "gem_cell_trajectory.npz"), steps=keep, sample=sample,
             positions=np.stack(pos)[keep][:, sample], fields=np.stack(E)[keep][:, sample], sigma=np.stack(sig),
             field_norm=np.linalg.norm(np.stack(E)[:, sample], axis=2), pair_abs=np.stack(pair_abs),
             n_steps=TRAJ_STEPS, n_charges=TRAJ_CHARGES, dt=params.dt, mobility=params.mobility,
             resolve_every=params.resolve_every)


if __name__ == "__main__":
    what = sys.argv[1:] or ["gem", "traj"]
    if "gem" in what:
        make_gem()
    if "traj" in what:
        make_traj()
