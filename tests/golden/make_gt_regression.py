"""Writes gt_regression.json: the oracle's error against the generators'
ground-truth tangents on helical scenes, noise-free and noisy, and the
fraction of points where its search reaches the dense brute-force optimum.

These are regression thresholds taken from the oracle's own runs (the paper
prints no such figure for synthetic data): tests/test_oracle_pins.py fails
when a change to the oracle makes the method measurably less accurate.
Run from the repository root:  python tests/golden/make_gt_regression.py
Calls only oracle/ and the seeded scene generator."""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gt_regression.json")


def axial(a, b):
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    return np.arctan2(c, np.abs(np.sum(a * b, axis=-1)))


def gt_case(name):
    """The helical scenes the thresholds are taken on (tiny recipe: 200
    helices, 12 views on a 120 degree arc, 256^2 f32, P = 3, 48 candidates,
    8 iterations, depth test on)."""
    rec = dict(scenegen.RECIPES["tiny"])
    rec["n_points"] = 4000
    if name == "helix_noise_free":
        rec.update(kappa=None, outliers=0.0, jitter=0.0)
    return rec


def bf_case(name):
    """Tiny brute-force scenes: 200 points on 40 helices, 4 views on a 120
    degree arc at 64^2, zero jitter; noise-free or von Mises kappa = 50."""
    rec = dict(scenegen.RECIPES["tiny"])
    rec.update(n_points=200, n_strands=40, n_views=4, res=64, arc_deg=120.0,
               outliers=0.0, jitter=0.0, kappa=None if name == "bf_noise_free" else 50.0)
    return rec


def run_gt(name, seed=0):
    rec = gt_case(name)
    sc = scenegen.make_scene(rec, seed)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth,
                      **scenegen.method_params(rec))
    d, c = o.fuse(sc.points)
    fin = np.isfinite(c)
    e = np.degrees(axial(d[fin], sc.gt[fin]))
    return dict(n=int(fin.sum()), mean_deg=float(e.mean()), median_deg=float(np.median(e)))


def run_bf(name, seed=3, n_points=100):
    rec = bf_case(name)
    sc = scenegen.make_scene(rec, seed)
    o = oracle.Oracle(sc.cams, sc.theta, sc.conf, depth=sc.depth, patch=3, n_candidates=48,
                      refine_iters=8, top_k=4)
    d, c = o.fuse(sc.points[:n_points])
    dense = oracle.lattice(1_000_000)
    ok = n = 0
    for i, p in enumerate(sc.points[:n_points]):
        if math.isinf(c[i]):
            continue
        n += 1
        ok += c[i] <= o.objective_many(p, dense).min() + 1e-4
    return dict(n=n, frac_at_optimum=ok / n)


def main():
    out = {"_note": "written by tests/golden/make_gt_regression.py from oracle runs"}
    for name in ("helix_noise_free", "helix_noisy"):
        out[name] = run_gt(name)
    for name in ("bf_noise_free", "bf_noisy"):
        out[name] = run_bf(name)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
