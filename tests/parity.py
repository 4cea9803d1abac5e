"""Parity protocol between the GPU library and the CPU oracle.

Directions are axial, so they are compared by the axial angle
atan2(|a x b|, |a . b|).  The search is a heuristic (a lattice argmin and a
pattern search), so it takes discrete decisions on floating-point costs; the
oracle takes them in binary64, the GPU in binary64 for view selection and
refinement and in binary32 for the lattice stage.  Per point:

  pass      axial angle(d_gpu, d_oracle) <= ANGLE_TOL
  near-tie  otherwise, if the two directions are equally good under the
            oracle's own objective: |J_o(d_gpu) - J_o(d_oracle)| <= COST_TOL
            (both sides: a GPU direction that is better than the oracle's is
            as much a disagreement as a worse one)
  fail      otherwise

Near-ties are allowed for at most MAX_TIE_FRAC of the points and failures
for at most MAX_FAIL_FRAC; both counts are printed by every parity test.
The GPU's reported cost must equal the oracle objective at the GPU's
direction: |cost_gpu - J_o(d_gpu)| <= COST_TOL for every point.

ANGLE_TOL = 1e-3 rad is the stated direction tolerance.  COST_TOL = 1e-5:
J is a mean of K values in [0, 1], each C |cos(.)| built from binary32
patch coefficients (relative rounding ~6e-8, so J errs by well under 1e-6)
and evaluated in binary64 for the reported cost.
"""
import numpy as np

ANGLE_TOL = 1e-3
COST_TOL = 1e-5
MAX_FAIL_FRAC = 1e-3
MAX_TIE_FRAC = 1e-3


def axial_angle(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    c = np.linalg.norm(np.cross(a, b), axis=-1)
    return np.arctan2(c, np.abs(np.sum(a * b, axis=-1)))


def compare(orc, points, d_gpu, c_gpu, d_o, c_o, angle_tol=ANGLE_TOL, cost_tol=COST_TOL):
    """Returns a dict of counts and the per-point classification."""
    d_gpu = np.asarray(d_gpu, np.float64)
    c_gpu = np.asarray(c_gpu, np.float64)
    inf_o = ~np.isfinite(c_o)
    inf_g = ~np.isfinite(c_gpu)
    res = {"n": len(points), "inf_mismatch": int(np.sum(inf_o != inf_g))}
    fin = ~inf_o & ~inf_g
    res["zero_dir_mismatch"] = int(np.sum(inf_g & (np.abs(d_gpu).sum(1) != 0)))
    ang = np.full(len(points), np.nan)
    ang[fin] = axial_angle(d_gpu[fin], d_o[fin])
    J_g = np.full(len(points), np.inf)
    if fin.any():
        J_g[fin] = orc.objective_each(points[fin], d_gpu[fin])
    cost_err = np.zeros(len(points))
    cost_err[fin] = np.abs(c_gpu[fin] - J_g[fin])
    dJ = np.zeros(len(points))
    dJ[fin] = J_g[fin] - np.asarray(c_o, np.float64)[fin]
    ok = fin & (ang <= angle_tol)
    tie = fin & ~ok & (np.abs(dJ) <= cost_tol)
    fail = fin & ~ok & ~tie
    res.update(
        n_finite=int(fin.sum()), n_pass=int(ok.sum()), n_tie=int(tie.sum()),
        n_fail=int(fail.sum()),
        max_cost_err=float(np.max(cost_err[fin])) if fin.any() else 0.0,
        n_cost_bad=int(np.sum(cost_err[fin] > cost_tol)),
        max_angle_pass=float(np.max(ang[ok])) if ok.any() else 0.0,
        max_angle=float(np.max(ang[fin])) if fin.any() else 0.0,
        median_angle=float(np.median(ang[fin])) if fin.any() else 0.0,
        max_abs_dJ=float(np.max(np.abs(dJ[fin]))) if fin.any() else 0.0,
    )
    res["fail_idx"] = np.nonzero(fail)[0]
    res["tie_idx"] = np.nonzero(tie)[0]
    res["cost_bad_idx"] = np.nonzero(fin & (cost_err > cost_tol))[0]
    return res


def summary(res):
    return {k: v for k, v in res.items() if not k.endswith("_idx")}


def assert_parity(res, max_fail_frac=MAX_FAIL_FRAC, max_tie_frac=MAX_TIE_FRAC,
                  max_cost_bad_frac=0.0):
    msg = summary(res)
    print("parity", msg, flush=True)
    n = max(1, res["n_finite"])
    assert res["inf_mismatch"] == 0, msg
    assert res["zero_dir_mismatch"] == 0, msg
    assert res["n_fail"] <= max_fail_frac * n, msg
    assert res["n_tie"] <= max_tie_frac * n, msg
    assert res["n_cost_bad"] <= max_cost_bad_frac * n, msg
