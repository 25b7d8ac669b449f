"""Pins of slice validation (Section 2.2): the three cases forced by hand-built probes."""
import numpy as np

from oracle import validate

LAM = np.array([-3.0, -2.5, -2.2, -1.0, -0.9, -0.1, 0.3, 0.8, 1.5, 2.7])


def nu(s):
    return int(np.sum(LAM < s))


def run(sigmas, thetas, resids, top=2.0):
    nus = [nu(s) for s in sigmas]
    return validate.validate(sigmas, nus, thetas, resids, top, nu(top))


def test_case_equal_counts_validates_everything():
    sig = [-2.0, 0.0, 1.0]
    th = [LAM[LAM < 0.0], LAM[(LAM > -2.0) & (LAM < 1.0)], LAM[(LAM > 0.0) & (LAM < 2.0)]]
    rs = [np.zeros(t.size) for t in th]
    out = run(sig, th, rs)
    assert [s["case"] for s in out["slices"]] == [validate.CASE_OK] * 4
    vals = [v[0] for v in out["validated"]]
    assert np.array_equal(vals, LAM[LAM < 2.0])
    # the tau split removes the duplicates that adjacent probes share
    assert len(vals) == len(set(vals))


def test_case_missing_is_flagged():
    sig = [-2.0, 0.0, 1.0]
    th = [LAM[LAM < -2.0], np.array([-0.1, 0.3]), LAM[(LAM > 0.0) & (LAM < 2.0)]]
    rs = [np.zeros(t.size) for t in th]
    out = run(sig, th, rs)
    # slice [-2, 0) holds -1.0, -0.9, -0.1 but the probes only report -0.1
    s1 = out["slices"][1]
    assert s1["n_exact"] == 3 and s1["n_cand"] == 1 and s1["case"] == validate.CASE_MISSING


def test_case_surplus_keeps_smallest_residuals():
    sig = [-2.0, 0.0, 1.0]
    th = [np.concatenate([LAM[LAM < 0.0], [-1.5]]), LAM[(LAM > -2.0) & (LAM < 1.0)],
          LAM[(LAM > 0.0) & (LAM < 2.0)]]
    rs = [np.zeros(t.size) for t in th]
    rs[0][-1] = 1e-3                                   # the spurious value is poorly converged
    out = run(sig, th, rs)
    s1 = out["slices"][1]
    assert s1["n_exact"] == 3 and s1["n_cand"] == 4 and s1["case"] == validate.CASE_TRIMMED
    vals = [v[0] for v in out["validated"]]
    assert -1.5 not in vals and np.array_equal(vals, LAM[LAM < 2.0])


def test_tau_tie_belongs_to_lower_probe():
    lam = np.array([-1.0, 0.0, 1.0])
    sig = [-0.5, 0.5]
    nus = [int(np.sum(lam < s)) for s in sig]
    th = [np.array([-1.0, 0.0]), np.array([0.0, 1.0])]    # both report the value at tau = 0
    rs = [np.array([0.0, 1e-14]), np.array([0.0, 0.0])]
    out = validate.validate(sig, nus, th, rs, 2.0, 3)
    src = [(v[0], v[2]) for v in out["validated"]]
    assert (0.0, 0) in src and (0.0, 1) not in src
    assert [s["case"] for s in out["slices"]] == [validate.CASE_OK] * 3


def test_end_slices_use_minus_infinity_and_top_boundary():
    sig = [-2.0, 1.0]
    th = [LAM[LAM < 1.0], LAM[(LAM > -2.0) & (LAM < 2.0)]]
    rs = [np.zeros(t.size) for t in th]
    out = run(sig, th, rs, top=2.0)
    assert out["slices"][0]["lo"] == -np.inf and out["slices"][0]["n_exact"] == nu(-2.0)
    assert out["slices"][-1]["hi"] == 2.0 and out["slices"][-1]["n_exact"] == nu(2.0) - nu(1.0)
