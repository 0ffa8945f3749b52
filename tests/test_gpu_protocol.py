"""The paper's transport protocol (Section 3.2) run on the GPU, against the oracle.

Each sweep point of ``paper_2302_09883_amd.protocol`` (level x threshold x
rule on the 128^2 transport test, float64) is a whole compressed run; the
oracle runs the same points patch by patch.  Per step, the number of stored
coefficients must agree (a keep / drop decision may differ only for a
coefficient within rounding of its threshold), and the final fields must agree
to round-off.  On the whole sweep: eps = 0 reproduces the uncompressed run,
the stored total is conserved, and the paper's trends hold (the ratio grows
with the threshold; the error against the exact solution is set by the
scheme at small thresholds).
"""
import sys

import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import transport_gaussian

from gpu_helpers import require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


POINTS = [(lev, thr, rule) for rule in ("constant", "accum", "capped") for lev in (1, 3, 5)
          for thr in (0.0, 0.0025, 0.01, 0.04)]


@pytest.mark.parametrize("level,thr,rule", POINTS)
def test_protocol_point_matches_oracle(level, thr, rule):
    from paper_2302_09883_amd import protocol as PR

    _say("protocol point", level, thr, rule)
    got = PR.run_point(level, thr, rule)
    g = O.Geometry(PR.N, PR.PATCH, O.BL53, level)
    run = O.CompressedRun(g, O.Scheme("fv_upwind", vel=PR.VEL, cfl=PR.CFL), thr, rule, np.float64)
    run.set_grid(transport_gaussian(PR.N, 0.0, PR.VEL, PR.LO, PR.HI)[None])
    want_nnz = []
    for _ in range(got["steps"]):
        run.step(1)
        want_nnz.append(int(run.nnz().sum()))
    d = np.abs(np.array(got["nnz_series"]) - np.array(want_nnz))
    # a flip needs a coefficient within a few ulps of its threshold
    assert d.max() <= 2, (d.max(), got["nnz_series"][-1], want_nnz[-1])
    sim = got["_field"]
    ref = run.grid()[0]
    assert np.max(np.abs(sim - ref)) <= 1e-9 * np.max(np.abs(ref)) + (thr * 4 if d.max() else 0.0)
    assert abs(got["ratio_final"] - run.ratio()) <= 0.01 * run.ratio()


def test_whole_sweep_trends():
    from paper_2302_09883_amd import protocol as PR

    _say("protocol sweep")
    res = PR.sweep()
    pts = res["points"]
    assert len(pts) == len(PR.LEVELS) * len(PR.THRESHOLDS) * len(PR.RULES)
    f0 = transport_gaussian(PR.N, 0.0, PR.VEL, PR.LO, PR.HI)
    # stored mass (trapezoid totals of the tiles = the grid sum) is conserved
    for p in pts:
        assert abs(p["total"] - f0.sum()) <= 1e-11 * f0.sum(), p
    for rule in PR.RULES:
        for lev in PR.LEVELS:
            row = sorted((p for p in pts if p["rule"] == rule and p["level"] == lev), key=lambda p: p["threshold"])
            # threshold 0 nullifies nothing: the run is the uncompressed one
            assert row[0]["threshold"] == 0.0 and row[0]["rel_l2_vs_plain"] <= 1e-12
            # the ratio does not fall as the threshold grows (Fig. 5)
            for a, b in zip(row[1:], row[2:]):
                assert b["ratio_mean"] >= 0.99 * a["ratio_mean"], (rule, lev, a["threshold"], b["threshold"])
            assert row[-1]["ratio_mean"] > row[0]["ratio_mean"]
    # at threshold 0 the error against the exact solution is the scheme's own
    base = res["l2_exact_uncompressed"]
    for p in pts:
        if p["threshold"] == 0.0:
            assert abs(p["l2_exact"] - base) <= 1e-9 * base
