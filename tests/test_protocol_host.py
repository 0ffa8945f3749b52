"""Host-side pieces of the transport protocol (Section 3.2), and its trends on the oracle."""
import numpy as np

from oracle import lbmz_oracle as O
from synth import transport_gaussian

from paper_2302_09883_amd import protocol as PR


def test_time_step_count():
    # dt = CFL h / max(alpha, beta) = 0.45 * (2/128) / 0.9 = 1/128, so t = 0.5 is 64 steps
    assert PR.steps_to(0.5, 128) == 64
    assert PR.steps_to(0.5, 256) == 128


def test_exact_solution_is_a_shift():
    # at t = 0.5 the centre moved by (0.45, 0.45) = 28.8 cells of h = 1/64
    f0 = transport_gaussian(128, 0.0)
    f1 = transport_gaussian(128, 0.5)
    assert f0.min() >= 1.0 and abs(f0.max() - (1 + np.exp(-30 * 2 * (1 / 128) ** 2))) < 1e-12
    assert np.allclose(f0.sum(), f1.sum(), rtol=1e-6)
    # a shift by whole cells is a roll: t = 32 h / 0.9 moves by 32 cells in x and y
    t = 32 * (2 / 128) / 0.9
    assert np.allclose(transport_gaussian(128, t), np.roll(f0, (32, 32), axis=(0, 1)), atol=1e-12)


def test_paper_l2_and_csr_bytes():
    a = np.zeros((128, 128))
    b = np.full((128, 128), 0.5)
    # (2/128)^2 * 128^2 * 0.25 = 4 * 0.25
    assert abs(PR.l2_paper(a, b) - 1.0) < 1e-12
    table = np.zeros((4, 1, 2), dtype=np.uint32)
    table[:, 0, 1] = [10, 0, 3 | O.MASK_BIT, 5]
    assert PR.csr_bytes(table, 65, 8) == 18 * 12 + 4 * 4 * 66


def test_oracle_trends_on_the_protocol():
    # the paper's Fig. 5 trend on a few points: more threshold, fewer
    # coefficients; and eps = 0 keeps the uncompressed result
    n = 128
    f0 = transport_gaussian(n, 0.0)[None]
    sch = O.Scheme("fv_upwind", vel=PR.VEL, cfl=PR.CFL)
    plain = f0.copy()
    for _ in range(16):
        plain = O.dense_step(plain, sch)
    ratios = []
    for thr in (0.0, 0.005, 0.04):
        run = O.CompressedRun(O.Geometry(n, 64, O.BL53, 4), sch, thr, O.RULE_CAPPED, np.float64)
        run.set_grid(f0)
        run.step(16)
        ratios.append(run.ratio())
        if thr == 0.0:
            assert np.max(np.abs(run.grid() - plain)) <= 1e-13
        assert abs(run.field_totals()[0] - f0.sum()) <= 1e-12 * f0.sum()
    assert ratios[0] < ratios[1] <= ratios[2]
