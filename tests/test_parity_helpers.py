"""Host logic of the parity helpers (no GPU)."""
import numpy as np

from tests.parity import tie_affected


def test_tie_flip_exempts_dependent_blocks_transitively():
    b = 16
    out_o = np.zeros((64, 64), np.uint8)
    out_g = out_o.copy()
    xh_o = {(0, 0): np.full((16, 16), 10.5), (2, 2): np.full((16, 16), 3.0),
            (3, 3): np.full((16, 16), 3.0)}
    info_o = [{"by": 0, "bx": 0, "round": 1}, {"by": 2, "bx": 2, "round": 2},
              {"by": 3, "bx": 3, "round": 3}]
    out_g[5, 5] = 1          # round 1 rounds a tie (10.5) the other way
    out_g[40, 40] = 7        # so block (2, 2) of round 2 differs, and (3, 3) reads it
    assert tie_affected(out_g, out_o, xh_o, info_o, b, 4, 24) == {(2, 2), (3, 3)}


def test_non_tie_difference_exempts_nothing():
    b = 16
    out_o = np.zeros((64, 64), np.uint8)
    out_g = out_o.copy()
    xh_o = {(0, 0): np.full((16, 16), 10.2), (2, 2): np.full((16, 16), 3.0)}
    info_o = [{"by": 0, "bx": 0, "round": 1}, {"by": 2, "bx": 2, "round": 2}]
    out_g[5, 5] = 1          # not a tie: a real error, which compare() reports
    assert tie_affected(out_g, out_o, xh_o, info_o, b, 4, 24) == set()
