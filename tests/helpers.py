"""Shared test helpers (inputs only; no QLC arithmetic)."""
import numpy as np

from conftest import read_golden


def paper_histogram():
    """A histogram whose rank order reproduces the rows printed in Tables 3
    and 4 and the ordering named in the Implementation section: the named
    symbols take their printed ranks, the other symbols fill the remaining
    ranks in ascending symbol order, and rank r gets the distinct count
    10 * (256 - r)."""
    fixed = {}
    for r, s in read_golden("paper_ranking_order.txt"):
        fixed[int(r)] = int(s)
    for s, r, _code in read_golden("paper_table3_encoder_lut.txt"):
        fixed[int(r)] = int(s)
    rest = [s for s in range(256) if s not in fixed.values()]
    order = []
    it = iter(rest)
    for r in range(256):
        order.append(fixed[r] if r in fixed else next(it))
    h = np.zeros(256, dtype=np.uint64)
    for r, s in enumerate(order):
        h[s] = 10 * (256 - r)
    return h, order
