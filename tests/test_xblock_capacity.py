"""Host check of the block-staged SpMV's LDS capacity (no GPU needed).

The traversal stages, per chunk of consecutive rows of one line of nodes, the
entries of x in the union of the rows' column boxes.  This test walks every
chunk of every line length, order, component count and Dirichlet choice on
the x axis, computes the staged count from the lattice geometry (a node's
columns are the free nodes that share a cell with it), and checks it against
the buffer size and chunk length the kernel source declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1708_01773_amd", "csrc", "fe_solve.hip")


def _constant(name):
    m = re.search(r"constexpr int %s = (\d+);" % name, open(SRC).read())
    assert m, name
    return int(m.group(1))


def _axis_boxes(n, k, lo_fixed, hi_fixed):
    """Per free lattice node along one axis: (first column, width) over free nodes."""
    N = n * k + 1
    lo, hi = (1 if lo_fixed else 0), (N - 2 if hi_fixed else N - 1)
    boxes = []
    for I in range(lo, hi + 1):
        cells = [c for c in (I // k - 1, I // k) if 0 <= c < n and c * k <= I <= (c + 1) * k]
        a, b = max(min(cells) * k, lo), min((max(cells) + 1) * k, hi)
        boxes.append((a, b - a + 1))
    return boxes


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("nc", [1, 2, 3])
def test_staged_box_fits_the_lds_buffer(k, nc):
    rows, cap = _constant("kXbRows"), _constant("kXbCap")
    across = (2 * k + 1) ** 2  # widest column box of the y and z lines
    worst = 0
    for n in range(1, 14):
        for lo_fixed in (False, True):
            for hi_fixed in (False, True):
                boxes = _axis_boxes(n, k, lo_fixed, hi_fixed)
                rpl = nc * len(boxes)
                for lr0 in range(0, rpl, rows):
                    lr1 = min(lr0 + rows, rpl)
                    (ca, _), (cb, wb) = boxes[lr0 // nc], boxes[(lr1 - 1) // nc]
                    worst = max(worst, nc * (cb + wb - ca) * across)
    bound = nc * ((rows - 1) // nc + 2 + 2 * k) * across
    assert worst <= bound <= cap, (worst, bound, cap)
