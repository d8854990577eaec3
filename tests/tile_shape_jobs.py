"""Jobs whose contraction plan uses every tall last-column shape (4 x 1 waves, 128 rows x 16, 48, 80
or 112 columns) and the 32-row shapes for short row tiles: a triatomic whose pair (0, 1) carries 23
functions per atom (529 = 4 x 128 + 17 pair rows: the 128-row shape, with a 17-row last tile) and whose
third atom carries n auxiliary functions, so that the pair grid's auxiliary columns (n + 2) leave a
last column tile of 12, 40, 70 or 100 columns.  Inputs only."""
import numpy as np

from conftest import MiniJob, Spec

# auxiliary count on the third atom -> launch shape (wm.wn.sc.wr) of its last column tile
TALL_CASES = {138: "2.1.1.4", 40: "2.3.1.4", 70: "2.5.1.4", 100: "2.7.1.4"}


def _aux_set(atom, count, z0):
    rows, l, k = [], 0, 0
    while len(rows) < count:
        for m in range(-l, l + 1):
            if len(rows) < count:
                rows.append([atom, l + 1 + (k % 2), l, m, z0 * 1.045 ** (len(rows) % 9) * 1.5 ** (k % 3)])
        l = (l + 1) % 4
        k += 1
    return rows


def _shells(a):
    rows = [[a, n, 0, 0, 0.7 + 0.3 * n + 0.1 * a] for n in range(1, 6)]
    rows += [[a, n, 1, m, 0.8 + 0.2 * n] for n in (2, 3) for m in (-1, 0, 1)]
    rows += [[a, 3, 2, m, 0.9] for m in range(-2, 3)] + [[a, 4, 3, m, 1.1] for m in range(-3, 4)]
    return rows


def tall_job(n_aux_third):
    xyz = np.array([[0.0, 0.0, 0.0], [1.9, 0.3, 0.2], [-0.5, 1.7, 0.4]])
    basis = _shells(0) + _shells(1) + [[2, 1, 0, 0, 1.5]]
    aux = _aux_set(2, n_aux_third, 1.9) + [[0, 1, 0, 0, 2.2], [1, 2, 1, 0, 1.8]]
    return MiniJob(xyz, [1.0, 1.0, 2.0], basis, aux, Spec(8, 8, 6, 4, 3))
