"""Host checks of the seeded workload generators (no GPU): the own-cell
correction layout, and the box blocks shared per box class (Section 4 reuses
one set of box corrections for every box of a size)."""
import numpy as np

from vp_workloads import generators as gen


def _blocks(cell_ptr, rowptr, col, val):
    out = []
    for k in range(len(cell_ptr) - 1):
        a, b = int(cell_ptr[k]), int(cell_ptr[k + 1])
        lo, hi = int(rowptr[a]), int(rowptr[b])
        assert hi - lo == (b - a) ** 2
        # every row lists exactly the cell's own nodes
        assert np.array_equal(col[lo:hi].reshape(b - a, b - a), np.tile(np.arange(a, b), (b - a, 1)))
        out.append(val[lo:hi])
    return out


def test_own_cell_csr_shared_classes():
    cell_ptr = np.array([0, 64, 128, 173, 237, 301, 346, 410], np.int64)
    cls = np.array([0, 0, -1, 1, 0, -1, 1], np.int64)
    rowptr, col, val = gen.own_cell_csr(cell_ptr, 5, cell_class=cls)
    b = _blocks(cell_ptr, rowptr, col, val)
    assert np.array_equal(b[0], b[1]) and np.array_equal(b[0], b[4])
    assert np.array_equal(b[3], b[6])
    assert not np.array_equal(b[0], b[3])
    assert not np.array_equal(b[2], b[5][:b[2].size])  # class -1 cells keep their own values
    # class blocks come from their own stream; unshared cells are the plain draw
    plain = gen.own_cell_csr(cell_ptr, 5)[2]
    lo, hi = int(rowptr[128]), int(rowptr[173])
    assert np.array_equal(val[lo:hi], plain[lo:hi])
    assert np.array_equal(b[0], np.random.default_rng([5, 1]).normal(0.0, 1e-3, 64 * 64))
    assert abs(val.std() / 1e-3 - 1.0) < 0.05


def test_own_cell_csr_unshared_default():
    cell_ptr = np.arange(0, 4 * 64 + 1, 64, dtype=np.int64)
    rowptr, col, val = gen.own_cell_csr(cell_ptr, 9)
    b = _blocks(cell_ptr, rowptr, col, val)
    assert len({bytes(x.tobytes()) for x in b}) == 4
