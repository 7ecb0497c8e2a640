"""Seeded synthetic inputs for the volume-potential hot path.

This module is shared by the CPU oracle and the GPU library's tests and
benchmark.  It draws node sets, quadrature weights, densities, sparse
correction matrices and target samples, and holds none of the method's
arithmetic (no Green's function, no expansions, no sums over pairs).

Node/weight conventions follow the paper's smooth target-independent rule
(Section 3.2, eq. Tk_smooth_quad; Section 4.2, eq. Rk_box): every cell carries
a fixed reference rule mapped into physical space, and the FMM source
"charge" of node j is its weight times the density value there.  Box cells
use an 8x8 tensor Gauss-Legendre rule (the paper uses Chebyshev nodes with a
Clenshaw-Curtis rule; the workloads here fix Gauss-Legendre instead), with
weights w = w_xi * w_eta * (side/2)^2 so that the weights of one box sum to
its area.  Triangle cells are ordered before boxes, as the paper orders its
cell list (Section 3.1, eq. Ck_Tk_Bk).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "gauss_legendre_box_nodes",
    "uniform_grid",
    "gaussian_sum_density",
    "own_cell_csr",
    "sample_indices",
    "config0",
    "config1",
    "config2",
    "config3",
    "config4",
    "uniform_config",
    "star_radius",
    "chebyshev_roots",
    "fejer_weights",
    "OversampledWorkload",
    "oversampled_grid",
    "config5",
    "config6",
]


@dataclasses.dataclass
class Workload:
    """One evaluation problem.

    x, y, w       : node coordinates and smooth-rule weights, float64 [n]
    f             : densities, float64 [nbatch, n]
    tx, ty        : target coordinates [m], or None when targets are the nodes
    rowptr/col/val: correction matrix in CSR form, rows = targets, cols = nodes
                    (int64 [m+1], int32 [nnz], float64 [nnz]); None = no rows
    root          : (x0, y0, side) of the square the quadtree is built on
    sample        : target indices at which large problems are checked
    name/meta     : description
    """

    name: str
    x: np.ndarray
    y: np.ndarray
    w: np.ndarray
    f: np.ndarray
    tx: Optional[np.ndarray]
    ty: Optional[np.ndarray]
    rowptr: Optional[np.ndarray]
    col: Optional[np.ndarray]
    val: Optional[np.ndarray]
    root: tuple
    sample: Optional[np.ndarray]
    meta: dict

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def m(self) -> int:
        return self.n if self.tx is None else int(self.tx.shape[0])

    @property
    def nbatch(self) -> int:
        return int(self.f.shape[0])

    @property
    def self_targets(self) -> bool:
        return self.tx is None


@dataclasses.dataclass
class OversampledWorkload(Workload):
    """A box grid whose density is given at p x p interpolation nodes per box
    (the targets) and whose smooth rule sits at q x q upsampled nodes (the
    sources, x/y/w).  f is [nbatch, m] at the targets; the correction columns
    index those values.  Box b holds targets b p^2 .. and sources b q^2 .."""

    nbox: int = 0
    p_interp: int = 0
    q_interp: int = 0

    @property
    def n_in(self) -> int:
        return int(self.f.shape[1])


# --------------------------------------------------------------------------
# Node sets
# --------------------------------------------------------------------------

def gauss_legendre_box_nodes(order: int = 8):
    """Reference tensor Gauss-Legendre rule on [-1,1]^2.

    Returns (xi, eta, wref) of length order^2 with node a = jy*order + jx
    (x fastest).  Reference weights sum to 4.
    """
    t, wt = np.polynomial.legendre.leggauss(order)
    xi = np.tile(t, order)
    eta = np.repeat(t, order)
    wref = np.repeat(wt, order) * np.tile(wt, order)
    return xi, eta, wref


def uniform_grid(nbox_side: int, lo: float = -1.0, hi: float = 1.0, order: int = 8):
    """Uniform nbox_side x nbox_side grid of boxes on [lo,hi]^2.

    Box b = iy*nbox_side + ix (x fastest); node a within a box as in
    gauss_legendre_box_nodes; global node index j = order^2 * b + a.
    """
    h = (hi - lo) / nbox_side
    xi, eta, wref = gauss_legendre_box_nodes(order)
    ix = np.tile(np.arange(nbox_side), nbox_side)
    iy = np.repeat(np.arange(nbox_side), nbox_side)
    cx = lo + (ix + 0.5) * h
    cy = lo + (iy + 0.5) * h
    x = (cx[:, None] + 0.5 * h * xi[None, :]).ravel()
    y = (cy[:, None] + 0.5 * h * eta[None, :]).ravel()
    w = np.broadcast_to(wref * (0.5 * h) ** 2, (nbox_side * nbox_side, order * order)).ravel().copy()
    return x, y, w


def chebyshev_roots(n: int) -> np.ndarray:
    """Roots of T_n on [-1, 1], ascending: -cos((2i+1) pi / (2n))."""
    i = np.arange(n)
    return -np.cos((2 * i + 1) * np.pi / (2 * n))


def fejer_weights(n: int) -> np.ndarray:
    """Weights of Fejer's first rule on the n roots of T_n (ascending):
    w_j = (2/n) [1 - 2 sum_{k=1}^{n/2} cos(2 k theta_j) / (4k^2 - 1)],
    theta_j = (2j+1) pi / (2n); they integrate every polynomial of degree
    < n exactly over [-1, 1]."""
    j = np.arange(n)
    theta = (2 * j + 1) * np.pi / (2 * n)
    k = np.arange(1, n // 2 + 1)
    s = np.cos(2 * np.outer(theta, k)) / (4 * k * k - 1)
    w = (2.0 / n) * (1.0 - 2.0 * s.sum(axis=1))
    return w[::-1].copy()  # theta ascending is x descending: reverse for ascending roots


def oversampled_grid(nbox_side: int, p: int, q: int, lo: float = -1.0, hi: float = 1.0):
    """Box grid (box b = iy*nbox_side + ix) with p x p Chebyshev-root
    targets and q x q Chebyshev-root sources per box (node a = jy*n + jx, x
    fastest), source weights Fejer x Fejer x (side/2)^2 (they sum to the box
    area).  Returns (tx, ty, x, y, w)."""
    h = (hi - lo) / nbox_side
    ix = np.tile(np.arange(nbox_side), nbox_side)
    iy = np.repeat(np.arange(nbox_side), nbox_side)
    cx = lo + (ix + 0.5) * h
    cy = lo + (iy + 0.5) * h

    def nodes(n):
        r = chebyshev_roots(n)
        xi, eta = np.tile(r, n), np.repeat(r, n)
        return ((cx[:, None] + 0.5 * h * xi[None, :]).ravel(), (cy[:, None] + 0.5 * h * eta[None, :]).ravel())

    tx, ty = nodes(p)
    x, y = nodes(q)
    wq = fejer_weights(q)
    wref = np.repeat(wq, q) * np.tile(wq, q)
    w = np.broadcast_to(wref * (0.5 * h) ** 2, (nbox_side * nbox_side, q * q)).ravel().copy()
    return tx, ty, x, y, w


def config5(nbox_side: int = 64, p: int = 8, q: int = 16, f_seeds=(50,), csr_seed: Optional[int] = 51,
            sample_seed: Optional[int] = 150, nsample: int = 4096):
    """Oversampled boxes (the paper's twofold oversampling q = 2p): a
    nbox_side^2 grid on [-1,1]^2, the density at 8x8 Chebyshev-root
    interpolation nodes per box (the targets), the smooth rule at 16x16
    Chebyshev-root nodes with Fejer weights (the sources), own-box
    correction rows over the box's density values (one shared 64 x 64
    block).  Default 64 x 64 boxes: 262,144 targets, 1,048,576 sources."""
    tx, ty, x, y, w = oversampled_grid(nbox_side, p, q)
    f = np.stack([gaussian_sum_density(tx, ty, s)[0] for s in f_seeds])
    nbox = nbox_side * nbox_side
    if csr_seed is None:
        rowptr = col = val = None
    else:
        cell_ptr = np.arange(0, tx.shape[0] + 1, p * p, dtype=np.int64)
        rowptr, col, val = own_cell_csr(cell_ptr, csr_seed, cell_class=np.zeros(nbox, np.int64))
    sample = None if sample_seed is None else sample_indices(tx.shape[0], nsample, sample_seed)
    return OversampledWorkload(name=f"oversampled{nbox_side}x{nbox_side}_cheb{p}to{q}", x=x, y=y, w=w, f=f,
                               tx=tx, ty=ty, rowptr=rowptr, col=col, val=val, root=(-1.0, -1.0, 2.0),
                               sample=sample, meta={"boxes": nbox}, nbox=nbox, p_interp=p, q_interp=q)


def config6(nbox_side: int = 128, lam: float = 10.0, nsample: int = 1024):
    """Modified Helmholtz workload: the 128 x 128-box grid of 8x8 GL nodes
    (1,048,576 nodes, one Gaussian-sum density, own-cell corrections with one
    shared block) with lambda = 10 (lambda^2 = 100, the value of the paper's
    modified Helmholtz experiment); meta["lambda"] carries it."""
    wl = uniform_config(nbox_side, [60], 61, 160, f"yukawa{nbox_side}x{nbox_side}_gl8_lambda{lam:g}", nsample=nsample)
    wl.meta["lambda"] = lam
    return wl


def gaussian_sum_density(x, y, seed: int, ncomp: int = 4, center_box: float = 0.8,
                         width_range=(0.05, 0.2), amp_range=(-1.0, 1.0)):
    """f(r) = sum_m A_m exp(-|r - c_m|^2 / sigma_m^2).

    Draw order with numpy.random.default_rng(seed): all amplitudes, then all
    centres (x, y pairs), then all widths.  Returns (f, params).
    """
    rng = np.random.default_rng(seed)
    A = rng.uniform(amp_range[0], amp_range[1], ncomp)
    c = rng.uniform(-center_box, center_box, (ncomp, 2))
    s = rng.uniform(width_range[0], width_range[1], ncomp)
    f = np.zeros_like(x)
    for k in range(ncomp):
        f += A[k] * np.exp(-((x - c[k, 0]) ** 2 + (y - c[k, 1]) ** 2) / s[k] ** 2)
    return f, {"A": A, "c": c, "sigma": s}


def own_cell_csr(cell_ptr: np.ndarray, seed: int, scale: float = 1e-3, cell_class=None):
    """Correction matrix whose row i holds the columns of node i's own cell.

    cell_ptr[k]..cell_ptr[k+1] is the contiguous node range of cell k; every
    node of a cell gets one row listing all nodes of that cell (sorted,
    diagonal included).  Values are N(0, scale^2) from default_rng(seed),
    drawn in row-major nnz order.  With cell_class, the cells of one class
    c >= 0 share one value block drawn from default_rng([seed, c + 1]) (the
    singular corrections of boxes are one lookup table for all boxes of a
    size, by translation invariance of G and the identical box mappings);
    cells of class -1 keep their own values.
    """
    cell_ptr = np.asarray(cell_ptr, dtype=np.int64)
    sizes = np.diff(cell_ptr)
    n = int(cell_ptr[-1])
    row_len = np.repeat(sizes, sizes)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_len, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    pos = 0
    for k in range(sizes.shape[0]):
        s = int(sizes[k])
        b = int(cell_ptr[k])
        block = np.tile(np.arange(b, b + s, dtype=np.int32), s)
        col[pos:pos + s * s] = block
        pos += s * s
    rng = np.random.default_rng(seed)
    val = rng.normal(0.0, scale, nnz)
    if cell_class is not None:
        blocks = {}
        pos = 0
        for k in range(sizes.shape[0]):
            s = int(sizes[k])
            c = int(cell_class[k])
            if c >= 0:
                if c not in blocks:
                    blocks[c] = np.random.default_rng([seed, c + 1]).normal(0.0, scale, s * s)
                val[pos:pos + s * s] = blocks[c]
            pos += s * s
    return rowptr, col, val


def sample_indices(m: int, count: int, seed: int):
    """count distinct target indices drawn uniformly with default_rng(seed), sorted."""
    rng = np.random.default_rng(seed)
    count = min(count, m)
    return np.sort(rng.choice(m, size=count, replace=False)).astype(np.int64)


# --------------------------------------------------------------------------
# Uniform-grid configurations
# --------------------------------------------------------------------------

def uniform_config(nbox_side: int, f_seeds, csr_seed: Optional[int], sample_seed: Optional[int],
                   name: str, nsample: int = 4096, shared_blocks: bool = True):
    """Uniform grid workload.  With shared_blocks every box carries one
    64 x 64 correction block (all boxes have one size and one map, so their
    singular corrections form one table); without, every value is drawn on
    its own (normal, standard deviation 1e-3)."""
    x, y, w = uniform_grid(nbox_side)
    fs = [gaussian_sum_density(x, y, s)[0] for s in f_seeds]
    f = np.stack(fs)
    if csr_seed is None:
        rowptr = col = val = None
    else:
        cell_ptr = np.arange(0, x.shape[0] + 1, 64, dtype=np.int64)
        cls = np.zeros(nbox_side * nbox_side, np.int64) if shared_blocks else None
        rowptr, col, val = own_cell_csr(cell_ptr, csr_seed, cell_class=cls)
    sample = None if sample_seed is None else sample_indices(x.shape[0], nsample, sample_seed)
    return Workload(name=name, x=x, y=y, w=w, f=f, tx=None, ty=None, rowptr=rowptr,
                    col=col, val=val, root=(-1.0, -1.0, 2.0), sample=sample,
                    meta={"boxes": nbox_side * nbox_side, "box_order": 8})


def config0():
    """16x16 boxes of 8x8 GL nodes on [-1,1]^2 (16,384 nodes), one density."""
    return uniform_config(16, [0], 1, None, "uniform16x16_gl8")


def config2():
    """128x128 boxes of 8x8 GL nodes (1,048,576 nodes), one density."""
    return uniform_config(128, [20], 21, 120, "uniform128x128_gl8")


def config3(nbatch: int = 16, shared_blocks: bool = True):
    """256x256 boxes of 8x8 GL nodes (4,194,304 nodes), 16 densities."""
    name = "uniform256x256_gl8_b16" + ("" if shared_blocks else "_per_entry_corr")
    return uniform_config(256, list(range(30, 30 + nbatch)), 46, 130, name, shared_blocks=shared_blocks)


def config4():
    """Differentiation workload on the 128x128 grid.

    Returns (workload_nodes, extra) where workload_nodes carries f (seed 41)
    and extra holds f_true (seed 40), the noise draw (seed 42, unit normal,
    to be scaled by 1e-3) and 4096 off-grid targets (seed 43) drawn
    U[-0.95,0.95]^2 and rejected when within 1e-4 of a node.
    """
    wl = uniform_config(128, [41], 21, 120, "uniform128x128_gl8_grad")
    f_true = gaussian_sum_density(wl.x, wl.y, 40)[0]
    noise = np.random.default_rng(42).standard_normal(wl.n)
    rng = np.random.default_rng(43)
    h = 2.0 / 128
    pts = []
    while len(pts) < 4096:
        p = rng.uniform(-0.95, 0.95, 2)
        # nearest node test: nodes of the containing box and its neighbours
        ix = min(int((p[0] + 1.0) / h), 127)
        iy = min(int((p[1] + 1.0) / h), 127)
        ok = True
        for jy in range(max(iy - 1, 0), min(iy + 2, 128)):
            for jx in range(max(ix - 1, 0), min(ix + 2, 128)):
                b = jy * 128 + jx
                d2 = (wl.x[64 * b:64 * b + 64] - p[0]) ** 2 + (wl.y[64 * b:64 * b + 64] - p[1]) ** 2
                if d2.min() < 1e-8:
                    ok = False
        if ok:
            pts.append(p)
    pts = np.array(pts)
    extra = {"f_true": f_true, "noise": noise, "tx": pts[:, 0].copy(), "ty": pts[:, 1].copy()}
    return wl, extra


# --------------------------------------------------------------------------
# Star-shaped domain with an adaptive box set and a triangle band
# --------------------------------------------------------------------------

def star_radius(theta):
    """Boundary r(theta) = 1 + 0.3 cos(5 theta) of the star-shaped domain."""
    return 1.0 + 0.3 * np.cos(5.0 * theta)


def _star_boxes(root_lo, root_side, base_level, gauss_centres, curve_l8, curve_l9, gauss_l9,
                clearance):
    """Leaves (level, ix, iy) of the adaptive box set, Morton order at level 9.

    A box is split while its level is below its target level: 9 if its
    centre lies within curve_l9 (radially, widened by the half-diagonal) of
    the curve or within gauss_l9 (+ half-diagonal) of a Gaussian centre, 8 if
    within curve_l8 of the curve, else base_level.  A leaf is kept when all
    four corners lie inside the curve with radial clearance >= clearance.
    """
    out = []

    def target_level(level, ix, iy):
        side = root_side / (1 << level)
        cx = root_lo + (ix + 0.5) * side
        cy = root_lo + (iy + 0.5) * side
        hd = 0.5 * np.sqrt(2.0) * side
        rho = np.hypot(cx, cy)
        th = np.arctan2(cy, cx)
        dcurve = abs(star_radius(th) - rho) - hd
        dg = np.min(np.hypot(gauss_centres[:, 0] - cx, gauss_centres[:, 1] - cy)) - hd
        if dcurve < curve_l9 or dg < gauss_l9:
            return 9
        if dcurve < curve_l8:
            return 8
        return base_level

    def inside(level, ix, iy):
        side = root_side / (1 << level)
        for ox in (0, 1):
            for oy in (0, 1):
                px = root_lo + (ix + ox) * side
                py = root_lo + (iy + oy) * side
                rho = np.hypot(px, py)
                th = np.arctan2(py, px)
                if rho > star_radius(th) - clearance:
                    return False
        return True

    def rec(level, ix, iy):
        if level < target_level(level, ix, iy):
            for c in range(4):
                rec(level + 1, 2 * ix + (c & 1), 2 * iy + (c >> 1))
        elif inside(level, ix, iy):
            out.append((level, ix, iy))

    n0 = 1 << base_level
    # visit base boxes in Morton order so leaves come out in Morton order
    order = sorted(((ix, iy) for iy in range(n0) for ix in range(n0)),
                   key=lambda p: _interleave(p[0], p[1]))
    for ix, iy in order:
        rec(base_level, ix, iy)
    return out


def _interleave(ix: int, iy: int) -> int:
    k = 0
    for b in range(16):
        k |= ((ix >> b) & 1) << (2 * b)
        k |= ((iy >> b) & 1) << (2 * b + 1)
    return k


def star_band_triangles(n_sectors: int = 2048):
    """The boundary band of the star domain: n_sectors angular sectors between
    rho = r - 0.01 and r, each split into two triangles; [2 n_sectors, 3, 2]
    vertex coordinates (counter-clockwise)."""
    th = 2.0 * np.pi * np.arange(n_sectors + 1) / n_sectors
    rout = star_radius(th)
    rin = rout - 0.01
    P_in = np.stack([rin * np.cos(th), rin * np.sin(th)], axis=1)
    P_out = np.stack([rout * np.cos(th), rout * np.sin(th)], axis=1)
    tris = []
    for k in range(n_sectors):
        tris.append((P_in[k], P_out[k], P_out[k + 1]))
        tris.append((P_in[k], P_out[k + 1], P_in[k + 1]))
    return np.array(tris)


def triangle_lattice_pattern(p: int = 9, shrink: float = 0.9):
    """A node pattern on the reference simplex for interpolation of total
    degree < p: the principal lattice (i, j) / (p - 1), i + j < p, contracted
    by `shrink` toward the centroid so every node is interior; p (p + 1) / 2
    nodes, with equal reference weights (summing to the area 1/2).  Returns
    (xi, eta, wref)."""
    if p == 1:  # one node: the centroid
        return np.array([1.0 / 3.0]), np.array([1.0 / 3.0]), np.array([0.5])
    lat = np.array([(i / (p - 1), j / (p - 1)) for i in range(p) for j in range(p - i)])
    ref = 1.0 / 3.0 + shrink * (lat - 1.0 / 3.0)
    n = ref.shape[0]
    return ref[:, 0].copy(), ref[:, 1].copy(), np.full(n, 0.5 / n)


def cell_maps(origins, A):
    """[ncell, 6] rows (o_x, o_y, A_00, A_01, A_10, A_11) of affine cell maps
    r = o + A zeta (origins [ncell, 2], A [ncell, 2, 2])."""
    origins = np.asarray(origins, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    return np.concatenate([origins, A.reshape(-1, 4)], axis=1)


def triangle_maps(tris):
    """Cell maps of triangles [ntri, 3, 2]: o = v0, A = [v1 - v0, v2 - v0] (columns)."""
    tris = np.asarray(tris, dtype=np.float64)
    A = np.stack([tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]], axis=2)
    return cell_maps(tris[:, 0], A)


def config1(n_sectors: int = 2048, tri_nodes: int = 45):
    """Star-shaped domain r = 1 + 0.3 cos 5 theta, about 1.5M nodes.

    Interior: adaptive boxes on [-1.3,1.3]^2 (base level 7, level 8 within
    0.15 of the curve, level 9 within 0.03 of the curve or 0.05 of a Gaussian
    centre; distances are radial, from the box, i.e. centre distance less the
    half-diagonal), kept when inside with clearance 0.005; 8x8 GL nodes per
    box.  This gives 1,488,064 nodes (20,371 boxes, 4,096 triangles).
    Boundary band: n_sectors angular sectors between rho = r - 0.01 and r,
    each split into two triangles; each triangle gets tri_nodes nodes at
    Dirichlet(1,1,1) barycentric points with Dirichlet(1,...,1) weights
    scaled to the triangle area (seed 11).  Density: three Gaussians of
    width 1e-2, amplitudes U[-1,1], centres inside rho < 0.8 r (seed 10).
    Correction rows hold each node's own cell (seed 12).  Triangles first.
    """
    rng = np.random.default_rng(10)
    A = rng.uniform(-1.0, 1.0, 3)
    cents = []
    while len(cents) < 3:
        p = rng.uniform(-1.3, 1.3, 2)
        if np.hypot(p[0], p[1]) < 0.8 * star_radius(np.arctan2(p[1], p[0])):
            cents.append(p)
    cents = np.array(cents)
    sig = np.full(3, 1e-2)

    # --- triangle band
    rng_t = np.random.default_rng(11)
    tris = star_band_triangles(n_sectors)
    tx_list, ty_list, tw_list = [], [], []
    for (a, b, c) in tris:
        lam = rng_t.dirichlet(np.ones(3), tri_nodes)
        px = lam[:, 0] * a[0] + lam[:, 1] * b[0] + lam[:, 2] * c[0]
        py = lam[:, 0] * a[1] + lam[:, 1] * b[1] + lam[:, 2] * c[1]
        area = 0.5 * abs((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]))
        ww = rng_t.dirichlet(np.ones(tri_nodes)) * area
        tx_list.append(px)
        ty_list.append(py)
        tw_list.append(ww)
    xt = np.concatenate(tx_list)
    yt = np.concatenate(ty_list)
    wt = np.concatenate(tw_list)

    # --- adaptive boxes
    leaves = _star_boxes(-1.3, 2.6, 7, cents, 0.15, 0.03, 0.05, 0.005)
    xi, eta, wref = gauss_legendre_box_nodes(8)
    lv = np.array([l for (l, _, _) in leaves])
    ixs = np.array([i for (_, i, _) in leaves])
    iys = np.array([j for (_, _, j) in leaves])
    side = 2.6 / (1 << lv)
    cx = -1.3 + (ixs + 0.5) * side
    cy = -1.3 + (iys + 0.5) * side
    xb = (cx[:, None] + 0.5 * side[:, None] * xi[None, :]).ravel()
    yb = (cy[:, None] + 0.5 * side[:, None] * eta[None, :]).ravel()
    wb = (wref[None, :] * (0.5 * side[:, None]) ** 2).ravel()

    x = np.concatenate([xt, xb])
    y = np.concatenate([yt, yb])
    w = np.concatenate([wt, wb])
    f = np.zeros_like(x)
    for k in range(3):
        f += A[k] * np.exp(-((x - cents[k, 0]) ** 2 + (y - cents[k, 1]) ** 2) / sig[k] ** 2)
    ntri = len(tris)
    cell_ptr = np.concatenate([np.arange(0, ntri * tri_nodes + 1, tri_nodes, dtype=np.int64),
                               ntri * tri_nodes + np.arange(64, 64 * len(leaves) + 1, 64, dtype=np.int64)])
    # triangles: own values each; boxes: one shared block per box level
    cell_class = np.concatenate([np.full(ntri, -1, np.int64), lv.astype(np.int64)])
    rowptr, col, val = own_cell_csr(cell_ptr, 12, cell_class=cell_class)
    sample = sample_indices(x.shape[0], 4096, 110)
    return Workload(name="star_adaptive", x=x, y=y, w=w, f=f[None, :], tx=None, ty=None,
                    rowptr=rowptr, col=col, val=val, root=(-1.3, -1.3, 2.6), sample=sample,
                    meta={"triangles": ntri, "boxes": len(leaves),
                          "levels": {int(l): int((lv == l).sum()) for l in np.unique(lv)},
                          "gauss_centres": cents, "gauss_amps": A})
