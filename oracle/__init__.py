"""CPU oracle for the volume-potential hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check (__graft_entry__.smoke) and bench.py's
cpu_baseline leg may import, call, link or execute anything in this package.
The GPU library never does, and the two share no code: the only inputs they
share come from the seeded generators in vp_workloads.

  direct.c / direct.py : float64 direct sums (smooth part, correction part,
                         adjoint, target gradient), OpenMP over targets
  tree.py              : plain quadtree and U/V/W/X lists by definition
  expansions.py        : multipole/local coefficients by definition
  fmm_truncated.py     : what an order-p FMM computes on a uniform tree
  oversample.py        : the box oversampling map O_{p,q} (Chebyshev values ->
                         coefficients -> values at finer roots) and the
                         oversampled smooth sum with its adjoint
  yukawa.py            : the modified Helmholtz (Yukawa) smooth sum with
                         G = (lambda^2 / 2 pi) K_0(lambda r), and its transpose
  corrections.py       : own-cell singular correction blocks of boxes and
                         straight triangles (exact integrals of G against the
                         cell's Lagrange basis, less the smooth rule), by polar
                         coordinates about the target
"""
