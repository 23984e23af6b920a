"""CPU oracle for the affine-view-simulation / ORB / Hamming-matching hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
NumPy definition of what the GPU library computes, written from the paper
("Feature Point Extraction for Extra-Affine Image", arXiv 2503.03479) and the
ORB / ASIFT constructions it builds on.  Floating point work is fp64, all ORB
and matching work is exact integer arithmetic (int64).  Only tests/,
__graft_entry__.smoke() and bench.py's CPU-baseline leg may import it; the
product library (paper_2503_03479_amd) never does, and the two share no code.

Modules
  plan      -- sampling grid (Sec. III.B), camera map of eq. (2), canvases,
               pyramid sizes and per-level keypoint quotas
  simulate  -- anti-alias blur and Lanczos-4 resampling (eqs. (3)-(4))
  orb       -- pyramid, FAST-9, Harris top-N, orientation, smoothing, rBRIEF
  match     -- brute-force Hamming nearest neighbour with ratio test (Sec. III.B,
               Sec. IV.C), best view pair, back-mapping and precision (eqs. (5)-(6))
  pipeline  -- the composition: simulate both images, extract, match all view pairs
  diffwarp  -- the Lanczos-4 warp of an fp image as a function of the six camera
               parameters, and its adjoint (image and parameter gradients)
  geometry  -- homography RANSAC over matched points (Sec. III.C) and the inlier
               ratio of eq. (7)
"""
from . import plan, simulate, orb, match, pipeline, diffwarp, geometry  # noqa: F401
