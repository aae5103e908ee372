"""FP64 CPU oracle for the convolution-surface lattice slicer.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 restatement
of what the slicing path computes, written from the paper (Liu et al.,
"Memory-Efficient Modeling and Slicing of Large-Scale Adaptive Lattice
Structures", Secs. 3-4).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the
native library and imports nothing from it.

Modules
  field     -- kernel (Eq. 5), per-strut integral (Eqs. 6-7), field sums
  slicer    -- slice heights, active set (Eq. 8), the event sweep to the same sets,
               per-slice field and the inside test
  binning   -- the (slab, tile, strut) bin set the native binning must equal
  contours  -- marching squares on the binary slice image (Sec. 4)
  polylines -- sub-pixel contour endpoints and the chaining of segments
               into closed loops / open chains (the step after Sec. 4)
  support   -- self-support metrics Gamma, Psi (Sec. 5.2, Eqs. 11-14) and
               dGamma/dv
  density   -- per-voxel density by the inside test at pixel centres
               (Sec. 5, Eq. 9) and a smooth voxel-density loss with its
               field gradient, for the radius adjustment of Sec. 5.3
  gradient  -- derivatives of a pixel-weighted field sum with respect to
               strut weights and node positions

Readings of the paper that this oracle fixes (each is restated where used):
  * Eq. (6) integrates over the edge by arclength; the s-integral of Eq. (7)
    is multiplied by the chord length l (its Jacobian).
  * inside <=> sum_i r_i I_i(p) >= C (the larger sum lies near the skeleton).
  * slice k lies at z0 + (k + 1/2) dz.
"""
