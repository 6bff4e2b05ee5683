"""Plain, slow FP64 CPU oracle of the heightfield renderer's per-frame path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code with the HIP library: it is written from the paper
(Cornel, Horvath, Waser 2022, "An Attempt of Adaptive Heightfield Rendering
with Complex Interpolants Using Ray Casting") and from the public definitions
of the methods it cites.

Modules and the passage each follows:

* ``quadtree``   -- the adaptive grid the method consumes (Section 2: values at
                    the centres of an adaptive grid).  The paper does not say
                    how the grid is made; the refinement rule is a reading.
* ``neighbours`` -- the per-cell buffer of potentially influencing cells
                    (Section 4, the startup precomputation of the set I).
* ``camera``     -- pinhole rays, one per pixel (Section 5).
* ``cascades``   -- cascade fitting (Section 3): frustum/box intersection,
                    hull, logarithmic splits, clipping, overlap, stable fit.
* ``discretize`` -- the visibility texture (Section 3, last paragraph) and
                    the truncated-Gaussian weighted sum (Eq. 1 and Eq. 2).
* ``maxmip``     -- maximum mipmap of Tevs et al. 2008 (cited in Section 5).
* ``raycast``    -- first ray/bilinear-patch hit per cascade and the convex
                    blend in cascade overlaps (Section 5); the cell walk is
                    plain C in ``oracle/c`` for speed, FP64 throughout.
* ``adjoint``    -- hand-derived gradients of hit depth with respect to
                    texel heights, and of Eq. 2 with respect to leaf values
                    and widths; central finite differences.
* ``composite``  -- several heightfields per frame (Section 2's terrain and
                    water depths, Table 1's passes): the nearest first hit.

Parity status of each function is stated in its docstring ("pinned by ..."
naming the tests that pin it, or "parity unpinned").
"""
