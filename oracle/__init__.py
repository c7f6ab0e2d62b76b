"""Plain FP64 CPU oracle for the l1-regularised least-squares solver core.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1503_03520_amd``) and imports nothing from it; the one
module both sides may use is ``seeded_inputs`` (random test vectors, no
arithmetic of the method).

Contents (each function cites the passage of Fountoulakis & Gondzio,
"Performance of first- and second-order methods for l1-regularized least
squares problems", arXiv:1503.03520, that it follows):

* ``philox``    -- Philox-4x32-10 (Salmon et al., SC'11), the counter-based
                   generator that every random draw of an instance comes from.
* ``instance``  -- the instance generator: Givens rounds, Sigma, IGen
                   (section 3.1), the SVD-known A of eq. (16) (section 4),
                   operator products MvPA / MvPAt, explicit A for tests;
                   IGen2 (section 3.2) for m < n over the same matrices.
* ``cfista``    -- the FISTA of ``fista`` in C with OpenMP (fista_omp.c),
                   bitwise the same iterates, for the CPU baseline.
* ``fista``     -- FISTA (section 8.1), soft-thresholding, the Lasso duality
                   gap, power iteration for L.
* ``bruteforce``-- sign-pattern enumeration of the reduced problem (13) for
                   n <= 12.
* ``sgt``       -- the A = Sigma G^T class of sections 8.4 to 8.9: sigma and
                   x* laws (Procedures OsGen, OsGen3), kappa_rho (eq. (17)).
* ``newton``    -- smoothed Newton-CG on the pseudo-Huber problem (8)
                   (section 2, section 8.1 item pdNCG, section 8.3 params).
* ``polish``    -- FP64 support/sign polish on the reduced problem (13).
* ``pcdm``      -- PCDM (section 8.1 item PCDM, beta of section 8.3) with
                   tau-nice sampling on the generator's instances.
"""
