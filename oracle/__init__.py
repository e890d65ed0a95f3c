"""CPU oracle for the mixed-variational phononic band-structure path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (the HIP library and its Python binding) never
imports it and shares no code with it.

The oracle is a plain, slow FP64 implementation written from the paper
(Lu, Yang, Guest, Srivastava, "3-D phononic crystals with ultra-wide band
gaps"), in SI units, in the paper's own orientation of the matrices:

* ``geometry``   lattices, reciprocal vectors, plane-wave set, k-paths
* ``materials``  Voigt compliance and the density/compliance interpolation
* ``fourier``    centroid-rule Fourier coefficients by direct sums
* ``assembly``   the integrals I, Omega, Phi and H (Eqs. 5-7, 16, 19)
* ``solve``      Schur complement and generalized Hermitian eigensolve (Eq. 4)
* ``adjoint``    design sensitivities (Eqs. 12-15, 20-21)
* ``objective``  normalized gap (Eq. 10) and its KS-smoothed form
* ``brute``      brute-force companions: homogeneous closed form, the
                 unreduced saddle-point system, the materialised-derivative
                 sensitivity, a plane-wave-expansion comparator

Every function is pinned by a ``-m "not gpu"`` test against a closed form,
an invariant, a brute-force route or finite differences.  Nothing the
paper prints pins a band value (its designs exist only in figures), so
"parity with a printed band structure" is unpinned.
"""
