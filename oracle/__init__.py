"""FP64 CPU oracle for Multipolynomial Monte Carlo trace estimation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The GPU product path (``paper_2402_00016_amd``) never imports it, and
this package never imports the product path: the two share no kernels,
headers, helpers, tables or pre/post-processing.  The only module both sides
use is the seeded input generator ``paper_2402_00016_amd.inputs`` (gauge links),
which holds none of the method's arithmetic.

Every function is a plain, slow, obviously correct statement of what the paper
computes, in FP64:

* ``philox``    -- counter-based Philox4x32-10 generator and Z(4) noise
                   (the noise of the Hutchinson estimator, Sec. 1).
* ``lattice``   -- indexing, DeGrand-Rossi gammas, dense Wilson matrix for
                   small lattices, free-field closed forms.
* ``wilson``    -- matrix-free Wilson-Dirac operator M (plain C, OpenMP).
* ``krylov``    -- Arnoldi / one GMRES(d) cycle, harmonic Ritz values,
                   Leja ordering (Sec. 3).
* ``poly``      -- GMRES polynomials p(M), pi(M) and the double polynomial
                   p_in(M) p_out(phi_in(M)) (Sec. 3, Sec. 5).
* ``deflation`` -- polynomial-preconditioned Arnoldi eigenpairs, left vectors
                   and the deflated level term (Sec. 7, Sec. 8).
* ``solve``     -- deflated restarted GMRES main solves and dense solves.
* ``estimator`` -- level samples and the multipolynomial combination
                   (eq. 2, Sec. 6 multipolynomial formula, Sec. 7).

Parity status of each function is listed in its module docstring.
"""
