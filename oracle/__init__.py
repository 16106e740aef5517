"""CPU oracle for the even-odd Wilson-Dirac solves -- TEST INFRASTRUCTURE ONLY.

A plain, slow, complex128 NumPy implementation of what the GPU path computes,
written from the paper (Barthou et al., "Automated Code Generation for Lattice
Quantum Chromodynamics and beyond", arXiv:1401.2039):

* ``gamma``   -- the spin matrices and their identities (Fig. "id").
* ``wilson``  -- the Dirac operator of Fig. "dirac", its even/odd blocks and
                 the Schur complement of the "schur" template (Sec. 2).
* ``solvers`` -- the CGNR template (Fig. "CG"), its composition with the Schur
                 template as the goal statement asks, and the added BiCGStab,
                 FGMRES and flexible CG.
* ``ptc``     -- the parallel-transport network used as a learned
                 preconditioner (an addition; not in the paper).
* ``storage`` -- what the reduced-precision storage classes represent.
* ``dense``   -- dense assembly of small operators for brute-force checks.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  The GPU path never calls it, and it shares no code
with the GPU path: the only common code is the input generator ``latgen``.
"""
