"""MI355X (gfx950) even-odd Wilson-Dirac operator and solvers.

The computation of Barthou et al., "Automated Code Generation for Lattice
Quantum Chromodynamics and beyond" (arXiv:1401.2039): applying the Wilson-Dirac
hopping matrix (Fig. "dirac") inside the CGNR template (Fig. "CG") composed with
the Schur-complement template, behind the C ABI of include/qiral.h and
implemented in hand-written HIP kernels (csrc/).  This package is the thin
Python binding: ``api`` marshals torch tensors (device memory, streams) into
the C calls; nothing is computed in Python.
"""
from .api import (  # noqa: F401
    Lattice, Network, qiral_field_bytes, qiral_gauge_bytes, qiral_lattice_create, qiral_solve_workspace_bytes,
    qiral_solve_batch_workspace_bytes, qiral_solve_static, qiral_lattice_destroy, qiral_field_import,
    qiral_field_export, qiral_dslash_eo, qiral_apply_M, qiral_tune, qiral_solve, qiral_solve_batch, solve_params,
)
from ._lib import (  # noqa: F401
    F64, F32, F16S, EVEN, ODD, FULL, OP_D, OP_DDAG, OP_SCHUR, OP_SCHUR_DAG, CGNR_EO, BICGSTAB_EO,
    FGMRES_NN, CRNR_EO, FCG_NN, SYSTEM_DEFAULT, SYSTEM_SCHUR, SYSTEM_FULL, LINKS_F32, LINKS_F16, RECON12, RECON18, QiralError,
)
