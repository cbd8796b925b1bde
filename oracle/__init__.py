"""FP64 CPU oracle for the FMM-accelerated BEM of arXiv:1007.4591.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1007_4591_amd``) and never imports it.

Contents
--------
* ``dense``         -- ctypes front end of ``bem_dense.c``: the dense
                       discrete operators (A, A^T, B, B^T, C, C^T, forces),
                       GMRES, solvation energy, BIBEE and the adjoint.
* ``closed_forms``  -- Born ion, Kirkwood sphere series and the BIBEE sphere
                       series (pins of the dense oracle).
* ``tree``          -- the octree, Morton keys and interaction lists by
                       their definitions (brute force).
* ``harmonics``     -- solid harmonics and multipole / local expansions by
                       their definitions (scipy Legendre functions).
* ``panel_integrals`` -- exact integrals of the Green's function and its
                       gradient over flat triangles, and the near-quadrature
                       K' (exact integrals for close panel pairs).
* ``lpb``           -- dense linearised Poisson-Boltzmann BEM (screened
                       solvent): the second-kind system for the surface
                       potential and its normal derivative, energies.
"""
from .dense import *  # noqa: F401,F403
from . import closed_forms, tree, harmonics, panel_integrals, lpb  # noqa: F401
