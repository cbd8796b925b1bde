"""Electrostatic binding free energy (Section 4.4, eq.
binding-free-energy-estimate): dG_bind = dG_complex - dG_protein -
dG_inhibitor, each a solvation energy of its own surface and charges.

Builds one tree per molecule and calls ``bemfmm_binding_energy`` (the
composition itself runs behind the C-ABI): the full BEM solve or one of the
three BIBEE variants.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import (ENERGY_BEM, ENERGY_BIBEE_CFA, ENERGY_BIBEE_P, ENERGY_BIBEE_PLUS_HALF, FP32_REFINED, Params,
               binding_energy as _binding_energy, build_tree)

_METHODS = {"bem": ENERGY_BEM, "cfa": ENERGY_BIBEE_CFA, "p": ENERGY_BIBEE_P, "plus_half": ENERGY_BIBEE_PLUS_HALF}


@dataclass
class Molecule:
    verts: object       # (V, 3)
    tris: object        # (N, 3) int32
    charge_pos: object  # (Q, 3)
    q: object           # (Q,)


def binding_energy(complex_: Molecule, protein: Molecule, inhibitor: Molecule, method: str = "bem",
                   params: Params | None = None, tol: float = 1e-6, precision: int = FP32_REFINED) -> dict:
    """dG_bind = dG_complex - dG_protein - dG_inhibitor, with the parts
    (kcal/mol); method is 'bem', 'cfa', 'p' or 'plus_half'."""
    trees = [build_tree(m.verts, m.tris, m.charge_pos, params) for m in (complex_, protein, inhibitor)]
    return _binding_energy(trees[0], complex_.q, trees[1], protein.q, trees[2], inhibitor.q, method=_METHODS[method],
                           precision=precision, tol=tol)
