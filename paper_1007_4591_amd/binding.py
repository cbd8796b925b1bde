"""Electrostatic binding free energy by composition (Section 4.3,
eq. binding-free-energy-estimate): dG_bind = dG_complex - dG_protein -
dG_inhibitor, each a solvation energy of its own surface and charges.

Composition only: every energy comes from the C-ABI (``solve_bem`` +
``solvation_energy`` for the full BEM, ``bibee_energy`` for BIBEE/CFA or
BIBEE/P).
"""
from __future__ import annotations

from dataclasses import dataclass

from . import (BIBEE_CFA, BIBEE_P, FP32_REFINED, Params, bibee_energy, build_tree, solvation_energy,
               solve_bem)


@dataclass
class Molecule:
    verts: object       # (V, 3)
    tris: object        # (N, 3) int32
    charge_pos: object  # (Q, 3)
    q: object           # (Q,)


def solvation(m: Molecule, method: str = "bem", params: Params | None = None, tol: float = 1e-6,
              precision: int = FP32_REFINED) -> float:
    """Solvation energy of one molecule (kcal/mol): method 'bem', 'cfa' or 'p'."""
    t = build_tree(m.verts, m.tris, m.charge_pos, params)
    if method == "bem":
        x, _ = solve_bem(t, m.q, tol=tol, precision=precision)
        return solvation_energy(t, m.q, x, precision=0)
    kind = {"cfa": BIBEE_CFA, "p": BIBEE_P}[method]
    return bibee_energy(t, m.q, kind=kind, precision=0)


def binding_energy(complex_: Molecule, protein: Molecule, inhibitor: Molecule, method: str = "bem",
                   params: Params | None = None, tol: float = 1e-6, precision: int = FP32_REFINED) -> dict:
    """dG_bind = dG_complex - dG_protein - dG_inhibitor, with the parts."""
    c = solvation(complex_, method, params, tol, precision)
    p = solvation(protein, method, params, tol, precision)
    i = solvation(inhibitor, method, params, tol, precision)
    return {"complex": c, "protein": p, "inhibitor": i, "binding": c - p - i}
