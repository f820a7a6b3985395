"""Problem description: sites, operator terms and couplings.

A model is the input list of the paper's pseudocode (App. A): the local spins s_i (or boson cut-offs),
the one-site couplings and the pair list with its J^{alpha beta} table, generalised to a flat list of
terms so that every coupling can be a separate real parameter (needed for the coupling gradient).

    H(theta) = sum_t theta[param_t] * w_t * O_{op_a}^{(site_a)} O_{op_b}^{(site_b)}

with site_b = -1 for a one-site term.  Operators (local matrices are defined by the consumers, not here):

    OP_Z      S_z on a spin site (eigenvalue m), n = a^dagger a on a boson site
    OP_Z2     (S_z)^2, or n^2 on a boson site                       (one-site only)
    OP_RAISE  S_+ on a spin site, a^dagger on a boson site
    OP_LOWER  S_- on a spin site, a on a boson site
    OP_RAISE2 (S_+)^2, or a^dagger^2                                (one-site only)
    OP_LOWER2 (S_-)^2, or a^2                                       (one-site only)

Sites are listed most significant first (site 0 is the leftmost Kronecker factor), following the
multiplier definition of Sec. III.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

SPIN, BOSON = 0, 1
OP_Z, OP_Z2, OP_RAISE, OP_LOWER, OP_RAISE2, OP_LOWER2 = 0, 1, 2, 3, 4, 5
OP_LOCAL_BASE = 16          # op OP_LOCAL_BASE + i: entry i of Model.local_ops


@dataclass(frozen=True)
class Site:
    """kind SPIN: k = 2s (local dimension k+1).  kind BOSON: k = n_max (local dimension k+1)."""
    kind: int
    k: int

    @property
    def d(self) -> int:
        return self.k + 1


def spin_site(two_s: int) -> Site:
    return Site(SPIN, int(two_s))


def boson_site(n_max: int) -> Site:
    return Site(BOSON, int(n_max))


@dataclass(frozen=True)
class Term:
    site_a: int
    op_a: int
    site_b: int = -1
    op_b: int = OP_Z
    param: int = 0
    w: complex = 1.0


@dataclass(frozen=True)
class LocalOp:
    """A general one-site operator on one band: <n|O|n - shift> = values[n] for the target digit n
    (entries whose source n - shift is outside 0..d-1 are ignored)."""
    site: int
    shift: int
    values: tuple


@dataclass
class Model:
    sites: List[Site]
    terms: List[Term]
    theta: np.ndarray                     # float64 [n_params]
    name: str = ""
    meta: dict = field(default_factory=dict)
    local_ops: List[LocalOp] = field(default_factory=list)

    @property
    def n_params(self) -> int:
        return int(len(self.theta))

    @property
    def dim(self) -> int:
        return dim_of(self.sites)

    def site_arrays(self):
        kind = np.array([s.kind for s in self.sites], dtype=np.int32)
        k = np.array([s.k for s in self.sites], dtype=np.int32)
        return kind, k

    def term_arrays(self):
        """Structure-of-arrays view of the term list (what the C interfaces take)."""
        n = len(self.terms)
        ints = np.zeros((n, 5), dtype=np.int32)
        w = np.zeros((n, 2), dtype=np.float64)
        for i, t in enumerate(self.terms):
            ints[i] = (t.site_a, t.op_a, t.site_b, t.op_b, t.param)
            w[i] = (complex(t.w).real, complex(t.w).imag)
        return ints, w


def dim_of(sites: Sequence[Site]) -> int:
    D = 1
    for s in sites:
        D *= s.d
    return D


def xxz_bond_terms(i: int, j: int, p_xy: int, p_z: int) -> List[Term]:
    """J_xy (S^x S^x + S^y S^y) + J_z S^z S^z on bond (i, j), written as
    (J_xy/2)(S_+ S_- + S_- S_+) + J_z S_z S_z with J_xy = theta[p_xy], J_z = theta[p_z]."""
    return [
        Term(i, OP_RAISE, j, OP_LOWER, p_xy, 0.5),
        Term(i, OP_LOWER, j, OP_RAISE, p_xy, 0.5),
        Term(i, OP_Z, j, OP_Z, p_z, 1.0),
    ]
