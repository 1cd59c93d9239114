"""Module-I inputs in the paper's conventions, mapped onto a request.

Host-side argument preparation only (no physics).  The paper's ODF run takes
its settings from keyword lines of an input file and its T-P grid from a
separate grid file (App. G, the module-I input example and the T-P grid
description):

* ``velocities values n v_1 ... v_n`` — the microturbulences [km/s]; one
  table per value (0 km/s when the keyword is absent);
* ``mean arithmetic`` (after ``odf``) — arithmetic sub-bin means instead of
  the geometric default;
* ``abundance scale s`` — a linear factor on every element heavier than He;
* ``abundance change Z v [Z v ...]`` — for H and He the number fraction
  N/N_tot, for heavier elements log10(N/N_tot);
* the grid file: the numbers of temperatures and pressures on the first two
  lines, then the temperatures, then the pressures, one per line.

The engine wants abundances by number relative to hydrogen, A = N/N_H, and
an expanded point list.  Readings: pressures in the grid file are taken as
log10 P [dyn cm^-2] unless ``log_pressure=False``; the point list runs over
the microturbulences outermost, then T, then P (P fastest).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .workload import Points


@dataclass
class OdfInput:
    vturbs_kms: list = field(default_factory=lambda: [0.0])
    mean: str = "geometric"
    abundance_scale: float = 1.0
    abundance_change: dict = field(default_factory=dict)   # Z -> value as written


def parse_odf_input(text: str) -> OdfInput:
    """The module-I keywords that the engine uses; other lines are ignored."""
    out = OdfInput()
    for raw in text.splitlines():
        tok = raw.split()
        i = 0
        while i < len(tok):
            t = tok[i].lower()
            nxt = tok[i + 1].lower() if i + 1 < len(tok) else ""
            if t == "velocities" and nxt == "values":
                n = int(tok[i + 2])
                out.vturbs_kms = [float(x) for x in tok[i + 3:i + 3 + n]]
                if len(out.vturbs_kms) != n:
                    raise ValueError(f"velocities values: {n} values announced, {len(out.vturbs_kms)} given")
                i += 3 + n
            elif t == "mean" and nxt in ("arithmetic", "geometric"):
                out.mean = nxt
                i += 2
            elif t == "abundance" and nxt == "scale":
                out.abundance_scale = float(tok[i + 2])
                i += 3
            elif t == "abundance" and nxt == "change":
                i += 2
                while i + 1 < len(tok) and tok[i].lstrip("+-").isdigit():
                    out.abundance_change[int(tok[i])] = float(tok[i + 1])
                    i += 2
            else:
                i += 1
    return out


def abundances_relative_to_h(inp: OdfInput, atomic_numbers) -> np.ndarray:
    """A_s = N_s / N_H for the species with the given atomic numbers (Z >= 2).

    H and He are written as number fractions, heavier elements as
    log10(N/N_tot), and the scale multiplies every element heavier than He.
    """
    ch = inp.abundance_change
    if 1 not in ch or not ch[1] > 0.0:
        raise ValueError("the hydrogen number fraction (abundance change 1 ...) is needed")
    x_h = ch[1]
    out = np.empty(len(atomic_numbers))
    for k, z in enumerate(atomic_numbers):
        z = int(z)
        if z not in ch:
            raise ValueError(f"no abundance for element {z}")
        if z == 2:
            frac = ch[2]
        elif z > 2:
            frac = inp.abundance_scale * 10.0 ** ch[z]
        else:
            raise ValueError("hydrogen is not a species of the table")
        out[k] = frac / x_h
    return out


def parse_tpgrid(text: str, vturbs_kms, log_pressure: bool = True) -> Points:
    """Expanded point list of a T-P grid file at the given microturbulences."""
    vals = [v for v in text.split()]
    n_t, n_p = int(vals[0]), int(vals[1])
    nums = [float(v) for v in vals[2:]]
    if len(nums) != n_t + n_p:
        raise ValueError(f"T-P grid: {n_t} + {n_p} values announced, {len(nums)} given")
    T = np.asarray(nums[:n_t])
    P = np.asarray(nums[n_t:])
    lp = P if log_pressure else np.log10(P)
    V = np.asarray(vturbs_kms, dtype=np.float64)
    VV, TT, PP = np.meshgrid(V, T, lp, indexing="ij")
    return Points(TT.ravel().astype(np.float64), PP.ravel().astype(np.float64), VV.ravel().astype(np.float64))
