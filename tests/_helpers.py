"""Shared test helpers: accepted seeded states and error metrics."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1401_4350_amd.inputs import Workload, make_state

MARGIN = 1e-9


def accepted_state(w: Workload, seed: int, max_attempts: int = 20):
    """Draw make_state(w, seed, attempt) until no pair distance lies within
    1e-9 sigma of r_c or r_v (the neighbour set and the cut-off decisions are
    then insensitive to rounding order)."""
    for attempt in range(max_attempts):
        s = make_state(w, seed, attempt)
        m = oracle.pair_margin(s.x, s.box, [w.rcut, w.rcut + w.skin])
        if m > MARGIN:
            return s
    raise RuntimeError("no accepted state")


def cond_rel_err(got, ref, scale):
    """max_i,c |got - ref| / max(scale, 1e-300): the per-component error
    normalised by the sum of the magnitudes of the terms that make it up."""
    return float(np.max(np.abs(got - ref) / np.maximum(scale, 1e-300)))
