"""Algorithmic work of the method, counted on its definition (the 12-component
first-order system integrated by the Dormand-Prince 5(4) pair with ode45's
error norm and control, Sec. 2.1 and Fig. 2), not on any implementation.

Convention: an add, subtract, multiply, divide, compare/min/max, square root,
cosine or power counts 1 FLOP; a fused multiply-add counts 2; absolute values
and copies count 0.

Per step attempt (accepted or rejected):
  stage coefficient products h a_sj, 20 non-zero a_sj            20
  stage inputs y + sum_j (h a_sj) k_j, 20 terms x 12 components  480
  stage times t + c_s h (5 fused) and t + h                       11
  6 force evaluations x 36 (difference 3, r^2 5, 1/r^2 1, s^2 and
    s^3 2, 4C4 - 8C8 s^2 2, product 1, /m 2, trap factors 6,
    ion accelerations 9, atom accelerations 3, Omega t 1, cos 1)  216
  error vector sum_j e_j k_j, 6 terms x 12 components             132
  weighted infinity norm (2 max, 1 divide, 1 running max per
    component) and the factor |h|                                 49
  error test, step-size update and step set-up                    14
                                                          total  922
Per accepted step: closest-approach test w = d . (v_ion - v_atom),
  sign and radius tests, running minimum, exit test              16
Per trajectory: f(t0, y0), the initial step and the observables'
  initial values (92), and the final observables (48)            140
"""
from __future__ import annotations

import numpy as np

from . import workload as W

FLOP_PER_ATTEMPT = 922
FLOP_PER_ACCEPTED = 16
FLOP_PER_TRAJECTORY = 140


def algorithmic_flops(obs: np.ndarray) -> float:
    """Algorithmic FLOPs of one integration whose observables are ``obs``."""
    nsteps = float(np.sum(obs[W.OBS["nsteps"]]))
    nfailed = float(np.sum(obs[W.OBS["nfailed"]]))
    n = obs.shape[1]
    return (FLOP_PER_ATTEMPT * (nsteps + nfailed) + FLOP_PER_ACCEPTED * nsteps
            + FLOP_PER_TRAJECTORY * n)
