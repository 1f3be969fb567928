"""Grid friction force on an ideal planar front (the paper's Fig. 3 study).

The total force is the system sum of the bracket of Eq. 4,
F = sum_p sum_k w_k (lambda^2 / |r_k|^2 D_k - g_k'(phi_p)), which the library
evaluates on the device from the field alone (spfm_force: the step's
right-hand side without the driving force, FP64, compensated sum).  The front
lives on the paper's 300 x 1 x 1 line between contact-angle walls whose angles
hold the exact front (sin(alpha) = n . e), so the stencil neighbours off the
line see the analytic profile.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

LINE = (1, 1, 300)   # (nz, ny, nx)


def front_forces(S, *, coupling: str, lam: float, n, shifts: Sequence[float],
                 u=(1.0, 0.0, 0.0), stencil: int = 26):
    """F for the front of normal n shifted by each value of `shifts` along n.
    S is the loaded binding module (paper_1910_05180_amd.spfm).  The context
    never steps, so its time step is not checked against the stability bound."""
    nv = np.asarray(n, dtype=np.float64)
    nv = nv / np.linalg.norm(nv)
    out = []
    with S.Spfm(LINE, lam=lam, mu=0.0, stencil=stencil, dtype="f64", coupling=coupling, u=u,
                walls=7, wall_sin=S.front_wall_sin(nv), allow_unstable=True, kernel="plain") as s:
        for c in shifts:
            s.init_front(nv, float(c))
            out.append(s.force())
    return out


def amplitude(S, *, coupling: str, lam: float, n, u=(1.0, 0.0, 0.0), samples: int = 12,
              stencil: int = 26) -> float:
    """Half the peak-to-peak force over shifts spanning one grid spacing."""
    F = front_forces(S, coupling=coupling, lam=lam, n=n, u=u, stencil=stencil,
                     shifts=[k / samples for k in range(samples)])
    return 0.5 * (max(F) - min(F))
