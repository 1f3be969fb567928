"""Grid friction force on an ideal planar front (the paper's Fig. 3 study).

The total force is the system sum of the bracket of Eq. 4,
F = sum_p sum_k w_k (lambda^2 / |r_k|^2 D_k - g_k'(phi_p)); on the grid it is
the sum of the rates at mu = 0 over A = 2M / (3 C_Gamma lambda^2).  The front
lives on the paper's 300 x 1 x 1 line between contact-angle walls whose angles
hold the exact front (sin(alpha) = n . e), so the stencil neighbours off the
line see the analytic profile.  One FP64 step of the library gives
F = (sum phi_after - sum phi_before) / (dt A) from its compensated sums.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

LINE = (1, 1, 300)   # (nz, ny, nx)


def front_forces(S, *, coupling: str, lam: float, n, shifts: Sequence[float],
                 u=(1.0, 0.0, 0.0), stencil: int = 26, dt: float = 0.1):
    """F for the front of normal n shifted by each value of `shifts` along n.
    S is the loaded binding module (paper_1910_05180_amd.spfm)."""
    nv = np.asarray(n, dtype=np.float64)
    nv = nv / np.linalg.norm(nv)
    out = []
    with S.Spfm(LINE, lam=lam, mu=0.0, stencil=stencil, dtype="f64", coupling=coupling, u=u,
                walls=7, wall_sin=S.front_wall_sin(nv), dt=dt, allow_unstable=True,
                kernel="plain") as s:
        info = s.info()
        A = 2.0 * info["M"] / (3.0 * info["C_Gamma"] * lam * lam)
        for c in shifts:
            s.init_front(nv, float(c))
            before = s.diagnostics()["sum_phi"]
            s.step(1)
            after = s.diagnostics()["sum_phi"]
            out.append((after - before) / (dt * A))
    return out


def amplitude(S, *, coupling: str, lam: float, n, u=(1.0, 0.0, 0.0), samples: int = 12,
              stencil: int = 26) -> float:
    """Half the peak-to-peak force over shifts spanning one grid spacing."""
    F = front_forces(S, coupling=coupling, lam=lam, n=n, u=u, stencil=stencil,
                     shifts=[k / samples for k in range(samples)])
    return 0.5 * (max(F) - min(F))
