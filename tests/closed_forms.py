"""Closed forms that pin the oracle and the HIP path independently of either
(test helpers; no registration code)."""
import math

import numpy as np


def decoupled_ramp_history(nx, ny, nz, t, alpha, iters):
    """Closed-form history of the passive force (Eq 1 with alpha) on S = x,
    M = x + t (0 < t <= 1), with a smoothing so narrow that it is the identity
    (sigma 0.05, R 1: the side weights are about 1e-87).  t = 0.75 keeps
    every grid value of M exact in FP32.  Every voxel then
    evolves on its own, and only its x position matters:
      - interior x: grad S = 1, D = t - v, so e = t - v obeys
        e' = e - e / (alpha^2 e^2 + 1);
      - x = 0: grad S = 1/2 (clamped neighbour) and the sample x - v < 0
        clamps onto M(0) = t, so D = t for ever and v grows by
        (t / 2) / (alpha^2 t^2 + 1/4) per iteration;
      - x = nx - 1: grad S = 1/2, D = t - v = e, so
        e' = e - (e / 2) / (alpha^2 e^2 + 1/4).
    Returns the rows (sum|dr|, sum|v| before the update, mean D^2, l) of
    Sec 2.4's relative norm over the whole volume."""
    a2 = alpha * alpha
    e_int, e_end, v0 = t, t, 0.0
    rows = []
    for _ in range(iters):
        dr0 = 0.5 * t / (a2 * t * t + 0.25)
        dri = e_int / (a2 * e_int * e_int + 1.0)
        dre = 0.5 * e_end / (a2 * e_end * e_end + 0.25)
        s1 = ny * nz * (abs(dr0) + (nx - 2) * abs(dri) + abs(dre))
        s2 = ny * nz * (abs(v0) + (nx - 2) * abs(t - e_int) + abs(t - e_end))
        mse = (t * t + (nx - 2) * e_int * e_int + e_end * e_end) / nx
        rows.append((s1, s2, mse, s1 / s2 if s2 > 0 else math.nan))
        v0, e_int, e_end = v0 + dr0, e_int - dri, e_end - dre
    return np.array(rows)


def decoupled_ramp(nx, ny, nz, t):
    gx = np.broadcast_to(np.arange(nx, dtype=float), (nz, ny, nx)).copy()
    return gx, gx + t


def stop_eps(l, n_stop):
    """An eps for which the rule l(n-10) - l(n) <= eps first holds at
    iteration n_stop (midway between that drop and the one before, which the
    closed form shows to decrease monotonically)."""
    d = {n: l[n - 10] - l[n] for n in range(11, len(l))}
    assert all(d[n] > d[n + 1] for n in range(11, len(l) - 1))
    return 0.5 * (d[n_stop] + d[n_stop - 1])
