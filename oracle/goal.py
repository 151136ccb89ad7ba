"""Goal function of the paper's parameter-fitting study (Sec. 4.3): test
infrastructure only, written from eq:goal, eq:goalvariance, eq:goalsigma and
eq:residuall.

Sample trajectory i of parameter vector k gives, per region j (the set C(j)
of its nodes) and time t, the vector of compartment counts summed over C(j);
the goal compares their mean over the N trajectories with the same sums of a
reference trajectory. The integral over t in [0, T] is taken as the sum over
the daily records (dt = 1 day, the state at the end of each day).
"""
import numpy as np


def goal(regional, reference):
    """regional[D][N][J][Nc]: regional aggregates of N sample trajectories;
    reference[D][J][Nc]: those of the reference trajectory. Returns
    (G^2, VG^2) of eq:goal and eq:goalvariance (VG^2 = 0 for N = 1)."""
    x = np.asarray(regional, dtype=np.float64)
    ref = np.asarray(reference, dtype=np.float64)
    N = x.shape[1]
    mean = x.sum(axis=1) / N                          # x-bar_j(t; k)
    G2 = float(((mean - ref) ** 2).sum())             # sum over t, j of || . ||^2
    if N < 2:
        return G2, 0.0
    sigma2 = ((x - mean[:, None]) ** 2).sum(axis=(1, 3)) / (N - 1)   # eq:goalsigma, [D][J]
    return G2, float(sigma2.sum())


def residual(G, G_ref):
    """Relative residual R(k) of eq:residuall."""
    return abs(G - G_ref) / abs(G_ref)
