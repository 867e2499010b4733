"""Cost model of the method (oracle side; test infrastructure).

  I(A, eps1) = omega * N1 + N2                  eq. (4)
  E = (1 - I / I_dp) * 100 %                     eq. (12)
  E over a test set uses sums of I and I_dp      eq. (27)
  class label = argmin over eps1 = 10^-t, t = 2..7, of I; ties go to the
                larger eps1 (smaller t)          classification section, eq. (23)
  N_S bound without preconditioning               eq. (26)
"""

from __future__ import annotations

import math

EPS1_CANDIDATES = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7)


def cost_I(n1: int, n2: int, omega: float) -> float:
    return omega * n1 + n2


def efficiency(I: float, I_dp: float) -> float:
    return (1.0 - I / I_dp) * 100.0


def overall_efficiency(Is, I_dps) -> float:
    return (1.0 - sum(Is) / sum(I_dps)) * 100.0


def label_from_sweep(n1s, n2s, omega: float) -> int:
    """Class t of the eps1 candidate with the smallest I (first = larger eps1 on ties)."""
    best_t, best_I = None, None
    for j, (a, b) in enumerate(zip(n1s, n2s)):
        I = cost_I(a, b, omega)
        if best_I is None or I < best_I:
            best_t, best_I = j + 2, I
    return best_t


def ns_bound(n: int, m: int, k_cg: float, k: int, alpha: float = 0.01) -> float:
    """Largest admissible training-sample size of eq. (26) (before rounding)."""
    c = m / n
    return alpha * 4.0 * (6.0 * c + 17.0) * n * k_cg / (44.0 + 3.0 * k)


def knn_iteration_cycles(k: int) -> int:
    """Cycles of one kNN iteration, eq. (24): 44 + 3k."""
    return 44 + 3 * k


def cg_dp_cycles(n: int, m: int, k_cg: float) -> float:
    """Cycles of unpreconditioned FP64 CG, eq. (19)."""
    return 4.0 * (6.0 * m + 17.0 * n) * k_cg


def bfs2_cycles(m: int) -> int:
    """Cycles of 2BFS: 2m (section on the complexity of the features)."""
    return 2 * m


def cg_iteration_bound(kappa: float, eps: float) -> int:
    """Iteration bound of eq. (9): ceil(0.5 * sqrt(kappa) * ln(2 / eps))."""
    return math.ceil(0.5 * math.sqrt(kappa) * math.log(2.0 / eps))
