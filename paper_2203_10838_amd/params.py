"""Parameter formulas from the paper used to configure a solve (host side)."""
from __future__ import annotations


def optimal_alpha(eta: int, fro2: float, smax2: float) -> float:
    """Optimal uniform relaxation alpha* = eta / (1 + (eta-1) sigma_max^2 / ||A||_F^2).

    Corollary cor:linear_convergence (b), uniform weights W = alpha I; alpha*(1) = 1 and
    1 < alpha* <= eta for eta > 1 (Remark rmk:rmk_lc).
    """
    return float(eta) / (1.0 + (float(eta) - 1.0) * smax2 / fro2)


def default_eta(m: int, n: int) -> int:
    """The experiments' default batch size eta = 1 + min(m, n)/10 (Sec. 5), rounded down."""
    return 1 + min(m, n) // 10
