"""Analytic solution of the ultra-relativistic Sod shock tube in (d+1) dimensions (App. D).

Oracle module (test infrastructure only; see ``oracle/__init__``).

An inviscid gas of massless particles, P = n T and eps = d P, starts at rest
with (P_L, n_L) for x < 0 and (P_R, n_R) for x > 0 (P_L > P_R).  The solution
is self-similar in w = x/t (c = 1):
* a rarefaction fan to the left, between its head x_H = -t/sqrt(d) and its
  tail x_T, along which n ((1 + beta)/(1 - beta))^(sqrt(d)/2) and
  P ((1 + beta)/(1 - beta))^((d+1)/(2 sqrt(d))) keep their left values and the
  fluid speed follows from the characteristic w = (beta - c_s)/(1 - beta c_s),
  c_s = 1/sqrt(d);
* a plateau of pressure P_C and speed beta_C, split by the contact
  discontinuity x_C = beta_C t into densities n_I (fan side) and n_II (shock
  side);
* a shock at x_S = beta_s t, whose speed and jump follow from the
  Rankine-Hugoniot conditions in the shock's rest frame.
P_C solves the matching of the fan's tail speed with the shock-side plateau
speed; it is found by bracketing root search on (P_R, P_L).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize


def _beta_c(d: int, PC: float, PR: float) -> float:
    """Plateau speed from the shock relations."""
    return math.sqrt(d * (PC - PR) ** 2 / ((PR + d * PC) * (PC + d * PR)))


def plateau_pressure(d: int, PL: float, PR: float) -> float:
    """P_C: the fan's tail speed, ((P_L/P_C)^k - 1)/((P_L/P_C)^k + 1) with k = 2 sqrt(d)/(d+1),
    equals the shock-side speed beta_C(P_C)."""
    k = 2.0 * math.sqrt(d) / (d + 1)

    def g(PC):
        r = (PL / PC) ** k
        return (r - 1.0) / (r + 1.0) - _beta_c(d, PC, PR)
    return optimize.brentq(g, PR * (1 + 1e-15), PL * (1 - 1e-15), xtol=1e-16, rtol=1e-15, maxiter=500)


def waves(d: int, PL: float, nL: float, PR: float, nR: float) -> dict:
    """The constants of the solution: P_C, beta_C, beta_s, n_I, n_II and the self-similar positions
    w = x/t of the fan's head and tail, the contact and the shock."""
    sd = math.sqrt(d)
    PC = plateau_pressure(d, PL, PR)
    bC = _beta_c(d, PC, PR)
    bs = math.sqrt((PR + d * PC) / (d * (PC + d * PR)))
    nI = nL * (PC / PL) ** (d / (d + 1))
    nII = nR * math.sqrt(PC * (PR + d * PC) / (PR * (PC + d * PR)))
    return {"PC": PC, "beta_C": bC, "beta_s": bs, "n_I": nI, "n_II": nII,
            "w_H": -1.0 / sd, "w_T": (bC - 1.0 / sd) / (1.0 - bC / sd), "w_C": bC, "w_S": bs}


def solution(d: int, PL: float, nL: float, PR: float, nR: float, x, t: float) -> dict:
    """n, P, T = P/n and beta at positions x (membrane at x = 0) and time t > 0."""
    x = np.asarray(x, dtype=np.float64)
    c = waves(d, PL, nL, PR, nR)
    sd = math.sqrt(d)
    w = x / t
    n = np.empty_like(x)
    P = np.empty_like(x)
    b = np.empty_like(x)
    left = w <= c["w_H"]
    fan = (w > c["w_H"]) & (w <= c["w_T"])
    zI = (w > c["w_T"]) & (w <= c["w_C"])
    zII = (w > c["w_C"]) & (w <= c["w_S"])
    right = w > c["w_S"]
    n[left], P[left], b[left] = nL, PL, 0.0
    wf = w[fan]
    ratio = (1.0 - 1.0 / sd) * (1.0 - wf) / ((1.0 + 1.0 / sd) * (1.0 + wf))
    n[fan] = nL * ratio ** (sd / 2.0)
    P[fan] = PL * ratio ** ((d + 1) / (2.0 * sd))
    b[fan] = (wf + 1.0 / sd) / (1.0 + wf / sd)
    n[zI], P[zI], b[zI] = c["n_I"], c["PC"], c["beta_C"]
    n[zII], P[zII], b[zII] = c["n_II"], c["PC"], c["beta_C"]
    n[right], P[right], b[right] = nR, PR, 0.0
    return {"n": n, "P": P, "T": P / n, "beta": b}
