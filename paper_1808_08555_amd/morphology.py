"""Equilibrium morphology of two droplets (fluids 0 and 1) in a matrix (fluid 2) from the
three interfacial tensions, by the Neumann inequalities behind the seven cases of the
paper's stability-diagram study (Sec. 4.1):

  sigma_gb >  sigma_rg + sigma_rb : fluid 0 completely engulfs fluid 1
  sigma_gb == sigma_rg + sigma_rb : critical engulfing of fluid 1 by fluid 0
  sigma_rb >  sigma_rg + sigma_gb : fluid 1 completely engulfs fluid 0
  sigma_rb == sigma_rg + sigma_gb : critical engulfing of fluid 0 by fluid 1
  sigma_rg >  sigma_rb + sigma_gb : separate droplets (non-engulfing)
  sigma_rg == sigma_rb + sigma_gb : kissing
  otherwise (a Neumann triangle)  : partial engulfing (Janus droplet)
"""
from __future__ import annotations

ENGULF_1_BY_0 = "complete engulfing of 1 by 0"
CRITICAL_1_BY_0 = "critical engulfing of 1 by 0"
ENGULF_0_BY_1 = "complete engulfing of 0 by 1"
CRITICAL_0_BY_1 = "critical engulfing of 0 by 1"
SEPARATE = "separate"
KISSING = "kissing"
PARTIAL = "partial engulfing"


def classify(sigma_rg: float, sigma_rb: float, sigma_gb: float, rtol: float = 1e-9) -> str:
    def cmp(big, a, b):
        d = big - (a + b)
        tol = rtol * (abs(big) + abs(a) + abs(b))
        return 0 if abs(d) <= tol else (1 if d > 0 else -1)

    c = cmp(sigma_gb, sigma_rg, sigma_rb)
    if c > 0:
        return ENGULF_1_BY_0
    if c == 0:
        return CRITICAL_1_BY_0
    c = cmp(sigma_rb, sigma_rg, sigma_gb)
    if c > 0:
        return ENGULF_0_BY_1
    if c == 0:
        return CRITICAL_0_BY_1
    c = cmp(sigma_rg, sigma_rb, sigma_gb)
    if c > 0:
        return SEPARATE
    if c == 0:
        return KISSING
    return PARTIAL
