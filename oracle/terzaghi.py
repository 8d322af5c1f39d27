"""Terzaghi one-dimensional consolidation (closed form; pin of the oracle).

A column of height H, drained at the top (p = 0), undrained and fixed at the
bottom, laterally confined, loaded at t = 0+ by a compressive stress of
magnitude ``load``.  With storage S_eps, Biot coefficient b and the
constrained modulus lambda + 2G, the initial (undrained) pressure is
p0 = b load / (b^2 + S_eps (lambda + 2G)) and the consolidation coefficient is
c_v = (kappa/mu) / (S_eps + b^2 / (lambda + 2G)).  The pressure at depth zeta
(measured down from the drained top) is the Fourier series
    p = sum_m (2 p0 / M_m) sin(M_m zeta / H) exp(-M_m^2 c_v t / H^2),
    M_m = pi (2m + 1) / 2.
Textbook result (Terzaghi 1923; e.g. Wang, Theory of Linear Poroelasticity).
"""
from __future__ import annotations

import numpy as np


def consolidation_coefficient(kappa, mu, S_eps, biot, lam, G):
    return (kappa / mu) / (S_eps + biot ** 2 / (lam + 2.0 * G))


def initial_pressure(load, S_eps, biot, lam, G):
    return biot * load / (biot ** 2 + S_eps * (lam + 2.0 * G))


def pressure(zeta, t, H, cv, p0, terms=2000):
    zeta = np.asarray(zeta, dtype=np.float64)
    m = np.arange(terms)
    M = np.pi * (2 * m + 1) / 2.0
    s = (2.0 * p0 / M)[None, :] * np.sin(np.outer(zeta / H, M)) * np.exp(-M ** 2 * cv * t / H ** 2)[None, :]
    return s.sum(axis=1)
