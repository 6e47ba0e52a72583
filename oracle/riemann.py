"""Exact ideal relativistic Riemann solution for P = e/3 (TEST INFRASTRUCTURE).

The paper validates its scheme on the Riemann problem of a membrane removed at
t = 0 between two equilibrated states at rest (the shock-tube section).  In the
limit of vanishing viscosity the lattice solution approaches the ideal
(Euler) relativistic Riemann solution, which for the ultra-relativistic
equation of state e = 3P has a closed form up to one scalar root:

  * left-moving rarefaction into the high-pressure state: the Riemann invariant
    artanh(beta) + (sqrt(3)/4) ln e is constant, so
    beta(e) = tanh((sqrt(3)/4) ln(e_L / e)); inside the fan the local
    characteristic speed (beta - c_s)/(1 - beta c_s) equals z/t, c_s = 1/sqrt(3);
  * right-moving shock into the low-pressure state at rest: the Taub jump gives
    beta*^2 = (P* - P_R)(e* - e_R) / ((P* + e_R)(e* + P_R)) and the shock speed
    follows from energy conservation across it, v_s = A beta* / (A - P* - e_R),
    A = (e* + P*) gamma*^2;
  * number density: isentropic n ~ e^(3/4) through the fan; across the shock
    n* = v_s n_R / (gamma* (v_s - beta*)) (particle-number conservation).

The two curves beta_rare(e) and beta_shock(e) meet at the intermediate state e*,
found by bracketing on (e_R, e_L).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.optimize import brentq

CS = 1.0 / math.sqrt(3.0)


def beta_rarefaction(e, e_L):
    return np.tanh((math.sqrt(3.0) / 4.0) * np.log(e_L / e))


def beta_shock(e, e_R):
    P, P_R = e / 3.0, e_R / 3.0
    return np.sqrt((P - P_R) * (e - e_R) / ((P + e_R) * (e + P_R)))


@dataclass
class Star:
    e_L: float
    e_R: float
    n_L: float
    n_R: float
    e_star: float
    beta_star: float
    v_shock: float
    n_star_L: float
    n_star_R: float

    @property
    def xi_head(self):
        return -CS

    @property
    def xi_tail(self):
        return (self.beta_star - CS) / (1.0 - self.beta_star * CS)


def solve(e_L: float, e_R: float, n_L: float = None, n_R: float = None) -> Star:
    """Intermediate state of the ideal Riemann problem (left state denser)."""
    if n_L is None:
        n_L = e_L ** 0.75
    if n_R is None:
        n_R = e_R ** 0.75
    assert e_L > e_R > 0
    f = lambda e: beta_rarefaction(e, e_L) - beta_shock(e, e_R)
    e_star = brentq(f, e_R * (1 + 1e-15), e_L * (1 - 1e-15), xtol=1e-16, rtol=1e-15, maxiter=500)
    b = float(beta_rarefaction(e_star, e_L))
    g2 = 1.0 / (1.0 - b * b)
    P = e_star / 3.0
    A = (e_star + P) * g2
    vs = A * b / (A - P - e_R)
    nL = n_L * (e_star / e_L) ** 0.75
    nR = vs * n_R / (math.sqrt(g2) * (vs - b))
    return Star(e_L, e_R, n_L, n_R, e_star, b, vs, nL, nR)


def profile(st: Star, xi: np.ndarray):
    """(e, beta, n) at similarity coordinates xi = (z - z0)/t."""
    xi = np.asarray(xi, dtype=np.float64)
    e = np.empty_like(xi)
    b = np.empty_like(xi)
    n = np.empty_like(xi)
    left = xi <= st.xi_head
    fan = (xi > st.xi_head) & (xi <= st.xi_tail)
    starL = (xi > st.xi_tail) & (xi <= st.beta_star)
    starR = (xi > st.beta_star) & (xi <= st.v_shock)
    right = xi > st.v_shock
    e[left], b[left], n[left] = st.e_L, 0.0, st.n_L
    bf = (xi[fan] + CS) / (1.0 + xi[fan] * CS)
    ef = st.e_L * np.exp(-(4.0 / math.sqrt(3.0)) * np.arctanh(bf))
    e[fan], b[fan], n[fan] = ef, bf, st.n_L * (ef / st.e_L) ** 0.75
    e[starL], b[starL], n[starL] = st.e_star, st.beta_star, st.n_star_L
    e[starR], b[starR], n[starR] = st.e_star, st.beta_star, st.n_star_R
    e[right], b[right], n[right] = st.e_R, 0.0, st.n_R
    return e, b, n


def lattice_profile(st: Star, nz: int, t: float, z0: float = None):
    """Exact fields at lattice cell centres k + 1/2 (membrane at z0 = nz/2), c = 1,
    one cell = one unit of length, t in the same units."""
    if z0 is None:
        z0 = nz / 2.0
    z = np.arange(nz) + 0.5
    return profile(st, (z - z0) / t)
