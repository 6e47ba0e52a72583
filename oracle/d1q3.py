"""Lumped one-dimensional form of the D3Q19 scheme (TEST INFRASTRUCTURE).

On an nx = ny = 1 lattice with periodic x and y every pull in x and y returns to
the cell itself, so the D3Q19 populations that share e_z move together.  Summing
the paper's equilibria (eqs. equil1s, equil2as, equil2bs) over each group, with
beta along z only (b_i = e_iz beta), gives a three-velocity scheme:

  group +1 (e_z = +1): weights 1/18 + 4/36 = 1/6,
  group  0 (e_z =  0): rest 1/3, plus 4/18 + 4/36 = 1/3 of moving directions,
  group -1 (e_z = -1): 1/6,

  F_pm   = (1/6) n gamma (1 pm 3 beta / c_l),   F_0 = (2/3) n gamma,
  G_pm   = (1/6) e gamma^2 [1/(gamma^2 c_l^2) pm 4 beta/c_l + 4 beta^2/c_l^2],
  G_0    = (1/3) e gamma^2 [4 - (1 + c_l^2)/(gamma^2 c_l^2) - 4 beta^2/c_l^2],

(the moving rest-group members contribute (1/3) e gamma^2 [1/(gamma^2 c_l^2) -
2 beta^2/c_l^2], the rest particle w_0 e gamma^2 [4 - (2 + c_l^2)/(gamma^2 c_l^2)
- 2 beta^2/c_l^2]).  Moments: N = sum F, E = sum G, M = c_l (G_+ - G_-).  This is
written from the formulas independently of the D3Q19 oracle and pins its
streaming, indexing and summation on 1-D problems.

Inversion under e = 3P: with W = (4/3) e gamma^2 the constraints give
3W^2 - 4EW + M^2 = 0; the physical root is W = (2E + sqrt(4E^2 - 3M^2))/3,
beta = M/W, e = 3(W - E), gamma = 1/sqrt(1 - beta^2), n = N/gamma.
"""
from __future__ import annotations

import numpy as np


def equilibria(n, e, beta, c_l):
    g2 = 1.0 / (1.0 - beta * beta)
    g = np.sqrt(g2)
    c2 = c_l * c_l
    F = np.stack([(1 / 6) * n * g * (1 - 3 * beta / c_l), (2 / 3) * n * g,
                  (1 / 6) * n * g * (1 + 3 * beta / c_l)])
    Gm = (1 / 6) * e * g2 * (1 / (g2 * c2) - 4 * beta / c_l + 4 * beta * beta / c2)
    Gp = (1 / 6) * e * g2 * (1 / (g2 * c2) + 4 * beta / c_l + 4 * beta * beta / c2)
    G0 = (1 / 3) * e * g2 * (4 - (1 + c2) / (g2 * c2) - 4 * beta * beta / c2)
    return F, np.stack([Gm, G0, Gp])


def invert(F, G, c_l):
    N = F.sum(axis=0)
    E = G.sum(axis=0)
    M = c_l * (G[2] - G[0])
    W = (2 * E + np.sqrt(4 * E * E - 3 * M * M)) / 3
    beta = M / W
    e = 3 * (W - E)
    n = N * np.sqrt(1 - beta * beta)
    return n, e, beta


def run(n0, e0, beta0, tau, c_l, nsteps, bc="outflow"):
    """Run nsteps on a line of nz cells; returns (n, e, beta) at the end.
    bc = 'outflow' (zero-gradient copy at both ends) or 'periodic'.  Every
    operation is analytic, so complex inputs (tau + i h, e0 + i h v) give
    complex-step derivatives."""
    as_arr = lambda a: np.asarray(a) if np.iscomplexobj(a) else np.asarray(a, float)
    F, G = equilibria(as_arr(n0), as_arr(e0), as_arr(beta0), c_l)
    om = 1.0 / tau
    for _ in range(nsteps):
        # pull streaming: + group comes from z-1, - group from z+1
        if bc == "periodic":
            F = np.stack([np.roll(F[0], -1), F[1], np.roll(F[2], 1)])
            G = np.stack([np.roll(G[0], -1), G[1], np.roll(G[2], 1)])
        else:
            F = np.stack([np.concatenate([F[0][1:], F[0][-1:]]), F[1],
                          np.concatenate([F[2][:1], F[2][:-1]])])
            G = np.stack([np.concatenate([G[0][1:], G[0][-1:]]), G[1],
                          np.concatenate([G[2][:1], G[2][:-1]])])
        n, e, b = invert(F, G, c_l)
        Fe, Ge = equilibria(n, e, b, c_l)
        F = F - om * (F - Fe)
        G = G - om * (G - Ge)
    return invert(F, G, c_l)
