"""Manufactured solutions: exact continuous right-hand side of paper Eq. (1)
(in the compact form of Eq. 12-15) for smooth analytic fields, built with
sympy from the continuous equations, independently of any discrete code.

RHS_i = d/dx_j E_ij - d/dx_j F_ij with
  E_j = [rho u_j, rho u_i u_j + p delta_ij, (e + p) u_j]
  F_j = [0, tau_ij, u_i tau_ij + (kappa + kappa_sgs) dT/dx_j]
where tau_ij = 2 (mu + mu_sgs)(S_ij - S_kk delta_ij / 3), mu from Sutherland's
law, kappa = mu Cp/Pr, kappa_sgs = mu_sgs Cp/Pr_sgs and, when requested, an
eddy viscosity mu_sgs = rho ls^2 sqrt(2 S_ij S_ij) with a fixed length ls,
and the isotropic SGS stress sigma_kk = 2 rho cl^2 (2 S_ij S_ij) with a fixed
length cl, which Eq. 1 adds to the momentum flux as sigma_kk delta_ij / 3 and
to the energy flux as sigma_kk u_j / 3.
The heat flux is taken as physical Fourier conduction (energy gains
div(kappa grad T)).
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp

X, Y, Z = sp.symbols("x y z", real=True)


def fields(gamma):
    rho = 1 + sp.Rational(1, 10) * sp.sin(X + sp.Rational(1, 2)) * sp.cos(Y) + sp.Rational(1, 20) * sp.cos(Z)
    u = sp.Rational(3, 10) * sp.sin(Y + sp.Rational(1, 5)) * sp.cos(Z) + sp.Rational(1, 10) * sp.cos(X)
    v = sp.Rational(1, 5) * sp.cos(X) * sp.sin(Z) + sp.Rational(1, 10)
    w = sp.Rational(1, 4) * sp.sin(X + Y) + sp.Rational(1, 20) * sp.cos(Z)
    p = (1 + sp.Rational(1, 10) * sp.cos(X) * sp.sin(Y + sp.Rational(2, 5)) * sp.cos(Z + sp.Rational(1, 10))) / gamma
    return rho, u, v, w, p


@functools.lru_cache(maxsize=None)
def exact_rhs(gamma, R_gas, mu_ref, T_ref, S_suth, Pr, Pr_sgs, ls, cl=0.0):
    """Returns (prim_fn, rhs_fn): numpy callables of (x, y, z)."""
    g = sp.nsimplify(gamma)
    rho, u, v, w, p = fields(g)
    vel = [u, v, w]
    xs = [X, Y, Z]
    T = p / (rho * R_gas)
    e = p / (g - 1) + rho * (u * u + v * v + w * w) / 2
    Cp = g * R_gas / (g - 1)
    th = T / T_ref
    mu = mu_ref * th ** sp.Rational(3, 2) * (1 + S_suth) / (th + S_suth)
    du = [[sp.diff(vel[a], xs[b]) for b in range(3)] for a in range(3)]
    S = [[(du[a][b] + du[b][a]) / 2 for b in range(3)] for a in range(3)]
    Skk = S[0][0] + S[1][1] + S[2][2]
    SS = sum(S[a][b] ** 2 for a in range(3) for b in range(3))
    if ls > 0:
        mu_sgs = rho * ls ** 2 * sp.sqrt(2 * SS)
    else:
        mu_sgs = sp.Integer(0)
    sig3 = 2 * rho * cl ** 2 * (2 * SS) / 3 if cl > 0 else sp.Integer(0)  # sigma_kk / 3
    tau = [[2 * (mu + mu_sgs) * (S[a][b] - (Skk / 3 if a == b else 0)) for b in range(3)] for a in range(3)]
    kap = mu * Cp / Pr + mu_sgs * Cp / Pr_sgs
    gradT = [sp.diff(T, xs[b]) for b in range(3)]
    rhs = []
    rhs.append(sum(sp.diff(rho * vel[j], xs[j]) for j in range(3)))
    for i in range(3):
        rhs.append(sum(sp.diff(rho * vel[i] * vel[j] + (p + sig3 if i == j else 0) - tau[i][j], xs[j])
                       for j in range(3)))
    rhs.append(sum(sp.diff((e + p + sig3) * vel[j] - sum(vel[i] * tau[i][j] for i in range(3)) - kap * gradT[j],
                           xs[j]) for j in range(3)))
    prim_fn = sp.lambdify((X, Y, Z), [rho, u, v, w, p], modules="numpy", cse=True)
    rhs_fn = sp.lambdify((X, Y, Z), rhs, modules="numpy", cse=True)
    return prim_fn, rhs_fn


def evaluate(fn, xyz):
    out = fn(xyz[0], xyz[1], xyz[2])
    return np.stack([np.broadcast_to(np.asarray(o, dtype=np.float64), xyz.shape[1:]) for o in out])
