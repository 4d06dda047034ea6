"""Seeded synthetic inputs: grids, flow parameters and initial states.

This module builds inputs only.  It holds none of the method's arithmetic
(no metrics, fluxes, dissipation, residual or time stepping); the one physical
relation it uses is the ideal-gas total energy e = p/(gamma-1) + rho|u|^2/2
(paper Eq. 2) to turn an analytic primitive field into the conserved input
state.  Both the oracle tests and the GPU path consume these arrays.

Every array is float64 on the padded box (nfields, nk+4, nj+4, ni+4): two
ghost layers per side, i fastest; interior index 0..n-1 is stored at n+2.
Coordinates are given on every node of the padded box; in a periodic
direction the ghost coordinates are the period-shifted images (the analytic
mappings below are periodic up to a translation, so evaluating them at the
ghost indices gives exactly that).

Workloads (nondimensional, acoustic scaling rho_inf = T_inf = c_inf = 1,
R = 1/gamma, p_inf = 1/gamma):
  * ``tgv_case``: Taylor-Green vortex, Mach 0.1, Re 1600, unit Cartesian
    metrics, periodic in all three directions.
  * ``jet_case``: one GPU's share of the paper's jet (Sec. 5.1): perfectly
    expanded Mach 1.4 jet, PR = TR = 1, Re_D = 1.57e6, on a stretched,
    smoothly wavy curvilinear grid (tanh clustering across the shear layers),
    periodic in i (axial) and k (spanwise), frozen far-field ghosts in j.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def flow_params(**over) -> dict:
    """Default flow/scheme parameters (jet values); keyword overrides."""
    p = dict(
        gamma=GAMMA,
        Pr=0.72,               # paper Eq. 4
        Pr_sgs=0.9,            # paper Eq. 5 (static closure)
        mu_ref=1.4 / 1.57e6,   # rho_j U_j D / Re_D with U_j = M_j c_inf = 1.4, D = 1
        T_ref=1.0,
        S_suth=110.4 / 288.15, # Sutherland S1 = 110.4 K over a 288.15 K reference
        R_gas=1.0 / GAMMA,
        sgs=1,
        Cs=0.17,
        k2=0.25,
        k4=1.0 / 64.0,
        alpha=0.5,
        cfl=0.5,
        CI=0.0,                # isotropic SGS constant (sigma_kk model); 0 = off
    )
    p.update(over)
    return p


def padded_indices(n: int) -> np.ndarray:
    """Index values -2 .. n+1 of one padded axis."""
    return np.arange(-2, n + 2, dtype=np.float64)


def cons_from_prim(rho, u, v, w, p, gamma=GAMMA) -> np.ndarray:
    """Conserved input state [rho, rho u, rho v, rho w, e] (Eq. 2)."""
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, e]), dtype=np.float64)


def _mesh(ni, nj, nk):
    I = padded_indices(ni)[None, None, :]
    J = padded_indices(nj)[None, :, None]
    K = padded_indices(nk)[:, None, None]
    return I, J, K


# ---------------------------------------------------------------------------
# Taylor-Green vortex on the unit Cartesian box
# ---------------------------------------------------------------------------
def tgv_case(n: int = 32, mach: float = 0.1, re: float = 1600.0, sgs: int = 1) -> dict:
    I, J, K = _mesh(n, n, n)
    shape = (n + 4, n + 4, n + 4)
    x = np.broadcast_to(I, shape)
    y = np.broadcast_to(J, shape)
    z = np.broadcast_to(K, shape)
    xyz = np.ascontiguousarray(np.stack([x, y, z]), dtype=np.float64)
    L = n / (2.0 * math.pi)
    V0 = mach  # c0 = 1
    rho0, p0 = 1.0, 1.0 / GAMMA
    u = V0 * np.sin(x / L) * np.cos(y / L) * np.cos(z / L)
    v = -V0 * np.cos(x / L) * np.sin(y / L) * np.cos(z / L)
    w = np.zeros(shape)
    p = p0 + rho0 * V0 * V0 / 16.0 * (np.cos(2 * x / L) + np.cos(2 * y / L)) * (np.cos(2 * z / L) + 2.0)
    rho = p / (flow_params()["R_gas"] * 1.0)  # uniform T0 = 1
    Q = cons_from_prim(rho, u, v, w, p)
    prm = flow_params(mu_ref=rho0 * V0 * L / re, sgs=sgs)
    return dict(name=f"tgv{n}", ni=n, nj=n, nk=n, bc=(0, 0, 0), xyz=xyz, Q=Q, params=prm,
                p_inf=p0, period=(float(n), float(n), float(n)))


# ---------------------------------------------------------------------------
# Jet shard grid: tanh clustering in j plus a smooth wavy mapping.
# ---------------------------------------------------------------------------
def _logcosh(x):
    return np.logaddexp(x, -x) - math.log(2.0)


def _cluster(t, a=0.8, w=0.05, tR=0.55):
    """Integral of 1 - (a/2)[tanh((t+tR)/w) - tanh((t-tR)/w)]: spacing is
    (1-a) times the outer spacing for |t| < tR."""
    return t - a * (w / 2.0) * (_logcosh((t + tR) / w) - _logcosh((t - tR) / w))


def jet_grid(ni, nj, nk, Lx=7.5, Ly=10.0, Lz=2.5, m=2, amp=0.2) -> np.ndarray:
    """Coordinates (3, nk+4, nj+4, ni+4) of the curvilinear jet shard."""
    I, J, K = _mesh(ni, nj, nk)
    t = -1.0 + 2.0 * J / (nj - 1)
    Y1 = _cluster(np.array([1.0]))[0]
    Y = (Ly / 2.0) * _cluster(t) / Y1
    tin = -1.0 + 2.0 * np.arange(nj) / (nj - 1)
    dY = np.diff((Ly / 2.0) * _cluster(tin) / Y1).min()
    W = np.sin(2 * math.pi * m * I / ni) * np.sin(2 * math.pi * m * K / nk) * np.cos(math.pi * t)
    shape = (nk + 4, nj + 4, ni + 4)
    x = np.broadcast_to(Lx * I / ni + amp * (Lx / ni) * W, shape)
    y = np.broadcast_to(Y + amp * dY * W, shape)
    z = np.broadcast_to(Lz * K / nk + amp * (Lz / nk) * W, shape)
    return np.ascontiguousarray(np.stack([x, y, z]), dtype=np.float64)


def jet_state(xyz: np.ndarray, ni, nj, nk, seed=0, mach=1.4, R=0.5, theta=0.05, pert=0.01) -> np.ndarray:
    """Perfectly expanded jet: tanh double shear layer in y, Crocco-Busemann
    temperature (TR = 1), uniform p = p_inf, seeded velocity perturbations on
    the interior (uniform in [-1, 1], times a shear-layer envelope)."""
    y = xyz[1]
    Uj = mach
    u = 0.5 * Uj * (np.tanh((R + y) / (2 * theta)) + np.tanh((R - y) / (2 * theta)))
    s = u / Uj
    T = 1.0 + 0.5 * (GAMMA - 1.0) * mach * mach * s * (1.0 - s)
    p = np.full_like(u, 1.0 / GAMMA)
    rho = p / ((1.0 / GAMMA) * T)
    env = 4.0 * s * (1.0 - s)
    rng = np.random.default_rng(seed)
    r = rng.uniform(-1.0, 1.0, size=(3, nk, nj, ni))
    vel = [u.copy(), np.zeros_like(u), np.zeros_like(u)]
    inner = (slice(2, nk + 2), slice(2, nj + 2), slice(2, ni + 2))
    for c in range(3):
        vel[c][inner] += pert * Uj * r[c] * env[inner]
    return cons_from_prim(rho, vel[0], vel[1], vel[2], p)


def outside_state(case: dict, mach=1.4, R=0.5, theta=0.05, coflow=0.0, cross=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Outside state of the jet block's boundary faces on every node of the
    padded box: the unperturbed jet profile (the flat-hat-like tanh profile
    that the entrance imposes) with ambient pressure p_inf = 1/gamma, plus
    an optional uniform co-flow coflow * M_j along x and cross-flow
    cross * M_j.  Far from the jet this is the far-field state, whose
    velocity scale and temperature follow from the jet Mach number M_j."""
    y = case["xyz"][1]
    Uj = mach
    u = 0.5 * Uj * (np.tanh((R + y) / (2 * theta)) + np.tanh((R - y) / (2 * theta)))
    s = u / Uj
    T = 1.0 + 0.5 * (GAMMA - 1.0) * mach * mach * s * (1.0 - s)
    p = np.full_like(u, 1.0 / GAMMA)
    rho = p / ((1.0 / GAMMA) * T)
    vel = [u + (coflow + cross[0]) * Uj, np.full_like(u, cross[1] * Uj), np.full_like(u, cross[2] * Uj)]
    return cons_from_prim(rho, vel[0], vel[1], vel[2], p)


def jet_case(ni=256, nj=128, nk=128, seed=0, **kw) -> dict:
    scale = dict(Lx=7.5 * ni / 256, Ly=10.0, Lz=2.5 * nk / 128)
    scale.update({k: kw.pop(k) for k in list(kw) if k in ("Lx", "Ly", "Lz")})
    xyz = jet_grid(ni, nj, nk, **scale)
    Q = jet_state(xyz, ni, nj, nk, seed=seed)
    prm = flow_params(**kw)
    return dict(name=f"jet{ni}x{nj}x{nk}", ni=ni, nj=nj, nk=nk, bc=(0, 1, 0), xyz=xyz, Q=Q, params=prm,
                p_inf=1.0 / GAMMA, period=(scale["Lx"], None, scale["Lz"]))


# ---------------------------------------------------------------------------
# The paper's cylindrical O-grid (Sec. 3, Fig. 1; Tab. 2: 361 azimuthal
# points): i axial, j radial from the jet axis (j = 0 on the axis) to the far
# field, k azimuthal with the first and last points superposed.
# ---------------------------------------------------------------------------
def ogrid(ni, nj, nk=361, Lx=7.5, R_far=5.0) -> np.ndarray:
    """Coordinates (3, nk+4, nj+4, ni+4): x = Lx i / ni, y = r cos(th),
    z = r sin(th), th = 2 pi k / (nk - 1), with r(j) = R_far s(j / (nj - 1)),
    s the (odd) tanh-clustered map of the jet grid scaled to s(1) = 1, fine
    across the shear layer at r = 0.5 D.  Because s is odd, the ghost nodes
    j = -1, -2 are the points across the axis: (i, -m, k) coincides with
    (i, m, k + (nk - 1)/2)."""
    I, J, K = _mesh(ni, nj, nk)
    t = J / (nj - 1)
    r = R_far * _cluster(t) / _cluster(np.array([1.0]))[0]
    th = 2.0 * math.pi * K / (nk - 1)
    shape = (nk + 4, nj + 4, ni + 4)
    x = np.broadcast_to(Lx * I / ni, shape)
    y = np.broadcast_to(r * np.cos(th), shape)
    z = np.broadcast_to(r * np.sin(th), shape)
    return np.ascontiguousarray(np.stack([x, y, z]), dtype=np.float64)


def ogrid_case(ni=64, nj=48, nk=361, seed=0, Lx=None, R_far=5.0, mach=1.4, R=0.5, theta=0.05, pert=0.01,
               **kw) -> dict:
    """A round jet on the O-grid: the tanh profile in r, Crocco-Busemann T,
    uniform p, 1 % seeded velocity perturbations off the axis (shear-layer
    envelope).  Axis nodes hold the azimuthal mean of the ring j = 1, the
    duplicate azimuth k = nk - 1 equals k = 0.  i periodic (an axial shard),
    j: axis (bc 3) with frozen far-field ghosts at j-hi, k superposed."""
    Lx = 7.5 * ni / 256 if Lx is None else Lx
    xyz = ogrid(ni, nj, nk, Lx=Lx, R_far=R_far)
    r = np.sqrt(xyz[1] ** 2 + xyz[2] ** 2)
    Uj = mach
    u = 0.5 * Uj * (np.tanh((R + r) / (2 * theta)) + np.tanh((R - r) / (2 * theta)))
    sh = u / Uj
    T = 1.0 + 0.5 * (GAMMA - 1.0) * mach * mach * sh * (1.0 - sh)
    p = np.full_like(u, 1.0 / GAMMA)
    rho = p / ((1.0 / GAMMA) * T)
    env = 4.0 * sh * (1.0 - sh)
    rng = np.random.default_rng(seed)
    vel = [u.copy(), np.zeros_like(u), np.zeros_like(u)]
    inner = (slice(2, nk + 2), slice(3, nj + 2), slice(2, ni + 2))  # j >= 1
    for c in range(3):
        vel[c][inner] += pert * Uj * rng.uniform(-1.0, 1.0, size=(nk, nj - 1, ni)) * env[inner]
    Q = cons_from_prim(rho, vel[0], vel[1], vel[2], p)
    Q[:, nk + 1] = Q[:, 2]                                # duplicate azimuth
    Q[:, 2:nk + 2, 2] = Q[:, 2:nk + 1, 3].mean(axis=1)[:, None, :]  # axis: mean of ring j = 1
    prm = flow_params(**kw)
    return dict(name=f"ogrid{ni}x{nj}x{nk}", ni=ni, nj=nj, nk=nk, bc=(0, 3, 2), xyz=xyz, Q=Q, params=prm,
                p_inf=1.0 / GAMMA, period=(Lx, None, None))


# ---------------------------------------------------------------------------
# Generic test grids and states
# ---------------------------------------------------------------------------
def wavy_grid(ni, nj, nk, L=(1.0, 1.0, 1.0), amp=0.15, m=1) -> np.ndarray:
    """A box periodic in all three directions (periods L) with a smooth wavy
    interior mapping; every metric term is non-trivial."""
    I, J, K = _mesh(ni, nj, nk)
    a, b, c = 2 * math.pi * m * I / ni, 2 * math.pi * m * J / nj, 2 * math.pi * m * K / nk
    W1 = np.sin(a) * np.sin(b) * np.sin(c)
    W2 = np.sin(a + 0.3) * np.cos(b) * np.sin(2 * c)
    W3 = np.cos(a) * np.sin(2 * b + 0.1) * np.sin(c)
    shape = (nk + 4, nj + 4, ni + 4)
    x = np.broadcast_to(L[0] * (I / ni + amp / ni * (W1 + 0.5 * W2)), shape)
    y = np.broadcast_to(L[1] * (J / nj + amp / nj * (W2 + 0.5 * W3)), shape)
    z = np.broadcast_to(L[2] * (K / nk + amp / nk * (W3 + 0.5 * W1)), shape)
    return np.ascontiguousarray(np.stack([x, y, z]), dtype=np.float64)


def superposed_case(case: dict, axis: int) -> dict:
    """The block of a case that is periodic along `axis` (0 = i, 1 = j,
    2 = k), with one more node along it: node n is node 0 again (the first
    and last nodes superposed, as the azimuthal direction of the paper's
    O-grid), bc[axis] = 2.  Coordinates of node n and of the extra ghost
    plane are the period-shifted images; the state of node n is node 0's."""
    key = ("ni", "nj", "nk")[axis]
    n = case[key]
    ax = 3 - axis  # array axis of (c, k, j, i)

    def plane(a, x):  # padded plane of index x along the axis
        return np.take(a, x + 2, axis=ax)

    xyz, Q = case["xyz"], case["Q"]
    shift = plane(xyz, n) - plane(xyz, 0)  # one period
    px = [plane(xyz, x) for x in range(-2, n + 2)] + [plane(xyz, 2) + shift]
    pq = [plane(Q, x) for x in range(-2, n + 2)] + [plane(Q, 2)]
    pq[n + 2] = plane(Q, 0)  # node n is node 0
    out = dict(case)
    out[key] = n + 1
    out["xyz"] = np.ascontiguousarray(np.stack(px, axis=ax))
    out["Q"] = np.ascontiguousarray(np.stack(pq, axis=ax))
    bc = list(case["bc"])
    bc[axis] = 2
    out["bc"] = tuple(bc)
    out["name"] = case.get("name", "case") + f"_superposed{axis}"
    return out


def uniform_state(shape3, rho=1.0, vel=(0.8, 0.6, 0.7), p=1.0 / GAMMA) -> np.ndarray:
    one = np.ones(shape3)
    return cons_from_prim(rho * one, vel[0] * one, vel[1] * one, vel[2] * one, p * one)


def smooth_state(ni, nj, nk, seed=0, amp=0.05, base_vel=(0.3, -0.2, 0.1), modes=3) -> np.ndarray:
    """A random smooth periodic state: base flow plus a few seeded Fourier
    modes in index space (periodic in every direction)."""
    rng = np.random.default_rng(seed)
    I, J, K = _mesh(ni, nj, nk)
    shape = (nk + 4, nj + 4, ni + 4)
    fields = []
    base = [1.0, base_vel[0], base_vel[1], base_vel[2], 1.0 / GAMMA]
    for q in range(5):
        f = np.full(shape, base[q])
        for _ in range(modes):
            ka, kb, kc = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            a = rng.uniform(-1, 1) * amp * (abs(base[q]) if q in (0, 4) else 1.0)
            f = f + a * (np.cos(2 * math.pi * ka * I / ni + ph[0]) * np.cos(2 * math.pi * kb * J / nj + ph[1]) *
                         np.cos(2 * math.pi * kc * K / nk + ph[2]))
        fields.append(np.broadcast_to(f, shape))
    return cons_from_prim(*fields)


def periodic_case(ni, nj, nk, xyz, Q, **prm) -> dict:
    return dict(name=f"box{ni}x{nj}x{nk}", ni=ni, nj=nj, nk=nk, bc=(0, 0, 0), xyz=xyz, Q=Q,
                params=flow_params(**prm), p_inf=1.0 / GAMMA)


def interior(a: np.ndarray) -> np.ndarray:
    """Interior view (nf, nk, nj, ni) of a padded array."""
    return a[..., 2:-2, 2:-2, 2:-2]


# ---------------------------------------------------------------------------
# Device-side generator for large shards (same formulas, torch on the GPU;
# the random perturbations come from torch's device generator, so they differ
# from the numpy stream of jet_state).  Used for sizes whose host arrays
# would dominate the run time (e.g. 800 x 500 x 500).
# ---------------------------------------------------------------------------
def jet_case_device(ni, nj, nk, seed=0, device="cuda", Lx=None, Ly=10.0, Lz=None, m=2, amp=0.2, mach=1.4,
                    R=0.5, theta=0.05, pert=0.01):
    import torch
    Lx = 7.5 * ni / 256 if Lx is None else Lx
    Lz = 2.5 * nk / 128 if Lz is None else Lz
    f64 = dict(dtype=torch.float64, device=device)
    I_ = torch.arange(-2, ni + 2, **f64).view(1, 1, -1)
    J_ = torch.arange(-2, nj + 2, **f64).view(1, -1, 1)
    K_ = torch.arange(-2, nk + 2, **f64).view(-1, 1, 1)
    t = -1.0 + 2.0 * J_ / (nj - 1)

    def cl(x, a=0.8, w=0.05, tR=0.55):
        lc = lambda z: torch.logaddexp(z, -z) - math.log(2.0)
        return x - a * (w / 2.0) * (lc((x + tR) / w) - lc((x - tR) / w))
    Y1 = float(cl(torch.tensor([1.0], **f64))[0])
    Y = (Ly / 2.0) * cl(t) / Y1
    tin = -1.0 + 2.0 * torch.arange(nj, **f64) / (nj - 1)
    dY = float(torch.diff((Ly / 2.0) * cl(tin) / Y1).min())
    W = torch.sin(2 * math.pi * m * I_ / ni) * torch.sin(2 * math.pi * m * K_ / nk) * torch.cos(math.pi * t)
    shape = (nk + 4, nj + 4, ni + 4)
    xyz = torch.empty((3,) + shape, **f64)
    xyz[0] = (Lx * I_ / ni + amp * (Lx / ni) * W).expand(shape)
    xyz[1] = (Y + amp * dY * W).expand(shape)
    xyz[2] = (Lz * K_ / nk + amp * (Lz / nk) * W).expand(shape)
    y = xyz[1]
    u = 0.5 * mach * (torch.tanh((R + y) / (2 * theta)) + torch.tanh((R - y) / (2 * theta)))
    s_ = u / mach
    T = 1.0 + 0.5 * (GAMMA - 1.0) * mach * mach * s_ * (1.0 - s_)
    p = torch.full_like(u, 1.0 / GAMMA)
    rho = p / ((1.0 / GAMMA) * T)
    env = 4.0 * s_ * (1.0 - s_)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    vel = [u, torch.zeros_like(u), torch.zeros_like(u)]
    inner = (slice(2, nk + 2), slice(2, nj + 2), slice(2, ni + 2))
    for c in range(3):
        r = torch.rand((nk, nj, ni), generator=g, **f64) * 2.0 - 1.0
        vel[c][inner] += pert * mach * r * env[inner]
        del r
    Q = torch.empty((5,) + shape, **f64)
    Q[0] = rho
    Q[1] = rho * vel[0]
    Q[2] = rho * vel[1]
    Q[3] = rho * vel[2]
    Q[4] = p / (GAMMA - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return dict(name=f"jet{ni}x{nj}x{nk}", ni=ni, nj=nj, nk=nk, bc=(0, 1, 0), xyz=xyz, Q=Q, params=flow_params(),
                p_inf=1.0 / GAMMA, period=(Lx, None, Lz))
