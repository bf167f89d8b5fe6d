"""Seeded synthetic atmospheres for the leap-format dynamical core.

This module only builds input states.  It holds none of the step's arithmetic:
it draws terrain, winds, surface pressure and temperature deviations from
seeded spherical-harmonic and white-noise recipes and expresses them in the
IAP variables (U = P u, V = P v, Phi = P R T' / b with P = sqrt(p_s / p0)) on
the Arakawa C grid of Sec. III-B (U at (i+1/2, j), V at (i, j+1/2), scalars at
(i, j), rows j = 0..ny at colatitude j*pi/ny including both poles).

Both the GPU runs and the CPU oracle read the same arrays from here.

Recipe (per config): terrain from degree <= 8 harmonics with N(0,1)(n+1)^-2
coefficients scaled to [0, h_max]; winds u = u0 sin(theta) plus the rotational
wind of a per-level random streamfunction of degree <= L scaled to peak A;
p_s balanced with the solid-body wind, reduced by the terrain, times (1 +/- 1%)
uniform noise; T' ~ N(0, (0.01 T0)^2) iid.  Pole rows hold one value each.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import gammaln, lpmv

A_EARTH = 6.371e6
OMEGA = 7.292e-5
G = 9.80616
RD = 287.04
CP = 1004.64
P0 = 1.0e5
T0 = 300.0
KAPPA = RD / CP
B = math.sqrt(KAPPA * RD * T0)


@dataclasses.dataclass(frozen=True)
class GridConfig:
    name: str
    nx: int
    ny: int
    nz: int
    dt: float
    steps: int
    degree: int      # streamfunction degree L
    amp: float       # wind perturbation peak A (m/s)
    hmax: float      # terrain height max (m)
    seed: int
    u0: float = 20.0
    wind_noise: float = 0.0   # iid N(0, wind_noise^2) m/s added to u, v (ensemble members)


CONFIGS = {
    "c1": GridConfig("c1", 128, 64, 9, 600.0, 20, 10, 2.0, 2000.0, 101),
    "c2": GridConfig("c2", 256, 128, 30, 300.0, 100, 20, 5.0, 4000.0, 102),
    "c3": GridConfig("c3", 720, 360, 30, 240.0, 1, 20, 5.0, 4000.0, 103),
    "c4": GridConfig("c4", 1440, 720, 30, 120.0, 48, 40, 8.0, 6000.0, 104),
}


def ensemble_member(m: int) -> GridConfig:
    """Member m (0..23) of the mixed-resolution ensemble: 8 each of C1, C2, C3 grids."""
    base = [CONFIGS["c1"], CONFIGS["c2"], CONFIGS["c3"]][m // 8]
    return dataclasses.replace(base, name=f"e{m}", seed=500 + m, steps=50, wind_noise=0.5)


def _norm_legendre(n: int, m: int, x: np.ndarray) -> np.ndarray:
    """Associated Legendre function with the (n-m)!/(n+m)! normalisation."""
    f = math.exp(0.5 * (gammaln(n - m + 1) - gammaln(n + m + 1))) * math.sqrt(2 * n + 1)
    return f * lpmv(m, n, x)


def _harmonic_field(coef_c, coef_s, theta, lam, lmax, dtheta=False, dlam=False):
    """Sum_{n<=lmax, m<=n} N P_n^m(cos theta) (c cos m lam + s sin m lam) on theta x lam.

    coef_c/coef_s have shape (lmax+1, lmax+1, K); returns (K, len(theta), len(lam)).
    dtheta/dlam give the theta or lambda derivative instead.
    """
    x = np.cos(theta)
    st = np.sin(theta)
    K = coef_c.shape[2]
    ms = np.arange(lmax + 1)
    Acos = np.zeros((K, theta.size, lmax + 1))
    Asin = np.zeros((K, theta.size, lmax + 1))
    for n in range(1, lmax + 1):
        for m in range(0, n + 1):
            if dtheta:
                # (1 - x^2) dP/dx = (n + m) P_{n-1}^m - n x P_n^m and d/dtheta = -sin(theta) d/dx
                fn = math.exp(0.5 * (gammaln(n - m + 1) - gammaln(n + m + 1))) * math.sqrt(2 * n + 1)
                raw_n = lpmv(m, n, x)
                raw_m1 = lpmv(m, n - 1, x) if m <= n - 1 else 0.0
                val = -fn * ((n + m) * raw_m1 - n * x * raw_n) / st
            else:
                val = _norm_legendre(n, m, x)
            Acos[:, :, m] += val[None, :] * coef_c[n, m][:, None]
            Asin[:, :, m] += val[None, :] * coef_s[n, m][:, None]
    cosm = np.cos(np.outer(ms, lam))
    sinm = np.sin(np.outer(ms, lam))
    if dlam:
        # d/dlam (c cos + s sin) = m (-c sin + s cos)
        return (Asin * ms) @ cosm - (Acos * ms) @ sinm
    return Acos @ cosm + Asin @ sinm


def _coefs(rng, lmax, K, decay_pow=None):
    c = rng.standard_normal((lmax + 1, lmax + 1, K))
    s = rng.standard_normal((lmax + 1, lmax + 1, K))
    for n in range(lmax + 1):
        c[n, n + 1:] = 0.0
        s[n, n + 1:] = 0.0
        s[n, 0] = 0.0
        if decay_pow is not None:
            c[n] *= (n + 1.0) ** (-decay_pow)
            s[n] *= (n + 1.0) ** (-decay_pow)
    c[0] = 0.0
    s[0] = 0.0
    return c, s


def make_state(cfg: GridConfig):
    """Return dict with float64 arrays U (ny+1,nz,nx), V (ny,nz,nx), Phi (ny+1,nz,nx),
    ps (ny+1,nx), phis (ny+1,nx)."""
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    dlam = 2.0 * math.pi / nx
    dth = math.pi / ny
    lam_s = np.arange(nx) * dlam                 # scalar / V columns
    lam_u = (np.arange(nx) + 0.5) * dlam         # U columns
    th_s = np.arange(ny + 1) * dth               # scalar / U rows (poles included)
    th_v = (np.arange(ny) + 0.5) * dth           # V rows

    # terrain, degree <= 8, c ~ N(0,1) (n+1)^-2, scaled to [0, hmax]
    tc, ts = _coefs(rng, 8, 1, decay_pow=2.0)
    sfield = _harmonic_field(tc, ts, th_s, lam_s, 8)[0]
    sfield[0, :] = sfield[0, 0]
    sfield[ny, :] = sfield[ny, 0]
    h = cfg.hmax * (sfield - sfield.min()) / (sfield.max() - sfield.min())
    phis = G * h

    # winds: per-level streamfunction of degree <= L, rotational wind scaled to peak amp
    wc, ws = _coefs(rng, cfg.degree, nz)
    th_u = th_s[1:ny]
    up = _harmonic_field(wc, ws, th_u, lam_u, cfg.degree, dtheta=True) / A_EARTH
    vp = -_harmonic_field(wc, ws, th_v, lam_s, cfg.degree, dlam=True) / (A_EARTH * np.sin(th_v)[None, :, None])
    peak = max(np.abs(up).max(), np.abs(vp).max())
    up *= cfg.amp / peak
    vp *= cfg.amp / peak
    u = np.zeros((ny + 1, nz, nx))
    u[1:ny] = np.transpose(up, (1, 0, 2)) + cfg.u0 * np.sin(th_u)[:, None, None]
    v = np.transpose(vp, (1, 0, 2)).copy()
    if cfg.wind_noise > 0:
        u[1:ny] += cfg.wind_noise * rng.standard_normal(u[1:ny].shape)
        v += cfg.wind_noise * rng.standard_normal(v.shape)

    # surface pressure: solid-body balance, terrain reduction, 1% uniform noise
    lbal = (A_EARTH * OMEGA * cfg.u0 + 0.5 * cfg.u0 ** 2) * np.sin(th_s) ** 2 / (RD * T0)
    wrow = np.sin(th_s)
    lbal = lbal - (lbal * wrow).sum() / wrow.sum()
    xi = rng.uniform(-1.0, 1.0, (ny + 1, nx))
    xi[0, :] = xi[0, 0]
    xi[ny, :] = xi[ny, 0]
    ps = P0 * np.exp(lbal)[:, None] * np.exp(-phis / (RD * T0)) * (1.0 + 0.01 * xi)

    # temperature deviation T' ~ N(0, (0.01 T0)^2), one value per pole and level
    tp = 0.01 * T0 * rng.standard_normal((ny + 1, nz, nx))
    tp[0, :, :] = tp[0, :, :1]
    tp[ny, :, :] = tp[ny, :, :1]

    P = np.sqrt(ps / P0)
    Phi = P[:, None, :] * RD * tp / B
    PU = 0.5 * (P + np.roll(P, -1, axis=1))
    PV = 0.5 * (P[:-1] + P[1:])
    U = PU[:, None, :] * u
    U[0] = 0.0
    U[ny] = 0.0
    V = PV[:, None, :] * v
    return {"U": np.ascontiguousarray(U), "V": np.ascontiguousarray(V),
            "Phi": np.ascontiguousarray(Phi), "ps": np.ascontiguousarray(ps),
            "phis": np.ascontiguousarray(phis)}


def random_like(state: dict, seed: int) -> dict:
    """Unit-variance Gaussian fields of the state's shapes (pole rows replicated, U pole rows 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for k in ("U", "V", "Phi", "ps"):
        a = rng.standard_normal(state[k].shape)
        out[k] = a
    out["U"][0] = 0.0
    out["U"][-1] = 0.0
    return out
