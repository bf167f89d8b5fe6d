"""Independent vectorised NumPy evaluation of both tendencies (test helper).

Written from the difference equations, with whole-array shifts instead of
loops, so that an index or sign slip in either this file or the C++ oracle
shows up as a mismatch.  Small grids only.
"""
import math

import numpy as np


def _shift(a, s):
    """b[..., i] = a[..., i + s] (periodic in longitude)."""
    return np.roll(a, -s, axis=-1)


def geometry(nx, ny, nz):
    c = dict(a=6.371e6, omega=7.292e-5, rd=287.04, cp=1004.64, p0=1e5, t0=300.0)
    c["kappa"] = c["rd"] / c["cp"]
    c["b"] = math.sqrt(c["kappa"] * c["rd"] * c["t0"])
    dl, dt = 2 * math.pi / nx, math.pi / ny
    th = np.arange(ny + 1) * dt
    thv = (np.arange(ny) + 0.5) * dt

    def span(s):
        r = math.asin(math.sin(math.pi / 4) * math.sin(dl)) / math.asin(s * math.sin(dl))
        m = max(1, math.ceil(r - 1e-9))
        m += (m % 2 == 0)
        cap = (nx - 1) // 2
        cap -= (cap % 2 == 0)
        return min(m, cap)

    M = np.ones(ny + 1, dtype=int)
    for j in range(1, ny):
        M[j] = span(math.sin(th[j]))
    Mv = np.array([span(math.sin(t)) for t in thv])
    sigh = np.arange(nz + 1) / nz
    sig = 0.5 * (sigh[1:] + sigh[:-1])
    c.update(nx=nx, ny=ny, nz=nz, dl=dl, dt=dt, th=th, thv=thv, s=np.sin(th), sv=np.sin(thv),
             M=M, Mv=Mv, sigh=sigh, sig=sig, dsig=np.diff(sigh),
             acap=2 * math.pi * c["a"] ** 2 * (1 - math.cos(dt / 2)))
    return c


def _poles(a):
    a = a.copy()
    a[0] = a[0].mean(axis=-1, keepdims=True)
    a[-1] = a[-1].mean(axis=-1, keepdims=True)
    return a


def _zonal(F, M, mode, dxrow):
    """Leaped zonal difference on every row of F (rows first axis, lon last).

    mode '+': scalar -> U point i+1/2: F[i+n] - F[i+1-n]
    mode '-': U -> scalar point i:     F[i+n-1] - F[i-n]
    divided by M * dx_row."""
    out = np.zeros_like(F)
    for j in range(F.shape[0]):
        m = int(M[j])
        n = (m + 1) // 2
        if dxrow[j] == 0:
            continue
        if mode == "+":
            out[j] = (_shift(F[j], n) - _shift(F[j], 1 - n)) / (m * dxrow[j])
        else:
            out[j] = (_shift(F[j], n - 1) - _shift(F[j], -n)) / (m * dxrow[j])
    return out


def diagnose(g, st, phis):
    nx, ny, nz, a = g["nx"], g["ny"], g["nz"], g["a"]
    ps = _poles(st["ps"])
    F = _poles(st["Phi"])
    U = st["U"].copy()
    U[0] = 0
    U[-1] = 0
    V = st["V"]
    P = np.sqrt(ps / g["p0"])
    l = np.log(ps / g["p0"])
    q = l + _poles(phis) / (g["rd"] * g["t0"])
    RT = g["b"] * F / P[:, None, :]
    cl = np.log(g["sigh"][2:] / g["sigh"][1:-1])          # levels 1..nz-1
    cpk = np.log(g["sigh"][1:] / g["sig"])
    phi = cpk[None, :, None] * RT
    for k in range(nz):
        phi[:, k] += (cl[k:, None] * RT[:, k + 1:]).sum(axis=1) if k + 1 < nz else 0.0
    PU = 0.5 * (P + _shift(P, 1))
    PU[0] = 1
    PU[-1] = 1
    PV = 0.5 * (P[:-1] + P[1:])
    u = U / PU[:, None, :]
    u[0] = 0
    u[-1] = 0
    v = V / PV[:, None, :]
    MU = PU[:, None, :] * U
    MV = PV[:, None, :] * V
    dxrow = a * g["s"] * g["dl"]
    D = _zonal(MU, g["M"], "-", dxrow)
    svMV = g["sv"][:, None, None] * MV
    D[1:-1] += (svMV[1:] - svMV[:-1]) / (a * g["s"][1:-1, None, None] * g["dt"])
    D[0] = (a * g["dl"] * g["sv"][0] * MV[0].sum(axis=-1) / g["acap"])[:, None]
    D[-1] = (-a * g["dl"] * g["sv"][-1] * MV[-1].sum(axis=-1) / g["acap"])[:, None]
    S = np.zeros((ny + 1, nz + 1, nx))
    S[:, 1:] = np.cumsum(D * g["dsig"][None, :, None], axis=1)
    Pi = S[:, -1]
    sd = (g["sigh"][None, :, None] * Pi[:, None, :] - S) / (P ** 2)[:, None, :]
    sd[:, 0] = 0
    sd[:, -1] = 0
    dlp = _zonal(l[:, None, :], g["M"], "+", dxrow)[:, 0, :]      # at U points
    vgl = 0.5 * (u * dlp[:, None, :] + _shift(u * dlp[:, None, :], -1))
    gy = (l[1:] - l[:-1]) / (a * g["dt"])                          # at V rows
    vg = v * gy[:, None, :]
    vgl[1:-1] += 0.5 * (vg[1:] + vg[:-1])
    vgl[0] = vg[0].mean(axis=-1)[:, None]
    vgl[-1] = vg[-1].mean(axis=-1)[:, None]
    wp = vgl - (S[:, :-1] + 0.5 * D * g["dsig"][None, :, None]) / (g["sig"][None, :, None] * (P ** 2)[:, None, :])
    return dict(ps=ps, F=F, U=U, V=V, P=P, l=l, q=q, RT=RT, phi=phi, PU=PU, PV=PV, u=u, v=v,
                D=D, S=S, Pi=Pi, sd=sd, wp=wp, dxrow=dxrow)


def tend_A(g, st, phis):
    d = diagnose(g, st, phis)
    a, ny = g["a"], g["ny"]
    RT0 = g["rd"] * g["t0"]
    out = {}
    out["Phi"] = (g["b"] * d["P"][:, None, :] + g["kappa"] * d["F"]) * d["wp"]
    out["ps"] = -g["p0"] * d["Pi"]
    pg = (_zonal(d["phi"], g["M"], "+", d["dxrow"])
          + RT0 * _zonal(d["q"][:, None, :], g["M"], "+", d["dxrow"])
          + 0.5 * (d["RT"] + _shift(d["RT"], 1)) * _zonal(d["l"][:, None, :], g["M"], "+", d["dxrow"]))
    V = d["V"]
    Vx = 0.5 * (V + _shift(V, 1))                     # V averaged to i+1/2 on V rows
    VV = np.zeros_like(d["U"])
    VV[1:-1] = 0.5 * (Vx[1:] + Vx[:-1])
    cot = np.zeros(ny + 1)
    cot[1:-1] = np.cos(g["th"][1:-1]) / g["s"][1:-1]
    f = 2 * g["omega"] * np.cos(g["th"])
    fs = f[:, None, None] + d["u"] * cot[:, None, None] / a
    TU = -d["PU"][:, None, :] * pg - fs * VV
    TU[0] = 0
    TU[-1] = 0
    out["U"] = TU
    RTy = 0.5 * (d["RT"][1:] + d["RT"][:-1])
    pgy = ((d["phi"][1:] - d["phi"][:-1]) + RT0 * (d["q"][1:] - d["q"][:-1])[:, None, :]
           + RTy * (d["l"][1:] - d["l"][:-1])[:, None, :]) / (a * g["dt"])
    Ux = 0.5 * (d["U"] + _shift(d["U"], -1))           # U averaged to integer i
    ux = 0.5 * (d["u"] + _shift(d["u"], -1))
    UU = 0.5 * (Ux[1:] + Ux[:-1])
    uu = 0.5 * (ux[1:] + ux[:-1])
    fsv = 2 * g["omega"] * np.cos(g["thv"])[:, None, None] + uu * (np.cos(g["thv"]) / g["sv"])[:, None, None] / a
    out["V"] = -d["PV"][:, None, :] * pgy + fsv * UU
    return out


def _adv_zonal(vel, F, M, dxrow, vel_off_plus, vel_off_minus):
    out = np.zeros_like(F)
    for j in range(F.shape[0]):
        m = int(M[j])
        n = (m + 1) // 2
        if dxrow[j] == 0:
            continue
        op, om = vel_off_plus(n), vel_off_minus(n)
        out[j] = (_shift(vel[j], op) * _shift(F[j], m) - _shift(vel[j], om) * _shift(F[j], -m)) / (2 * m * dxrow[j])
    return out


def _vert(sdx, F, dsig):
    out = np.zeros_like(F)
    out += sdx[:, 1:] * np.concatenate([F[:, 1:], np.zeros_like(F[:, :1])], axis=1)
    out -= sdx[:, :-1] * np.concatenate([np.zeros_like(F[:, :1]), F[:, :-1]], axis=1)
    return out / (2 * dsig[None, :, None])


def tend_L(g, st, phis):
    d = diagnose(g, st, phis)
    a, ny = g["a"], g["ny"]
    vt = d["v"] * g["sv"][:, None, None]
    out = {"ps": np.zeros_like(st["ps"])}
    # Phi
    F = d["F"]
    L1 = _adv_zonal(d["u"], F, g["M"], d["dxrow"], lambda n: n - 1, lambda n: -n)
    L2 = np.zeros_like(F)
    L2[1:-1] = (vt[1:] * F[2:] - vt[:-1] * F[:-2]) / (2 * a * g["s"][1:-1, None, None] * g["dt"])
    cc = a * g["dl"] / (2 * g["acap"])
    L2[0] = (cc * (vt[0] * F[1]).sum(axis=-1))[:, None]
    L2[-1] = (-cc * (vt[-1] * F[-2]).sum(axis=-1))[:, None]
    L1[0] = 0
    L1[-1] = 0
    out["Phi"] = -(L1 + L2 + _vert(d["sd"], F, g["dsig"]))
    # U
    U = d["U"]
    ub = 0.5 * (_shift(d["u"], -1) + d["u"])                  # at integer p: (u[p-1]+u[p])/2
    L1 = _adv_zonal(ub, U, g["M"], d["dxrow"], lambda n: n, lambda n: 1 - n)
    vtu = 0.5 * (vt + _shift(vt, 1))
    L2 = np.zeros_like(U)
    L2[1:-1] = (vtu[1:] * U[2:] - vtu[:-1] * U[:-2]) / (2 * a * g["s"][1:-1, None, None] * g["dt"])
    sdu = 0.5 * (d["sd"] + _shift(d["sd"], 1))
    TU = -(L1 + L2 + _vert(sdu, U, g["dsig"]))
    TU[0] = 0
    TU[-1] = 0
    out["U"] = TU
    # V
    V = d["V"]
    uv = 0.5 * (d["u"][:-1] + d["u"][1:])
    L1 = _adv_zonal(uv, V, g["Mv"], a * g["sv"] * g["dl"], lambda n: n - 1, lambda n: -n)
    vts = np.zeros_like(F)
    vts[1:-1] = 0.5 * (vt[:-1] + vt[1:])
    Vn = np.concatenate([V[1:], np.zeros_like(V[:1])], axis=0)
    Vs = np.concatenate([np.zeros_like(V[:1]), V[:-1]], axis=0)
    L2 = (vts[1:] * Vn - vts[:-1] * Vs) / (2 * a * g["sv"][:, None, None] * g["dt"])
    sdv = 0.5 * (d["sd"][:-1] + d["sd"][1:])
    out["V"] = -(L1 + L2 + _vert(sdv, V, g["dsig"]))
    return out
