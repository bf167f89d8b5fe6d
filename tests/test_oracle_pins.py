"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage or the mathematical fact it checks.  None of them
re-types an oracle formula: they compare oracle outputs with printed values,
closed forms, invariants, symmetry, convergence order or an independent
brute-force evaluation.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2103_10114_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small_cfg(nx, ny, nz, degree=3, seed=7, hmax=2000.0):
    return dataclasses.replace(synth.CONFIGS["c1"], nx=nx, ny=ny, nz=nz, degree=degree, seed=seed, hmax=hmax)


def rest_state(o, ps_val=1e5):
    st = o.zeros()
    st["ps"][:] = ps_val
    return st


# ----------------------------------------------------------------------------- geometry (P1, P2)
def test_table5_zonal_spacing():
    """Sec. III-B Table V: zonal spacing at the equator and the rows nearest the poles."""
    g = json.load(open(os.path.join(GOLD, "table5_zonal_spacing.json")))
    for row in g["rows"]:
        res = row["res_deg"]
        nx, ny = int(round(360 / res)), int(round(180 / res))
        o = oracle.Oracle(nx, ny, 2)
        d, dv = o.zonal_spacing()
        got = [d[ny // 2] / 1e3, d[1] / 1e3, dv[0] / 1e3]
        want = [row["dx_equator"], row["dx_pole_u"], row["dx_pole_v"]]
        for gv, wv, dig in zip(got, want, row["digits"]):
            if dig < 0:   # printed entry beyond a sin(theta) dlam's digit (see note)
                assert abs(gv - wv) <= 0.01, (res, gv, wv)
            else:
                assert round(gv, dig) == pytest.approx(wv, abs=1e-9), (res, gv, wv)


def test_eq7_leap_counts():
    """Sec. III-B eq. 7: 82/41 at 0.5 deg and 173/87 at 0.25 deg on the two rows nearest the pole."""
    g = json.load(open(os.path.join(GOLD, "eq7_leap_counts.json")))
    for c in g["cases"]:
        o = oracle.Oracle(c["nx"], c["ny"], 2)
        m, mv, r, rv = o.leap_table()
        assert math.ceil(r[1]) == c["row1"]
        assert math.ceil(r[2]) == c["row2"]
        assert math.ceil(r[c["ny"] - 1]) == c["row1"]        # symmetric south
        assert m[1] % 2 == 1 and m[1] >= c["row1"]             # span made odd (Sec. III-B)


def test_leap_table_properties():
    """eq. 7: spans are odd, 1 equatorward of 45 deg (the reference spacing), and M*dx >= dx45."""
    for nx, ny in [(128, 64), (256, 128), (720, 360), (1440, 720)]:
        o = oracle.Oracle(nx, ny, 2)
        m, mv, r, rv = o.leap_table()
        d, dv = o.zonal_spacing()
        dx45 = o.constants()["a"] * math.cos(math.pi / 4) * 2 * math.pi / nx
        th = np.arange(ny + 1) * math.pi / ny
        for j in range(1, ny):
            assert m[j] % 2 == 1
            if abs(math.pi / 2 - th[j]) < math.pi / 4 - 1e-12:
                assert m[j] == 1
            assert m[j] * d[j] >= dx45 * (1 - 1e-6) or m[j] == 1
        assert np.all(mv % 2 == 1)
        assert np.array_equal(m[1:ny], m[1:ny][::-1]) and np.array_equal(mv, mv[::-1])
    # the largest spans at the four grids
    want = {(128, 64): (15, 29), (256, 128): (29, 59), (720, 360): (83, 163), (1440, 720): (163, 325)}
    for (nx, ny), (mu, mvv) in want.items():
        m, mv, _, _ = oracle.Oracle(nx, ny, 2).leap_table()
        assert (m.max(), mv.max()) == (mu, mvv)


def test_substep_rule():
    """3M adaptation calls per step (Sec. III-D): the sub-step count follows the CFL bound."""
    for key, want in [("c1", 2), ("c2", 2), ("c3", 4), ("c4", 4)]:
        c = synth.CONFIGS[key]
        assert oracle.Oracle(c.nx, c.ny, 2).substeps(c.dt) == want


# ----------------------------------------------------------------------------- operator symbols (P4)
def _row_theta(ny, j):
    return j * math.pi / ny


@pytest.mark.parametrize("nx,ny,j,m", [(64, 32, 2, 3), (64, 32, 5, 2), (128, 64, 4, 7), (96, 48, 16, 4)])
def test_delta_minus_symbol(nx, ny, j, m):
    """eq. 6 / Table VII (x,x-1)->(x+N-1,x-N): leaped divergence of a zonal wave of U, closed form."""
    o = oracle.Oracle(nx, ny, 2)
    M = o.leap_table()[0][j]
    c = o.constants()
    st = rest_state(o)
    lam_u = (np.arange(nx) + 0.5) * 2 * math.pi / nx
    st["U"][j, :, :] = np.cos(m * lam_u)
    D = o.column_diag(st)["D"][j, 0]
    lam = np.arange(nx) * 2 * math.pi / nx
    dx = M * c["a"] * math.sin(_row_theta(ny, j)) * 2 * math.pi / nx
    want = -2.0 * math.sin(m * M * math.pi / nx) * np.sin(m * lam) / dx
    np.testing.assert_allclose(D, want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("nx,ny,j,m", [(64, 32, 2, 3), (128, 64, 4, 7), (96, 48, 16, 4)])
def test_delta_plus_symbol(nx, ny, j, m):
    """Table VII (x+1,x)->(x+N,x-N+1): the linearised pressure-gradient of a zonal p_s wave at rest."""
    o = oracle.Oracle(nx, ny, 2)
    M = o.leap_table()[0][j]
    c = o.constants()
    st = rest_state(o)
    d = o.zeros()
    lam = np.arange(nx) * 2 * math.pi / nx
    d["ps"][j, :] = np.cos(m * lam)
    t = o.tl_tendency(st, d, "A")["U"][j, 0]
    dx = M * c["a"] * math.sin(_row_theta(ny, j)) * 2 * math.pi / nx
    lam_u = lam + math.pi / nx
    want = -c["rd"] * c["t0"] / c["p0"] * (-2.0 * np.sin(m * lam_u) * math.sin(m * M * math.pi / nx)) / dx
    np.testing.assert_allclose(t, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("nx,ny,j,m", [(64, 32, 2, 3), (128, 64, 4, 7), (96, 48, 30, 5)])
def test_delta_zero_symbol(nx, ny, j, m):
    """Table VII (x+1,x-1)->(x+2N-1,x-2N+1): advection of a zonal wave of Phi by a uniform u."""
    o = oracle.Oracle(nx, ny, 2)
    M = o.leap_table()[0][j]
    c = o.constants()
    st = rest_state(o)
    u0 = 10.0
    st["U"][1:ny] = u0
    lam = np.arange(nx) * 2 * math.pi / nx
    st["Phi"][j, :, :] = np.cos(m * lam)
    t = o.tendency(st, "L")["Phi"][j, 0]
    dx = M * c["a"] * math.sin(_row_theta(ny, j)) * 2 * math.pi / nx
    want = u0 * np.sin(m * lam) * math.sin(m * M * 2 * math.pi / nx) / dx
    np.testing.assert_allclose(t, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_leap_convergence_order():
    """At a fixed colatitude the span M is fixed, so the leaped zonal derivative converges at order 2."""
    errs = []
    for nx in (128, 256, 512):
        ny = nx // 2
        j = ny // 16                      # colatitude 11.25 deg on every grid
        o = oracle.Oracle(nx, ny, 2)
        c = o.constants()
        st = rest_state(o)
        u0 = 10.0
        st["U"][1:ny] = u0
        lam = np.arange(nx) * 2 * math.pi / nx
        m = 3
        st["Phi"][j, :, :] = np.cos(m * lam)
        t = o.tendency(st, "L")["Phi"][j, 0]
        exact = u0 * m * np.sin(m * lam) / (c["a"] * math.sin(_row_theta(ny, j)))
        errs.append(np.abs(t - exact).max())
        assert o.leap_table()[0][j] > 1
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < r < 2.1 for r in rates), rates


def test_meridional_divergence_convergence():
    """Divergence of a zonally uniform meridional flow converges at order 2 to (1/(a sin)) d(v sin)/dtheta."""
    errs = []
    for ny in (32, 64, 128):
        nx = 2 * ny
        o = oracle.Oracle(nx, ny, 1)
        a = o.constants()["a"]
        st = rest_state(o)
        thv = (np.arange(ny) + 0.5) * math.pi / ny
        st["V"][:, 0, :] = np.sin(2 * thv)[:, None]
        D = o.column_diag(st)["D"][:, 0, 0]
        th = np.arange(ny + 1) * math.pi / ny
        j = np.arange(1, ny)
        exact = (2 * np.cos(2 * th[j]) * np.sin(th[j]) + np.sin(2 * th[j]) * np.cos(th[j])) / (a * np.sin(th[j]))
        errs.append(np.abs(D[j] - exact).max() / np.abs(exact).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(r > 1.8 for r in rates), rates


# ----------------------------------------------------------------------------- column diagnostics
def test_hydrostatic_closed_form():
    """Isothermal deviation: phi'(sigma_k) = -R T' ln(sigma_k) exactly (integral of R T' dln sigma)."""
    o = oracle.Oracle(16, 8, 6)
    st = rest_state(o)
    c = o.constants()
    P = np.sqrt(st["ps"] / c["p0"])
    Tp = 2.5
    st["Phi"][:] = P[:, None, :] * c["rd"] * Tp / c["b"]
    phi = o.column_diag(st)["phi"]
    sig = (np.arange(6) + 0.5) / 6
    want = -c["rd"] * Tp * np.log(sig)
    np.testing.assert_allclose(phi[3, :, 5], want, rtol=1e-14)


STRETCHED = np.array([0.0, 0.02, 0.07, 0.15, 0.3, 0.5, 0.72, 1.0])


def _p2(o, st):
    """P^2 = p_s / p0 at scalar points, each pole value read as the mean of its stored row."""
    ps = st["ps"].copy()
    ps[0] = ps[0].mean()
    ps[-1] = ps[-1].mean()
    return ps / o.constants()["p0"]


def _diag_case(sigma):
    """A seeded atmosphere on a grid whose polar rows leap (M = 3, 5), uniform or stretched levels."""
    nz = 6 if sigma is None else len(STRETCHED) - 1
    cfg = small_cfg(48, 24, nz, degree=6, seed=11)
    st = synth.make_state(cfg)
    sh = None if sigma is None else STRETCHED
    o = oracle.Oracle(48, 24, nz, phis=st["phis"], sigma_half=sh)
    sigh = np.arange(nz + 1) / nz if sh is None else sh
    assert o.leap_table()[0].max() >= 5
    return o, st, sigh


@pytest.mark.parametrize("sigma", [None, "stretched"])
def test_layer_continuity(sigma):
    """Continuity in sigma coordinates (eq. 1, p_s line, with its vertical flux): in every layer of
    every column, D_k + ((P^2 sd)_{k+1} - (P^2 sd)_k) / dsig_k = -T_ps / p0, where sd is the step's own
    sigma-dot and T_ps its own p_s tendency; P^2 sd vanishes at the model top and the surface.
    A flipped sign of sigma-dot or a prefix sum shifted by one level breaks it."""
    o, st, sigh = _diag_case(sigma)
    cd = o.column_diag(st)
    tps = o.tendency(st, "A")["ps"]
    p0 = o.constants()["p0"]
    flux = _p2(o, st)[:, None, :] * cd["sd"]                      # (ny+1, nz+1, nx)
    assert np.all(flux[:, 0] == 0.0) and np.all(flux[:, -1] == 0.0)
    dsig = np.diff(sigh)
    lhs = cd["D"] + np.diff(flux, axis=1) / dsig[None, :, None]
    rhs = np.broadcast_to((-tps / p0)[:, None, :], lhs.shape)
    scale = np.abs(cd["D"]).max()
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(cd["Pi"], -tps / p0, rtol=0, atol=1e-14 * scale)


@pytest.mark.parametrize("sigma", [None, "stretched"])
def test_omega_over_p_definition(sigma):
    """omega = dp/dt with p = sigma p_s (the Omega~ of eq. 1 is P omega/p): at full level k,
    omega/p = (dp_s/dt)/p_s + v.grad(ln p_s) + sd_k / sigma_k, with dp_s/dt the step's own p_s
    tendency and sd_k the mean of the two half-level sigma-dots around the layer."""
    o, st, sigh = _diag_case(sigma)
    cd = o.column_diag(st)
    tps = o.tendency(st, "A")["ps"]
    ps = _p2(o, st) * o.constants()["p0"]
    sig = 0.5 * (sigh[:-1] + sigh[1:])
    sd_full = 0.5 * (cd["sd"][:, :-1] + cd["sd"][:, 1:])
    want = (tps / ps)[:, None, :] + cd["vgl"] + sd_full / sig[None, :, None]
    scale = np.abs(cd["wp"]).max()
    np.testing.assert_allclose(cd["wp"], want, rtol=0, atol=1e-12 * scale)
    # and the omega/p the Phi tendency multiplies: with U = V = 0 the only term left is dp_s/dt = 0
    rest = dict(st)
    rest["U"] = np.zeros_like(st["U"])
    rest["V"] = np.zeros_like(st["V"])
    assert np.all(o.column_diag(rest)["wp"] == 0.0)


def test_v_grad_l_convergence():
    """The horizontal advective part of omega/p converges at order 2 to its continuous value
    u/(a sin) dl/dlam + (v/a) dl/dtheta (colatitude, v toward increasing theta) on rows where the
    span is 1 (|latitude| < 40 deg), for analytic l = ln(p_s/p0), u and v."""
    errs = []
    for nx in (64, 128, 256):
        ny = nx // 2
        o = oracle.Oracle(nx, ny, 1)
        c = o.constants()
        a = c["a"]
        dl, dth = 2 * math.pi / nx, math.pi / ny
        th = np.arange(ny + 1) * dth
        thv = (np.arange(ny) + 0.5) * dth
        lam = np.arange(nx) * dl
        lamu = lam + 0.5 * dl

        def ell(t, lm):
            return 0.03 * np.cos(t) + 0.02 * np.sin(t) ** 2 * np.cos(2 * lm)

        ps = c["p0"] * np.exp(ell(th[:, None], lam[None, :]))
        ps[0] = ps[0].mean()
        ps[-1] = ps[-1].mean()
        P = np.sqrt(ps / c["p0"])
        u = 15 * np.sin(th)[:, None] + 4 * np.sin(th)[:, None] ** 2 * np.sin(lamu)[None, :]
        v = 5 * np.sin(thv)[:, None] * np.cos(lam)[None, :]
        st = o.zeros()
        st["ps"] = ps
        st["U"][:, 0] = 0.5 * (P + np.roll(P, -1, axis=1)) * u
        st["U"][0] = 0.0
        st["U"][-1] = 0.0
        st["V"][:, 0] = 0.5 * (P[:-1] + P[1:]) * v
        vgl = o.column_diag(st)["vgl"][:, 0]
        T, L = th[:, None], lam[None, :]
        us = 15 * np.sin(T) + 4 * np.sin(T) ** 2 * np.sin(L)
        vs = 5 * np.sin(T) * np.cos(L)
        dldl = -0.04 * np.sin(T) ** 2 * np.sin(2 * L)
        dldt = -0.03 * np.sin(T) + 0.04 * np.sin(T) * np.cos(T) * np.cos(2 * L)
        exact = us * dldl / (a * np.sin(T) + (T == 0)) + vs * dldt / a
        rows = np.abs(math.pi / 2 - th) < math.radians(40)
        assert np.all(o.leap_table()[0][rows] == 1)
        errs.append(np.abs(vgl[rows] - exact[rows]).max() / np.abs(exact[rows]).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


@pytest.mark.parametrize("nblocks", [1, 2, 3, 4, 7, 30])
def test_blocked_scan_equals_column_scan(nblocks):
    """Alg. 1 scans a gathered column; Alg. 2 regroups the same sum into local scans, block totals
    and an exclusive scan of the totals.  Applied to the step's own divergences, the blocked scan
    reproduces the prefix sums S_h = sigh_h Pi - P^2 sd_h inside the step for any block split."""
    nz = 30
    cfg = small_cfg(32, 16, nz, degree=5, seed=5)
    st = synth.make_state(cfg)
    o = oracle.Oracle(32, 16, nz, phis=st["phis"])
    cd = o.column_diag(st)
    sigh = np.arange(nz + 1) / nz
    S_step = sigh[None, :, None] * cd["Pi"][:, None, :] - _p2(o, st)[:, None, :] * cd["sd"]
    x = cd["D"] / nz
    beg = [b * nz // nblocks for b in range(nblocks + 1)]
    local = np.zeros((x.shape[0], nz + 1, x.shape[2]))
    tot = []
    for b in range(nblocks):
        acc = np.zeros((x.shape[0], x.shape[2]))
        for k in range(beg[b], beg[b + 1]):
            acc = acc + x[:, k]
            local[:, k + 1] = acc
        tot.append(acc)
    S_blk = np.zeros_like(local)
    run = np.zeros_like(tot[0])
    for b in range(nblocks):
        S_blk[:, beg[b] + 1:beg[b + 1] + 1] = local[:, beg[b] + 1:beg[b + 1] + 1] + run[:, None]
        run = run + tot[b]
    scale = np.abs(x).sum(axis=1).max()
    np.testing.assert_allclose(S_blk, S_step, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(run, cd["Pi"], rtol=0, atol=1e-14 * scale)


def test_mass_closed_form():
    """Uniform p_s: the mass is p_s times the summed cell areas, which for interior rows at
    theta_j = j pi/ny is 2 pi a^2 dth cot(dth/2) (sum_{j=1}^{ny-1} sin(j pi/ny) = cot(pi/(2 ny))),
    plus the two polar caps."""
    for nx, ny in [(64, 32), (128, 64), (90, 45)]:
        o = oracle.Oracle(nx, ny, 3)
        c = o.constants()
        dth = math.pi / ny
        st = rest_state(o, 9.5e4)
        m, _ = o.diagnostics(st)
        area = 2 * math.pi * c["a"] ** 2 * dth / math.tan(dth / 2) + 2 * c["acap"]
        assert m == pytest.approx(9.5e4 * area, rel=1e-12)   # rounding of an nx*ny-term sum
        assert abs(area / (4 * math.pi * c["a"] ** 2) - 1) < dth ** 2   # a sphere, to the quadrature order


def test_energy_closed_form():
    """U = c on every interior row, V = Phi = 0, p_s = p0, flat terrain: the energy measure is
    (p0/2g) c^2 times the summed interior cell areas (the sigma layers add up to 1)."""
    nx, ny, nz = 64, 32, 5
    o = oracle.Oracle(nx, ny, nz)
    cc = o.constants()
    st = rest_state(o, cc["p0"])
    st["U"][1:ny] = 7.0
    _, e = o.diagnostics(st)
    dth = math.pi / ny
    area_int = 2 * math.pi * cc["a"] ** 2 * dth / math.tan(dth / 2)
    assert e == pytest.approx(cc["p0"] / (2 * cc["g"]) * 49.0 * area_int, rel=1e-13)
    # the surface term: q = ln(p_s/p0) uniform gives (R T0 p0 / 2g) q^2 times the whole area
    st2 = rest_state(o, cc["p0"] * math.exp(0.01))
    _, e2 = o.diagnostics(st2)
    area = area_int + 2 * cc["acap"]
    assert e2 == pytest.approx(cc["rd"] * cc["t0"] * cc["p0"] / (2 * cc["g"]) * 1e-4 * area, rel=1e-10)


# ----------------------------------------------------------------------------- invariants (P6-P11)
def test_rest_state_bitwise_zero():
    """eq. 1 at rest: U = V = Phi = 0, p_s = p0, flat terrain give exactly zero tendencies."""
    o = oracle.Oracle(32, 16, 4)
    st = rest_state(o)
    for which in "AL":
        t = o.tendency(st, which)
        for k in t:
            assert np.all(t[k] == 0.0), (which, k)


def test_rest_state_with_terrain():
    """Terrain in hydrostatic balance (p_s = p0 exp(-phis/RT0)) at rest: tendencies vanish to rounding."""
    cfg = small_cfg(32, 16, 4)
    s = synth.make_state(cfg)
    o = oracle.Oracle(32, 16, 4, phis=s["phis"])
    c = o.constants()
    st = rest_state(o)
    st["ps"] = c["p0"] * np.exp(-s["phis"] / (c["rd"] * c["t0"]))
    t = o.tendency(st, "A")
    # scale: the terrain pressure-gradient term that cancels
    scale = c["rd"] * c["t0"] * np.abs(np.diff(s["phis"][5])).max() / (c["rd"] * c["t0"]) / 1e5
    assert np.abs(t["U"]).max() < 1e-11 * max(scale, 1.0)
    assert np.abs(t["V"]).max() < 1e-11 * max(scale, 1.0)
    assert np.abs(t["Phi"]).max() < 1e-20 and np.abs(t["ps"]).max() < 1e-20


def test_mass_conservation_c1():
    """Telescoping flux-form continuity + linear RK: global mass drift <= 1e-13 over C1's 20 steps."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    m0, _ = o.diagnostics(st)
    s = o.step(st, cfg.steps, cfg.dt)
    m1, _ = o.diagnostics(s)
    assert abs(m1 - m0) / m0 <= 1e-13
    for k in s:
        assert np.all(np.isfinite(s[k]))


def test_mass_tendency_sums_to_zero():
    """The area-weighted p_s tendency (incl. the polar caps) telescopes to zero."""
    cfg = small_cfg(64, 32, 5, degree=6)
    st = synth.make_state(cfg)
    o = oracle.Oracle(64, 32, 5, phis=st["phis"])
    t = o.tendency(st, "A")
    c = o.constants()
    th = np.arange(33) * math.pi / 32
    w = c["a"] ** 2 * np.sin(th) * (math.pi / 32) * (2 * math.pi / 64)
    tot = (w[1:32, None] * t["ps"][1:32]).sum() + c["acap"] * (t["ps"][0, 0] + t["ps"][32, 0])
    scale = (w[1:32, None] * np.abs(t["ps"][1:32])).sum()
    assert abs(tot) < 1e-14 * scale


def test_advection_skew_symmetry():
    """IAP skew form: sum w dsig F L(F) = 0 for F = U, V, Phi and any winds (energy property)."""
    cfg = small_cfg(64, 32, 6, degree=8)
    st = synth.make_state(cfg)
    o = oracle.Oracle(64, 32, 6, phis=st["phis"])
    c = o.constants()
    t = o.tendency(st, "L")
    ny = 32
    th = np.arange(ny + 1) * math.pi / ny
    thv = (np.arange(ny) + 0.5) * math.pi / ny
    w = c["a"] ** 2 * np.sin(th) * (math.pi / ny) * (2 * math.pi / 64)
    wv = c["a"] ** 2 * np.sin(thv) * (math.pi / ny) * (2 * math.pi / 64)
    ds = 1.0 / 6
    for key, wt, rows in [("U", w, slice(1, ny)), ("V", wv, slice(0, ny)), ("Phi", w, slice(1, ny))]:
        prod = wt[rows, None, None] * ds * st[key][rows] * t[key][rows]
        tot = prod.sum()
        scale = np.abs(prod).sum()
        if key == "Phi":
            for p in (0, ny):
                tot += c["acap"] * ds * (st["Phi"][p, :, 0] * t["Phi"][p, :, 0]).sum()
        assert abs(tot) < 1e-13 * scale, (key, tot, scale)


def test_periodicity():
    """Rolling every input by s columns rolls every tendency by s columns."""
    cfg = small_cfg(48, 24, 4, degree=6)
    st = synth.make_state(cfg)
    s = 7
    rolled = {k: np.roll(v, s, axis=-1) for k, v in st.items()}
    o1 = oracle.Oracle(48, 24, 4, phis=st["phis"])
    o2 = oracle.Oracle(48, 24, 4, phis=rolled["phis"])
    for which in "AL":
        t1 = o1.tendency(st, which)
        t2 = o2.tendency(rolled, which)
        for k in t1:
            want = np.roll(t1[k], s, axis=-1)
            np.testing.assert_allclose(t2[k], want, rtol=0, atol=1e-12 * np.abs(want).max())
            if k in ("U", "V"):   # rows away from the poles see no pole mean: bitwise
                assert np.array_equal(t2[k][3:-3], want[3:-3])


def test_equatorial_mirror():
    """j -> ny - j with V -> -V (southward positive) mirrors the tendencies (f flips with cos theta)."""
    cfg = small_cfg(32, 16, 4, degree=6)
    st = synth.make_state(cfg)
    mir = {"U": st["U"][::-1].copy(), "V": -st["V"][::-1].copy(), "Phi": st["Phi"][::-1].copy(),
           "ps": st["ps"][::-1].copy(), "phis": st["phis"][::-1].copy()}
    o1 = oracle.Oracle(32, 16, 4, phis=st["phis"])
    o2 = oracle.Oracle(32, 16, 4, phis=mir["phis"])
    for which in "AL":
        t1 = o1.tendency(st, which)
        t2 = o2.tendency(mir, which)
        for k, sgn in [("U", 1), ("V", -1), ("Phi", 1), ("ps", 1)]:
            want = sgn * t1[k][::-1]
            np.testing.assert_allclose(t2[k], want, rtol=0, atol=1e-12 * max(np.abs(want).max(), 1e-30))


def test_solid_body_balance_order2():
    """Solid-body wind u = u0 sin(theta) with the gradient-wind p_s: zonal terms vanish exactly and the
    meridional imbalance of the V tendency is O(dtheta^2)."""
    res = []
    for ny in (32, 64, 128):
        nx = 2 * ny
        o = oracle.Oracle(nx, ny, 2)
        c = o.constants()
        u0 = 20.0
        th = np.arange(ny + 1) * math.pi / ny
        lb = (c["a"] * c["omega"] * u0 + 0.5 * u0 ** 2) * np.sin(th) ** 2 / (c["rd"] * c["t0"])
        st = o.zeros()
        st["ps"][:] = c["p0"] * np.exp(lb)[:, None]
        P = np.sqrt(st["ps"] / c["p0"])
        PU = 0.5 * (P + np.roll(P, -1, axis=1))
        st["U"][1:ny] = (PU[1:ny] * u0 * np.sin(th[1:ny])[:, None])[:, None, :]
        t = o.tendency(st, "A")
        assert np.all(t["U"] == 0.0)
        tl = o.tendency(st, "L")
        assert np.abs(tl["U"]).max() == 0.0 and np.abs(tl["V"]).max() == 0.0
        scale = 2 * c["omega"] * u0
        res.append(np.abs(t["V"]).max() / scale)
    rates = [math.log2(res[i] / res[i + 1]) for i in range(2)]
    assert all(r > 1.8 for r in rates), (res, rates)


# ----------------------------------------------------------------------------- adjoint (P14)
def _tiny():
    cfg = small_cfg(16, 8, 3)
    st = synth.make_state(cfg)
    return cfg, st, oracle.Oracle(16, 8, 3, phis=st["phis"])


@pytest.mark.parametrize("which", ["A", "L"])
def test_adjoint_dot_tendency(which):
    """<J x, y> = <x, J^T y>: hand-written adjoint against the complex-step tangent-linear."""
    cfg, st, o = _tiny()
    x = synth.random_like(st, 11)
    y = synth.random_like(st, 12)
    a = oracle.dot(o.tl_tendency(st, x, which), y)
    b = oracle.dot(x, o.adj_tendency(st, y, which))
    assert abs(a - b) <= 1e-13 * abs(a)


def test_adjoint_dot_step_c1_grid():
    """Dot test of the whole step (3M adaptation + 3 advection stages) on the C1 grid."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"])
    x = synth.random_like(st, 1031)
    y = synth.random_like(st, 1032)
    a = oracle.dot(o.tl_step(st, x, cfg.dt), y)
    b = oracle.dot(x, o.adj_step(st, y, cfg.dt))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_adjoint_full_jacobian_tiny():
    """Brute force on a tiny grid: every TL column of the tendency Jacobian equals the adjoint row."""
    cfg = small_cfg(16, 8, 2)
    st = synth.make_state(cfg)
    o = oracle.Oracle(16, 8, 2, phis=st["phis"])
    keys = ["U", "V", "Phi", "ps"]
    shapes = {k: st[k].shape for k in keys}
    sizes = [int(np.prod(shapes[k])) for k in keys]
    n = sum(sizes)
    rng = np.random.default_rng(5)
    cols = rng.choice(n, 60, replace=False)

    def unit(idx):
        d = {k: np.zeros(shapes[k]) for k in keys}
        off = 0
        for k, sz in zip(keys, sizes):
            if idx < off + sz:
                d[k].reshape(-1)[idx - off] = 1.0
                return d
            off += sz

    def flat(d):
        return np.concatenate([d[k].reshape(-1) for k in keys])

    for which in "AL":
        for c in cols:
            col = flat(o.tl_tendency(st, unit(c), which))
            for r in rng.choice(n, 8, replace=False):
                row = flat(o.adj_tendency(st, unit(r), which))
                assert abs(col[r] - row[c]) <= 1e-12 * max(abs(col[r]), 1e-300) + 1e-300


def test_adjoint_central_fd():
    """Central finite differences of the step (eps = 1e-6 relative) against J^T at sampled points."""
    cfg = small_cfg(32, 16, 4, degree=5)
    st = synth.make_state(cfg)
    o = oracle.Oracle(32, 16, 4, phis=st["phis"])
    dt = 600.0
    rng = np.random.default_rng(1033)
    for trial in range(4):
        key = ["U", "V", "Phi", "ps"][trial]
        shp = st[key].shape
        idx = tuple(rng.integers(1 if (key == "U" and d == 0) else 0, s - (1 if (key == "U" and d == 0) else 0))
                    for d, s in enumerate(shp))
        if key == "ps" and idx[0] in (0, shp[0] - 1):
            idx = (idx[0] + (1 if idx[0] == 0 else -1),) + idx[1:]
        okey = ["Phi", "U", "ps", "V"][trial]
        oshp = st[okey].shape
        oidx = tuple(rng.integers(1, s - 1) if d == 0 else rng.integers(0, s) for d, s in enumerate(oshp))
        y = {k: np.zeros_like(v) for k, v in st.items() if k != "phis"}
        y[okey][oidx] = 1.0
        g = o.adj_step(st, y, dt)[key][idx]
        rms = np.sqrt(np.mean(st[key] ** 2))
        eps = 1e-6 * rms
        sp = {k: v.copy() for k, v in st.items() if k != "phis"}
        sm = {k: v.copy() for k, v in st.items() if k != "phis"}
        sp[key][idx] += eps
        sm[key][idx] -= eps
        fd = (o.step(sp, 1, dt)[okey][oidx] - o.step(sm, 1, dt)[okey][oidx]) / (2 * eps)
        assert abs(fd - g) <= 1e-6 * max(abs(g), abs(fd)) + 1e-10 * abs(o.adj_step(st, y, dt)[key]).max(), \
            (key, okey, fd, g)


# ----------------------------------------------------------------------------- brute force (P15)
@pytest.mark.parametrize("nx,ny,nz", [(16, 8, 3), (32, 16, 4)])
@pytest.mark.parametrize("which", ["A", "L"])
def test_numpy_brute_force(nx, ny, nz, which):
    """An independent vectorised NumPy evaluation of both tendencies equals the C++ oracle."""
    from tests import brute_numpy as bn
    cfg = small_cfg(nx, ny, nz, degree=4, seed=nx + nz)
    st = synth.make_state(cfg)
    o = oracle.Oracle(nx, ny, nz, phis=st["phis"])
    m, mv, _, _ = o.leap_table()
    g = bn.geometry(nx, ny, nz)
    assert np.array_equal(g["M"][1:ny], m[1:ny]) and np.array_equal(g["Mv"], mv)
    assert m.max() > 1 and mv.max() > 1            # the leap is active on this grid
    t = o.tendency(st, which)
    f = bn.tend_A if which == "A" else bn.tend_L
    b = f(g, st, st["phis"])
    for k in ("U", "V", "Phi", "ps"):
        scale = max(np.abs(t[k]).max(), 1e-300)
        np.testing.assert_allclose(b[k], t[k], rtol=0, atol=1e-12 * scale, err_msg=f"{which} {k}")


# ----------------------------------------------------------------------------- low-latitude filters
def _lat(ny, j, vrow=False):
    """Latitude in degrees of scalar/U row j or V row j (colatitude j dth or (j + 1/2) dth)."""
    return 90.0 - (j + (0.5 if vrow else 0.0)) * 180.0 / ny


def _filter_case(nx=64, ny=32, nz=2):
    o = oracle.Oracle(nx, ny, nz)
    lam = np.arange(nx) * 2 * math.pi / nx
    alt = (-1.0) ** np.arange(nx)
    st = o.zeros()
    # every row: a constant, a smooth wave and the 2-dlam wave
    row = 3.0 + 0.7 * np.cos(3 * lam) + 0.25 * alt
    st["U"][1:ny] = row
    st["V"][:] = row
    st["Phi"][1:ny] = row
    st["ps"][1:ny] = 1e5 + 10.0 * row
    return o, st, lam, alt


def test_filter_bands_and_simplified_filter():
    """Sec. III-B, Table IV: rows equatorward of 38 deg lose exactly their 2-dlam wave (the simplified
    filter) and keep every other zonal wave; rows poleward of 70 deg and the pole rows are untouched."""
    nx, ny = 64, 32
    o, st, lam, alt = _filter_case(nx, ny)
    out = o.filter(st)
    smooth = 3.0 + 0.7 * np.cos(3 * lam)
    for key, rows, vrow in (("U", range(1, ny), False), ("V", range(ny), True), ("Phi", range(1, ny), False)):
        for j in rows:
            lat = abs(_lat(ny, j, vrow))
            for k in range(2):
                got = out[key][j, k]
                if lat < 38:
                    np.testing.assert_allclose(got, smooth, rtol=0, atol=1e-14)
                elif lat > 70:
                    assert np.array_equal(got, st[key][j, k])
    for j in range(1, ny):
        if abs(_lat(ny, j)) < 38:
            np.testing.assert_allclose(out["ps"][j], 1e5 + 10 * smooth, rtol=0, atol=1e-9)
    for key in ("Phi", "ps", "U"):
        assert np.array_equal(out[key][0], st[key][0]) and np.array_equal(out[key][-1], st[key][-1])


def test_filter_three_point_operator():
    """Sec. III-B, Table IV: between 38 and 70 deg the filter is a symmetric 3-point operator
    F + r (F_{x-1} - 2 F + F_{x+1}) (checked by its impulse response), which keeps constants and the
    row sum, and which scales the 2-dlam wave by the ratio of the row's zonal spacing to the spacing at
    38 deg, cos(lat) / cos(38 deg); every other wave m is then scaled by 1 - 4 r sin^2(m dlam / 2)."""
    nx, ny = 64, 32
    o = oracle.Oracle(nx, ny, 1)
    lam = np.arange(nx) * 2 * math.pi / nx
    seen = 0
    for j in range(1, ny):
        lat = abs(_lat(ny, j))
        if not (38 <= lat <= 70):
            continue
        seen += 1
        st = o.zeros()
        st["Phi"][j, 0, 5] = 1.0                       # impulse
        st["Phi"][j, 0, 40] = 1.0
        imp = o.filter(st)["Phi"][j, 0]
        r = imp[4]
        assert imp[6] == r and imp[39] == r and imp[41] == r and abs(imp[5] - (1 - 2 * r)) < 1e-15
        assert np.count_nonzero(imp) == 6
        assert abs(imp.sum() - 2.0) < 1e-14
        st = o.zeros()
        st["Phi"][j, 0] = (-1.0) ** np.arange(nx)
        fac = o.filter(st)["Phi"][j, 0] / st["Phi"][j, 0]
        want = math.cos(math.radians(lat)) / math.cos(math.radians(38.0))
        np.testing.assert_allclose(fac, want, rtol=0, atol=1e-14)
        st["Phi"][j, 0] = 2.0 + np.cos(5 * lam)
        got = o.filter(st)["Phi"][j, 0]
        want5 = 2.0 + (1 - (1 - want) * math.sin(5 * math.pi / nx) ** 2) * np.cos(5 * lam)
        np.testing.assert_allclose(got, want5, rtol=0, atol=1e-14)
    assert seen >= 8


def test_filters_conserve_mass_c1():
    """Both filters keep each row's zonal sum, so the flux-form mass stays conserved: <= 1e-13 over
    C1's 20 steps with the filters applied after every step (and they do act: the state differs)."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], filters=True)
    m0, _ = o.diagnostics(st)
    s = o.step(st, cfg.steps, cfg.dt)
    m1, _ = o.diagnostics(s)
    assert abs(m1 - m0) / m0 <= 1e-13
    plain = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).step(st, 1, cfg.dt)
    filt = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], filters=True).step(st, 1, cfg.dt)
    assert np.abs(plain["V"] - filt["V"]).max() > 1e-6


def test_filters_adjoint_dot():
    """With the filters on, the hand-written adjoint of the step passes the dot test against the
    complex-step tangent-linear (each row filter is symmetric, so its transpose is itself)."""
    cfg = small_cfg(32, 16, 3, degree=4)
    st = synth.make_state(cfg)
    o = oracle.Oracle(32, 16, 3, phis=st["phis"], filters=True)
    x = synth.random_like(st, 81)
    y = synth.random_like(st, 82)
    jx = o.tl_step(st, x, cfg.dt)
    jty = o.adj_step(st, y, cfg.dt)
    lhs, rhs = oracle.dot(jx, y), oracle.dot(x, jty)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ----------------------------------------------------------------------------- p_s diffusion (kappa*)
def _rest_ps(o, ps):
    st = o.zeros()
    st["ps"] = np.array(ps, dtype=np.float64)
    return st


def test_ps_diffusion_zonal_symbol():
    """eq. 1's kappa* D_sa at rest (no winds, flat terrain, so -p0 Pi = 0): on a row whose span is M,
    a zonal p_s wave cos(m lam) gives kappa* (-4 sin^2(m M dlam / 2) / (M dx)^2) cos(m lam) from the
    leaped second difference, plus the meridional part of a zonally uniform row pattern (zero here)."""
    nx, ny = 96, 48
    o = oracle.Oracle(nx, ny, 2, kstar=3e5)
    c = o.constants()
    M = o.leap_table()[0]
    lam = np.arange(nx) * 2 * math.pi / nx
    for j, m in [(2, 3), (5, 4), (24, 7)]:
        ps = np.full((ny + 1, nx), 1e5)
        ps[j] += 50.0 * np.cos(m * lam)
        t = o.tendency(_rest_ps(o, ps), "A")["ps"][j]
        dx = M[j] * c["a"] * math.sin(j * math.pi / ny) * 2 * math.pi / nx
        zon = -4 * math.sin(m * M[j] * math.pi / nx) ** 2 / dx ** 2 * 50.0 * np.cos(m * lam)
        dy2 = c["a"] ** 2 * math.sin(j * math.pi / ny) * (math.pi / ny) ** 2
        sv = [math.sin((jj + 0.5) * math.pi / ny) for jj in (j - 1, j)]
        mer = -(sv[0] + sv[1]) / dy2 * 50.0 * np.cos(m * lam)   # the neighbours rows hold the mean
        np.testing.assert_allclose(t, 3e5 * (zon + mer), rtol=0, atol=1e-12 * np.abs(3e5 * (zon + mer)).max())


def test_ps_diffusion_converges_to_laplacian():
    """The flux-form D_sa converges at order 2 to the spherical Laplacian: for p_s = p0 (1 + e Y) with
    Y = sin(theta) cos(theta) cos(lam) = x z / r^2 (a degree-2 spherical harmonic, Laplacian -6/a^2 Y) on rows
    within 60 degrees of the equator (the leap span of each row is fixed as the grid refines)."""
    errs = []
    for ny in (48, 96, 192):
        nx = 2 * ny
        o = oracle.Oracle(nx, ny, 1, kstar=1.0)
        a = o.constants()["a"]
        th = np.arange(ny + 1) * math.pi / ny
        lam = np.arange(nx) * 2 * math.pi / nx
        Y = (np.sin(th) * np.cos(th))[:, None] * np.cos(lam)[None, :]
        ps = 1e5 * (1 + 1e-3 * Y)
        t = o.tendency(_rest_ps(o, ps), "A")["ps"]
        exact = -6.0 / a ** 2 * 1e5 * 1e-3 * Y
        rows = np.abs(90 - np.degrees(th)) <= 60
        errs.append(np.abs(t[rows] - exact[rows]).max() / np.abs(exact[rows]).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


def test_ps_diffusion_conserves_mass():
    """The flux form telescopes: the area-weighted sum of kappa* D_sa over the sphere (caps included)
    vanishes, and the global mass stays conserved over C1's steps with kappa* = 2e5 m^2/s (which
    changes the state)."""
    cfg = synth.CONFIGS["c1"]
    st = synth.make_state(cfg)
    o = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], kstar=2e5)
    rest = dict(st)
    rest["U"] = np.zeros_like(st["U"])
    rest["V"] = np.zeros_like(st["V"])
    t = o.tendency(rest, "A")["ps"]
    c = o.constants()
    ny, nx = cfg.ny, cfg.nx
    th = np.arange(ny + 1) * math.pi / ny
    w = c["a"] ** 2 * np.sin(th) * (math.pi / ny) * (2 * math.pi / nx)
    tot = (w[1:ny, None] * t[1:ny]).sum() + c["acap"] * (t[0, 0] + t[ny, 0])
    scale = (w[1:ny, None] * np.abs(t[1:ny])).sum()
    assert abs(tot) < 1e-13 * scale and scale > 0
    m0, _ = o.diagnostics(st)
    s = o.step(st, 10, cfg.dt)
    m1, _ = o.diagnostics(s)
    assert abs(m1 - m0) / m0 <= 1e-13
    s0 = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"]).step(st, 1, cfg.dt)
    s1 = oracle.Oracle(cfg.nx, cfg.ny, cfg.nz, phis=st["phis"], kstar=2e5).step(st, 1, cfg.dt)
    assert np.abs(s0["ps"] - s1["ps"]).max() > 1e-3


def test_ps_diffusion_adjoint_dot():
    """With kappa* on, the hand-written adjoint (tendency and whole step) passes the dot test against
    the complex-step tangent-linear."""
    cfg = small_cfg(32, 16, 3, degree=4)
    st = synth.make_state(cfg)
    o = oracle.Oracle(32, 16, 3, phis=st["phis"], kstar=2e5)
    x = synth.random_like(st, 83)
    y = synth.random_like(st, 84)
    for which in "AL":
        jx = o.tl_tendency(st, x, which)
        jty = o.adj_tendency(st, y, which)
        lhs, rhs = oracle.dot(jx, y), oracle.dot(x, jty)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs), which
    jx = o.tl_step(st, x, cfg.dt)
    jty = o.adj_step(st, y, cfg.dt)
    lhs, rhs = oracle.dot(jx, y), oracle.dot(x, jty)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
