"""Pins of the oracle's grid coupling (section 2.4): leaf location, the
block-boundary value rule, trilinear space+time interpolation, and the
derived fields Eqs. 2-4 need (section 2.1) against closed forms."""
import math

import numpy as np
import pytest

import fte_workloads as W

DEG = W.DEG
AU = W.AU


def small_amr(n_levels=3, xi_map=0, periodic=True, seed=0, n_snap=1):
    n1, bx = (16, 8, 16), (4, 4, 4)
    rng = np.random.default_rng(seed)
    marks = {}

    def refine(L, I, J, K):
        key = (L, I, J, K)
        if key not in marks:
            marks[key] = rng.random() < (0.35 if L == 1 else 0.3)
        return marks[key]

    leaves = W.amr_leaves(n1, bx, n_levels, refine, phi_periodic=periodic)
    if xi_map == 0:
        dxi = 1.9 * AU / n1[0]
    else:
        dxi = math.log(20.0) / n1[0]
    dph = (2 * math.pi if periodic else 200 * DEG) / n1[2]
    return W.grid_desc(xi_map, 0.1 * AU, dxi, 30 * DEG, 120 * DEG / n1[1], 0.0 if periodic else 10 * DEG, dph,
                       n1, bx, leaves, n_levels, n_snap=n_snap, t_s0=0.0, dt_s=3600.0, phi_periodic=periodic)


def xi_of(g, r):
    return np.log(r / g["r_lo"]) if g["xi_map"] == 1 else r - g["r_lo"]


def test_amr_leaves_tile_and_balance():
    g = small_amr()
    leaves = g["leaves"]
    n1, bx = g["n1"], g["bx"]
    L = g["n_levels"]
    fine = [n1[a] << (L - 1) for a in range(3)]
    owner = -np.ones(fine, dtype=np.int64)
    for i, (lev, I, J, K) in enumerate(leaves):
        s = 1 << (L - lev)
        sl = tuple(slice(B * bx[a] * s, (B + 1) * bx[a] * s) for a, B in enumerate((I, J, K)))
        assert np.all(owner[sl] == -1)
        owner[sl] = i
    assert np.all(owner >= 0)
    lev_of = leaves[owner, 0]
    # face and diagonal neighbours differ by at most one level
    for ax in range(3):
        for sh in (1, -1):
            nb = np.roll(lev_of, sh, axis=ax)
            d = np.abs(nb - lev_of)
            if ax < 2:  # no wrap along xi and theta
                idx = [slice(None)] * 3
                idx[ax] = slice(0, 1) if sh == 1 else slice(-1, None)
                d[tuple(idx)] = 0
            assert d.max() <= 1
    assert len(np.unique(leaves[:, 0])) == L


def test_find_leaf_brute_force(orc):
    g = small_amr()
    raw = np.zeros((1, len(g["leaves"]), 64, 6))
    G = orc.Grid(g, raw)
    rng = np.random.default_rng(3)
    n1 = np.array(g["n1"], float)
    pts = rng.random((3000, 3)) * n1
    # points on block and cell faces (half-open cells go to the upper side)
    pts[:200] = np.floor(pts[:200] * 4) / 4
    for p in pts:
        leaf, lev, cell = G.find_leaf(p)
        found = []
        for i, (L, I, J, K) in enumerate(g["leaves"]):
            s = 2.0 ** (L - 1)
            ok = all(B * g["bx"][a] <= p[a] * s < (B + 1) * g["bx"][a] for a, B in enumerate((I, J, K)))
            if ok:
                found.append(i)
        assert found == [leaf]
        assert lev == g["leaves"][leaf][0]
        assert np.array_equal(cell, np.floor(p * 2.0 ** (lev - 1)).astype(np.int64))


@pytest.mark.parametrize("xi_map,periodic", [(0, False), (1, False), (1, True)])
def test_block_boundary_rule_exact_for_affine(orc, xi_map, periodic):
    """Virtual values at level-L centres (same-level copy, mean of finer
    children, trilinear from coarser centres) reproduce any field affine in
    (xi, theta, phi) wherever the centre lies inside the domain."""
    g = small_amr(xi_map=xi_map, periodic=periodic, seed=5)
    rng = np.random.default_rng(11)
    coef = rng.normal(size=(6, 5))
    if periodic:
        coef[:, 3] = 0.0       # affine in phi is not periodic
    coef[:, 4] = 0.0
    coef[:, 1] /= g["dxi"]     # O(1) change per cell
    r, th, ph = W.cell_centres(g)
    raw = W.affine_fields(xi_of(g, r), th, ph, 0.0, coef)[None]
    G = orc.Grid(g, raw)
    checked = 0
    for lev, I, J, K in g["leaves"]:
        for L in sorted({max(1, lev - 1), lev, min(g["n_levels"], lev + 1)}):
            s = 2.0 ** (L - lev)
            # a ring of cells around the block at level L
            for _ in range(12):
                c = np.array([rng.integers(int(B * g["bx"][a] * s) - 1, int((B + 1) * g["bx"][a] * s) + 1)
                              for a, B in enumerate((int(I), int(J), int(K)))])
                n = np.array([g["n1"][a] << (L - 1) for a in range(3)])
                # centres whose coarser stencil stays inside the domain (beyond
                # the edges the rule holds values constant, not affine)
                m = 2 if periodic else 3
                p1 = (c + 0.5) * 2.0 ** (1 - L)
                inside = np.all((p1[:m] >= 1.0) & (p1[:m] <= np.array(g["n1"][:m]) - 1.0))
                if not inside:
                    continue
                h = 2.0 ** (1 - L)
                xi = (c[0] + 0.5) * g["dxi"] * h
                tt = g["th_lo"] + (c[1] + 0.5) * g["dth"] * h
                cp = c[2] % n[2] if periodic else c[2]
                pp = g["ph_lo"] + (cp + 0.5) * g["dph"] * h
                want = coef[:, 0] + coef[:, 1] * xi + coef[:, 2] * tt + coef[:, 3] * pp
                got = G.raw_virtual(0, L, c)
                assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(coef).sum()), (L, c)
                checked += 1
    assert checked > 200


def _sph_basis(th, ph):
    st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
    return np.array([[st * cp, st * sp, ct], [ct * cp, ct * sp, -st], [-sp, cp, 0.0]])


@pytest.mark.parametrize("xi_map", [0, 1])
def test_interpolation_exact_for_affine_space_time(orc, xi_map):
    """Trilinear space interpolation and linear time weighting reproduce a
    wind whose spherical V components are affine in (xi, theta, phi, t)."""
    g = small_amr(xi_map=xi_map, periodic=False, seed=2, n_snap=3)
    rng = np.random.default_rng(4)
    coef = rng.normal(size=(6, 5))
    coef[:, 4] *= 1e-3
    coef[3:, :] = 0.0
    coef[3, 0] = 1.0           # B radial and uniform
    coef[:, 1] /= g["dxi"]
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.affine_fields(xi_of(g, r), th, ph, k * 3600.0, coef) for k in range(3)])
    G = orc.Grid(g, raw)
    p = dict(mass=W.M_P, lambda_ref=AU, dt=1.0, bg_kind="grid")
    n1 = np.array(g["n1"], float)
    for _ in range(300):
        s = 1.0 + rng.random(3) * (n1 - 2.0)
        xi = s[0] * g["dxi"]
        rr = g["r_lo"] * math.exp(xi) if xi_map == 1 else g["r_lo"] + xi
        tt = g["th_lo"] + s[1] * g["dth"]
        pp = g["ph_lo"] + s[2] * g["dph"]
        t = rng.random() * 2 * 3600.0
        x = rr * np.array([math.sin(tt) * math.cos(pp), math.sin(tt) * math.sin(pp), math.cos(tt)])
        st, out = orc.fields(p, G, x, t)
        assert st == 0
        V_sph = _sph_basis(tt, pp) @ out[0:3]
        want = coef[:3, 0] + coef[:3, 1] * xi + coef[:3, 2] * tt + coef[:3, 3] * pp + coef[:3, 4] * t
        assert np.allclose(V_sph, want, rtol=1e-9, atol=1e-9 * np.abs(coef[:3]).sum())


def test_zero_gradient_beyond_edges_and_phi_wrap(orc):
    cfg = W.tiny_parker()
    g = cfg["grid"]
    G = orc.Grid(g, W.make_raw(g, cfg["wind"]))
    p = dict(mass=W.M_P, lambda_ref=AU, dt=1.0, bg_kind="grid")
    # below the first radial centre the fields are those of the first centre
    st1, a = orc.fields(p, G, np.array([0.06 * AU, 0.0, 0.0]) @ np.eye(3), 0.0)
    st2, b = orc.fields(p, G, np.array([0.1 * AU + 0.49 * g["dxi"], 0.0, 0.0]), 0.0)
    assert st1 == 0 and st2 == 0
    assert np.allclose(a, b, rtol=1e-12)
    # phi just below 2 pi and just above 0 interpolate across the seam
    eps = 1e-9
    x1 = AU * np.array([math.cos(-eps), math.sin(-eps), 0.0])
    x2 = AU * np.array([math.cos(eps), math.sin(eps), 0.0])
    _, f1 = orc.fields(p, G, x1, 0.0)
    _, f2 = orc.fields(p, G, x2, 0.0)
    assert np.allclose(f1[0:3], f2[0:3], rtol=0, atol=1e-2)          # V, m/s
    assert np.allclose(f1[3:6], f2[3:6], rtol=0, atol=1e-8)          # b
    for k, sc in ((6, 1e-5), (7, 1e-6), (8, 1e-11), (9, 1e-12)):
        assert abs(f1[k] - f2[k]) < 1e-6 * sc


# ---------------------------------------------------------------------------
# derived fields against an independent Cartesian finite-difference evaluation
# of the analytic wind (Richardson-extrapolated, error ~ h^4)
# ---------------------------------------------------------------------------
def _cart_vb(wind, x, t, kw):
    r = np.linalg.norm(x)
    th = math.acos(x[2] / r)
    ph = math.atan2(x[1], x[0]) % (2 * math.pi)
    f = np.asarray(wind(np.array([r]), np.array([th]), np.array([ph]), t, **kw))[0]
    E = _sph_basis(th, ph)
    V = E.T @ f[:3]
    B = E.T @ f[3:]
    return V, B / np.linalg.norm(B)


def _analytic_derived(wind, x, t, kw, h=2e6, ht=20.0):
    def grad(fun):
        G = np.zeros((3, 3))
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1.0
            d1 = (fun(x + h * e) - fun(x - h * e)) / (2 * h)
            d2 = (fun(x + 0.5 * h * e) - fun(x - 0.5 * h * e)) / h
            G[:, d] = (4 * d2 - d1) / 3
        return G
    GV = grad(lambda y: _cart_vb(wind, y, t, kw)[0])
    Gb = grad(lambda y: _cart_vb(wind, y, t, kw)[1])
    V, b = _cart_vb(wind, x, t, kw)
    dVdt = (_cart_vb(wind, x, t + ht, kw)[0] - _cart_vb(wind, x, t - ht, kw)[0]) / (2 * ht)
    return dict(divV=np.trace(GV), bbgV=b @ GV @ b, divb=np.trace(Gb), bDV=b @ (dVdt + GV @ V),
                curv=Gb @ b, V=V, b=b)


def test_parker_closed_forms(orc):
    """Independent FD evaluation agrees with the Parker closed forms
    (div V = 2V/r, bb:grad V = V sin^2 psi / r, div b = cos psi (2/r - a^2 r/(1+a^2 r^2)))."""
    x = AU * np.array([math.cos(0.3), math.sin(0.3), 0.1])
    d = _analytic_derived(W.parker_wind, x, 0.0, {})
    r = np.linalg.norm(x)
    th = math.acos(x[2] / r)
    V0 = 400e3
    a = W.OMEGA_SYNODIC * math.sin(th) / V0
    psi = math.atan(a * r)
    assert d["divV"] == pytest.approx(2 * V0 / r, rel=1e-7)
    assert d["bbgV"] == pytest.approx(V0 * math.sin(psi) ** 2 / r, rel=1e-6)
    assert d["divb"] == pytest.approx(math.cos(psi) * (2 / r - a * a * r / (1 + a * a * r * r)), rel=1e-6)
    assert abs(d["bDV"]) < 1e-9 * V0 * V0 / r


def _derived_errors(orc, g, wind, kw, snap, cells):
    raw = W.make_raw(g, wind, **kw) if False else None
    r, th, ph = W.cell_centres(g)
    raw = np.stack([wind(r, th, ph, g["t_s0"] + k * g["dt_s"], **kw) for k in range(g["n_snap"])])
    G = orc.Grid(g, raw)
    errs = {k: [] for k in ("divV", "bbgV", "divb", "bDV", "curv")}
    for (L, c) in cells:
        out = G.derived_virtual(snap, L, np.array(c))
        h = 2.0 ** (1 - L)
        xi = (c[0] + 0.5) * g["dxi"] * h
        rr = g["r_lo"] * math.exp(xi) if g["xi_map"] == 1 else g["r_lo"] + xi
        tt = g["th_lo"] + (c[1] + 0.5) * g["dth"] * h
        pp = g["ph_lo"] + (c[2] + 0.5) * g["dph"] * h
        x = rr * np.array([math.sin(tt) * math.cos(pp), math.sin(tt) * math.sin(pp), math.cos(tt)])
        d = _analytic_derived(wind, x, g["t_s0"] + snap * g["dt_s"], kw)
        E = _sph_basis(tt, pp)
        curv = E.T @ out[10:13]
        scale_v = abs(d["divV"]) + 1e-30
        errs["divV"].append(abs(out[6] - d["divV"]) / scale_v)
        errs["bbgV"].append(abs(out[7] - d["bbgV"]) / scale_v)
        errs["divb"].append(abs(out[8] - d["divb"]) / (abs(d["divb"]) + np.linalg.norm(d["curv"])))
        errs["bDV"].append(abs(out[9] - d["bDV"]) / (scale_v * 400e3))
        errs["curv"].append(np.linalg.norm(curv - d["curv"]) / (np.linalg.norm(d["curv"]) + abs(d["divb"])))
    return {k: max(v) for k, v in errs.items()}


def test_parker_derived_second_order(orc):
    """Derived fields of the steady Parker wind converge at second order to the
    independent evaluation (error ratio ~4 per halving of the cell size)."""
    res = []
    for n in (32, 64):
        n1, bx = (n, n // 2, n), (8, 8, 8)
        g = W.grid_desc(0, 0.1 * AU, 1.9 * AU / n, 30 * DEG, 120 * DEG / (n // 2), 0.0, 2 * math.pi / n, n1, bx,
                        W.uniform_leaves(n1, bx), 1)
        # interior cells whose centres sit near 1 au, mid latitudes
        cells = []
        for fr in (0.35, 0.5, 0.62):
            for ft in (0.4, 0.55):
                for fp in (0.1, 0.6):
                    c = (int(fr * n), int(ft * n // 2), int(fp * n))
                    cells.append((1, c))
        res.append(_derived_errors(orc, g, W.parker_wind, {}, 0, cells))
    for k in ("divV", "bbgV", "divb", "curv"):
        assert res[1][k] < 0.5 * res[0][k] or res[1][k] < 1e-6, (k, res)
        assert res[1][k] < 0.02, (k, res)


def test_cir_derived_time_dependent(orc):
    """On the stretched, time-dependent CIR grid the derived fields (including
    b . dV/dt with its explicit time derivative across snapshots) approach the
    independent evaluation as the grid is refined."""
    res = []
    for f in (1, 2):
        n1, bx = (24 * f, 6 * f, 48 * f), (4, 2 * f, 4)
        dxi = math.log(1.6) / n1[0]
        g = W.grid_desc(1, 0.5 * AU, dxi, 80 * DEG, 20 * DEG / n1[1], 0.0, 2 * math.pi / n1[2], n1, bx,
                        W.uniform_leaves(n1, bx), 1, n_snap=3, t_s0=0.0, dt_s=1800.0 / f)
        cells = []
        for fr in (0.4, 0.7):
            for fp in np.linspace(0.05, 0.95, 7):
                cells.append((1, (int(fr * n1[0]), n1[1] // 2, int(fp * n1[2]))))
        res.append(_derived_errors(orc, g, W.cir_wind, dict(width=40 * DEG, width_rare=80 * DEG), 1, cells))
    for k in ("divV", "bbgV", "divb", "bDV"):
        assert res[1][k] < 0.5 * res[0][k] or res[1][k] < 1e-4, (k, res)
