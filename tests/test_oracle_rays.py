"""Pins for the oracle's ray tracer and ray-to-grid tables (CPU only).

Each test checks the oracle against something other than itself: closed
forms for straight rays and for rays in linear slowness / linear velocity
media, invariants of the ray equations, dynamic ray tracing for the
spreading, reciprocity, and a brute-force rasterisation of a tiny fan.
"""
import math

import numpy as np
import pytest

import workload as W
from oracle import rays


def _homog(nrays=360, alpha=5.0):
    g = W.centred_grid(96, 0.5e-3, 16, 20e-3, 1500.0)
    c = np.full((g.ny, g.nx), 1500.0)
    al = np.full_like(c, alpha)
    to = W.resolve_trace_opts(g, c, nrays)
    return g, c, al, to


def test_homogeneous_travel_time_amplitude_absorption():
    """Straight rays: T = r/c0 up to the wavefront sag r dpsi^2 / (8 c0);
    a = sqrt(c0 / (8 pi r)) (J = r exactly for chords on a circle, Eq. 7);
    B = alpha0 r (Eq. 5, absorption integrated along the ray)."""
    g, c, al, to = _homog()
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / c, al)
    X, Y = g.pixel_centres()
    pos = g.element_positions()
    dpsi = math.pi / to.n_rays
    dr = 1500.0 * to.dtau
    for e in (0, 3, 11):
        r = np.hypot(X - pos[e, 0], Y - pos[e, 1]).ravel()
        cov = np.isfinite(T[e])
        assert cov.mean() > 0.5
        sag = r * dpsi ** 2 / 8.0
        bound = (r + 2.0 * dr) * dpsi ** 2 / (8.0 * 1500.0) + 1e-16
        assert np.all(np.abs(T[e][cov] - r[cov] / 1500.0) <= bound[cov])
        far = cov & (r > 5e-3)
        aref = np.sqrt(1500.0 / (8.0 * math.pi * r[far]))
        # linear interpolation of r^(-1/2) across a step dr: (3/32)(dr/r)^2
        rel_bound = (3.0 / 32.0) * (dr / r[far]) ** 2 * 1.2 + 2.0 * sag[far] / r[far] + 1e-12
        assert np.all(np.abs(A[e][far] / aref - 1.0) <= rel_bound)
        assert np.all(np.abs(B[e][cov] - 5.0 * r[cov]) <= 5.0 * 1.1 * (r[cov] + 2 * dr) * dpsi ** 2 / 8 + 1e-15)
        # uncovered pixels are NaN with zero a and B
        assert np.all(A[e][~cov] == 0.0) and np.all(B[e][~cov] == 0.0)


def test_homogeneous_receiver_tables():
    g, c, al, to = _homog(alpha=0.0)
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / c, None)
    pos = g.element_positions()
    d = np.hypot(pos[:, None, 0] - pos[None, :, 0], pos[:, None, 1] - pos[None, :, 1])
    dpsi = math.pi / to.n_rays
    from oracle.invert import receiver_mask
    msk = receiver_mask(g.m, 0.75)
    assert np.all(np.isfinite(Tr[msk]))
    assert np.all(np.abs(Tr - d / 1500.0)[msk] <= (d[msk] + 1e-3) * dpsi ** 2 / (8 * 1500.0) + 1e-16)
    assert np.all(Tr[np.arange(g.m), np.arange(g.m)] == 0.0)   # the source point itself


def test_linear_slowness_closed_form_rays():
    """s = s0 + g y is reproduced exactly by bilinear interpolation, so the
    traced nodes must sit on the analytic rays: with p = px (conserved),
    x - x_e = (p/g)[ln(s + sqrt(s^2 - p^2))] and
    T = (1/g)[s sqrt(s^2-p^2)/2 + p^2 ln(s + sqrt(s^2-p^2))/2] between s_e and s."""
    g = W.centred_grid(121, 0.5e-3, 8, 25e-3, 1500.0)
    X, Y = g.pixel_centres()
    s0 = 1.0 / 1500.0
    gs = 0.02 * s0 / 0.03
    S = s0 + gs * Y
    to = W.resolve_trace_opts(g, 1.0 / S, 64)
    e = 6   # the bottom element: its whole fan goes towards +y
    fan = rays.trace_fan(g, to, S, None, e)
    xe, ye = g.element_positions()[e]
    se = s0 + gs * ye
    F = lambda s, p: np.log(s + np.sqrt(s * s - p * p))
    Gf = lambda s, p: 0.5 * s * np.sqrt(s * s - p * p) + 0.5 * p * p * F(s, p)
    for j in range(to.n_rays):
        L = fan["L"][j]
        assert L > 10
        x, y = fan["x"][:L + 1, j], fan["y"][:L + 1, j]
        p = fan["px"][0, j]
        assert np.all(fan["px"][:L + 1, j] == p)           # dp_x/dtau = ds/dx / s = 0
        ap = abs(p)
        sy = s0 + gs * y
        xex = xe + np.sign(p) * (ap / gs) * (F(sy, ap) - F(se, ap))
        tex = (Gf(sy, ap) - Gf(se, ap)) / gs
        assert np.max(np.abs(x - xex)) < 1e-12
        assert np.max(np.abs(fan["tau"][:L + 1] - tex)) < 1e-15


def test_linear_velocity_travel_time():
    """c = c0 + g y: circular-arc rays with
    T = (1/g) arccosh(1 + g^2 r^2 / (2 c(x_e) c(x)))."""
    g = W.centred_grid(200, 0.25e-3, 8, 22e-3, 1500.0)
    X, Y = g.pixel_centres()
    gg = 800.0
    cl = 1500.0 + gg * Y
    to = W.resolve_trace_opts(g, cl, 1440)
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / cl, None, 0, 8)
    pos = g.element_positions()
    for e in range(8):
        xe, ye = pos[e]
        ce = 1500.0 + gg * ye
        Tex = np.arccosh(1.0 + gg * gg * ((X - xe) ** 2 + (Y - ye) ** 2) / (2.0 * ce * cl)) / gg
        Te = T[e].reshape(X.shape)
        cov = np.isfinite(Te) & (np.hypot(X, Y) < 20e-3)
        assert cov.mean() > 0.45
        assert np.max(np.abs(Te - Tex)[cov]) < 1e-10


def test_linear_velocity_spreading_matches_dynamic_ray_tracing():
    """With c_nn = 0 dynamic ray tracing gives J = (1/c_e) int c^2 dtau for a
    point source; the oracle's J = c / (8 pi a^2) comes from neighbour rays."""
    g = W.centred_grid(200, 0.25e-3, 8, 22e-3, 1500.0)
    X, Y = g.pixel_centres()
    gg = 800.0
    cl = 1500.0 + gg * Y
    to = W.resolve_trace_opts(g, cl, 1440)
    e = 6
    fan = rays.trace_fan(g, to, 1.0 / cl, None, e)
    ce = 1.0 / rays.bilinear(g, 1.0 / cl, 1.0 / 1500.0, fan["x"][0:1, 0], fan["y"][0:1, 0])[0][0]
    for j in (100, 400, 720, 1000, 1300):
        L = fan["L"][j]
        x, y = fan["x"][:L + 1, j], fan["y"][:L + 1, j]
        cn = 1.0 / rays.bilinear(g, 1.0 / cl, 1.0 / 1500.0, x, y)[0]
        c2 = cn * cn
        integral = np.concatenate([[0.0], np.cumsum(0.5 * (c2[1:] + c2[:-1]) * to.dtau)])
        Jdyn = integral / ce
        Jray = cn / (8.0 * math.pi * fan["amp"][:L + 1, j] ** 2)
        far = Jdyn > 2e-3
        assert np.max(np.abs(Jray[far] / Jdyn[far] - 1.0)) < 2e-5


def test_eikonal_invariant_fourth_order():
    """|p| c(x) = 1 is conserved by the ray equations (Eq. 6).  A field
    s = s0 (1 + a x + b y + d x y) is reproduced exactly by the bilinear
    interpolant (no gradient kinks), so classic RK4 must conserve it to
    O(dtau^4): halving dtau shrinks the drift about 16 times."""
    g = W.centred_grid(121, 0.5e-3, 8, 25e-3, 1500.0)
    X, Y = g.pixel_centres()
    L, s0 = 0.03, 1.0 / 1500.0
    sfun = lambda x, y: s0 * (1.0 + 0.02 * x / L + 0.015 * y / L + 0.3 * x * y / L ** 2)
    S = sfun(X, Y)
    to = W.resolve_trace_opts(g, 1.0 / S, 90)
    drift = []
    for fac in (1.0, 0.5):
        t2 = W.TraceOpts(90, to.dtau * fac, to.tau_max, to.j_min)
        mx = 0.0
        for e in range(8):
            fan = rays.trace_fan(g, t2, S, None, e)
            for j in range(0, 90, 7):
                n = fan["L"][j]
                x, y = fan["x"][:n + 1, j], fan["y"][:n + 1, j]
                pn = np.hypot(fan["px"][:n + 1, j], fan["py"][:n + 1, j])
                mx = max(mx, float(np.max(np.abs(pn / sfun(x, y) - 1.0))))
        drift.append(mx)
    assert drift[0] < 2e-12
    assert drift[0] / drift[1] > 8.0


def test_reciprocity_smooth_heterogeneous():
    """T_e(x_r) = T_r(x_e), B_e(x_r) = B_r(x_e) and, from the symmetry of the
    paraxial Q2, c(x_r)/J_e(x_r) = c(x_e)/J_r(x_e), i.e. a_e(x_r) = a_r(x_e).
    In a smooth weak medium the only errors are discretisation ones; the
    amplitude bound reflects RK4's first-order direction error where rays
    cross the gradient kinks of the bilinear field."""
    g = W.centred_grid(128, 0.5e-3, 32, 28e-3, 1500.0)
    X, Y = g.pixel_centres()
    bump = np.exp(-((X - 4e-3) ** 2 + (Y - 2e-3) ** 2) / (2 * (8e-3) ** 2))
    c = 1500.0 + 10.0 * bump - 6.0 * np.exp(-((X + 6e-3) ** 2 + (Y + 5e-3) ** 2) / (2 * (7e-3) ** 2))
    al = 3.0 * bump
    to = W.resolve_trace_opts(g, c, 360)
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / c, al)
    from oracle.invert import receiver_mask
    msk = receiver_mask(g.m, 0.75)
    assert np.all(np.isfinite(Tr[msk]))
    assert np.max(np.abs(Tr - Tr.T)[msk]) < 2e-9
    assert np.max(np.abs(Br - Br.T)[msk]) < 2e-5
    assert np.max(np.abs(Ar / Ar.T - 1.0)[msk]) < 1e-2


def test_bilinear_interpolation_properties():
    """Exact at pixel centres, exact for linear fields, background outside."""
    g = W.centred_grid(10, 1e-3, 4, 3e-3, 1500.0)
    X, Y = g.pixel_centres()
    rng = np.random.default_rng(3)
    f = rng.uniform(1, 2, X.shape)
    v, gx, gy = rays.bilinear(g, f, 7.0, X.ravel(), Y.ravel())
    assert np.array_equal(v, f.ravel())
    lin = 2.0 + 3.0 * X - 5.0 * Y
    xq = rng.uniform(X.min(), X.max() - 1e-9, 200)
    yq = rng.uniform(Y.min(), Y.max() - 1e-9, 200)
    v, gx, gy = rays.bilinear(g, lin, 7.0, xq, yq)
    assert np.allclose(v, 2.0 + 3.0 * xq - 5.0 * yq, rtol=0, atol=1e-13)
    assert np.allclose(gx, 3.0, atol=1e-9) and np.allclose(gy, -5.0, atol=1e-9)
    v, gx, gy = rays.bilinear(g, f, 7.0, np.array([1.0, -0.2]), np.array([0.0, 0.3]))
    assert np.all(v == 7.0) and np.all(gx == 0.0) and np.all(gy == 0.0)


def _mesh_triangles(fan, nr):
    """Every triangle of the wavefront mesh whose cell has both rays alive at
    its later step, as node indices (n, j) of its three vertices, in the
    order of the triangle index 2 (n nr + j) + t: t = 0 is (P[n][j],
    P[n][j+1], P[n+1][j+1]), t = 1 is (P[n][j], P[n+1][j+1], P[n+1][j])."""
    L = fan["L"]
    nmax = fan["x"].shape[0] - 1
    n, j = np.meshgrid(np.arange(nmax), np.arange(nr - 1), indexing="ij")
    n, j = n.ravel(), j.ravel()
    live = (n + 1 <= L[j]) & (n + 1 <= L[j + 1])
    n, j = n[live], j[live]
    vn = np.stack([np.stack([n, n, n + 1], 1), np.stack([n, n + 1, n + 1], 1)], 1)   # [cell][t][vertex]
    vj = np.stack([np.stack([j, j + 1, j + 1], 1), np.stack([j, j + 1, j], 1)], 1)
    idx = np.stack([2 * (n * nr + j), 2 * (n * nr + j) + 1], 1)
    return vn.reshape(-1, 3), vj.reshape(-1, 3), idx.reshape(-1)


def _all_candidates(g, to, fan, pts):
    """Every (point, triangle) pair with the point inside the closed triangle:
    barycentrics from signed areas (lambda_a = [PBC]/[ABC] and cyclic), each
    >= -1e-12.  Returns point, triangle index, T, a, B per pair.  Pixel
    centres are matched against the triangles' bounding boxes widened by a
    nanometre, ring points against every triangle."""
    vn, vj, idx = _mesh_triangles(fan, to.n_rays)
    X, Y = fan["x"][vn, vj], fan["y"][vn, vj]          # [K][3]
    Tv = vn * to.dtau
    Av, Bv = fan["amp"][vn, vj], fan["b"][vn, vj]
    pts = np.asarray(pts, np.float64)
    npx = g.n_pixels
    k_list, q_list = [], []
    # pixel centres: candidate pairs from the bounding boxes
    pad = 1e-9
    ilo = np.maximum(np.ceil((X.min(1) - pad - g.x0) / g.h), 0).astype(np.int64)
    ihi = np.minimum(np.floor((X.max(1) + pad - g.x0) / g.h), g.nx - 1).astype(np.int64)
    jlo = np.maximum(np.ceil((Y.min(1) - pad - g.y0) / g.h), 0).astype(np.int64)
    jhi = np.minimum(np.floor((Y.max(1) + pad - g.y0) / g.h), g.ny - 1).astype(np.int64)
    wi, wj = np.maximum(ihi - ilo + 1, 0), np.maximum(jhi - jlo + 1, 0)
    cnt = wi * wj
    k = np.repeat(np.arange(len(idx)), cnt)
    off = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ii = ilo[k] + off % np.maximum(wi[k], 1)
    jj = jlo[k] + off // np.maximum(wi[k], 1)
    k_list.append(k)
    q_list.append(jj * g.nx + ii)
    # ring points: every triangle
    for r in range(npx, len(pts)):
        k_list.append(np.arange(len(idx)))
        q_list.append(np.full(len(idx), r))
    k, q = np.concatenate(k_list), np.concatenate(q_list)
    px, py = pts[q, 0], pts[q, 1]
    ax, ay, bx, by, cx, cy = X[k, 0], Y[k, 0], X[k, 1], Y[k, 1], X[k, 2], Y[k, 2]

    def cross(ux, uy, vx, vy):
        return ux * vy - uy * vx

    area = cross(bx - ax, by - ay, cx - ax, cy - ay)
    ok = area != 0.0
    la = cross(bx - px, by - py, cx - px, cy - py) / np.where(ok, area, 1.0)
    lb = cross(cx - px, cy - py, ax - px, ay - py) / np.where(ok, area, 1.0)
    lc = cross(ax - px, ay - py, bx - px, by - py) / np.where(ok, area, 1.0)
    ok &= (la >= -1e-12) & (lb >= -1e-12) & (lc >= -1e-12)
    k, q, la, lb, lc = k[ok], q[ok], la[ok], lb[ok], lc[ok]
    lam = np.stack([la, lb, lc], 1)
    return (q, idx[k], (lam * Tv[k]).sum(1), (lam * Av[k]).sum(1), (lam * Bv[k]).sum(1))


def _check_plain_first_arrival(g, to, fan, T, A, B, quantum):
    """Compare the oracle's tables for one emitter (pixels then ring points,
    T = NaN where uncovered) with the plain first-arrival rule applied to
    every candidate: minimum interpolated T, exact ties to the smaller
    triangle index.  Returns (covered points, points with arrivals of two
    branches at least 1e-8 s apart, near-tie branch points).  A near-tie
    branch point has its two smallest candidates within `quantum` seconds
    of each other with amplitudes more than 1e-9 apart (relative): only
    there may a rule that orders arrivals to within `quantum` pick another
    branch; such points are exempt from the value check and counted."""
    pts = list(zip(*[a.ravel() for a in g.pixel_centres()])) + [tuple(p) for p in g.element_positions()]
    q, tri, t, a, b = _all_candidates(g, to, fan, pts)
    order = np.lexsort((tri, t, q))
    q, tri, t, a, b = q[order], tri[order], t[order], a[order], b[order]
    first = np.ones(len(q), bool)
    first[1:] = q[1:] != q[:-1]
    second = np.zeros(len(q), bool)
    second[1:] = first[:-1] & ~first[1:]
    covered = np.zeros(len(pts), bool)
    covered[q[first]] = True
    assert np.array_equal(np.isfinite(T), covered), "coverage differs from the plain rule"
    pf = q[first]
    Tb, Ab, Bb = t[first], a[first], b[first]
    # spread of arrival times per point (several branches where the wavefront folds)
    last = np.ones(len(q), bool)
    last[:-1] = q[1:] != q[:-1]
    spread = t[last] - Tb
    multi = int((spread > 1e-8).sum())
    # the runner-up candidate of each point that has one
    ps = q[second]
    t2 = np.full(len(pts), np.inf)
    a2 = np.full(len(pts), np.nan)
    t2[ps], a2[ps] = t[second], a[second]
    near = (t2[pf] - Tb <= quantum) & (np.abs(a2[pf] - Ab) > 1e-9 * np.abs(Ab))
    chk = ~near
    assert np.all(np.abs(T[pf][chk] - Tb[chk]) <= 1e-15 * Tb[chk] + 1e-21)
    assert np.all(np.abs(A[pf][chk] - Ab[chk]) <= 1e-11 * np.abs(Ab[chk]))
    assert np.all(np.abs(B[pf][chk] - Bb[chk]) <= 1e-11 * np.maximum(np.abs(Bb[chk]), 1e-3))
    return int(covered.sum()), multi, int(near.sum())


def _fold_counts(fan, nr):
    """Mesh cells of each orientation (sign of triangle 0's area): both signs
    mean neighbouring rays have crossed, i.e. the wavefront has folded."""
    vn, vj, _ = _mesh_triangles(fan, nr)
    vn, vj = vn[0::2], vj[0::2]
    X, Y = fan["x"][vn, vj], fan["y"][vn, vj]
    area = (X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0]) - (Y[:, 1] - Y[:, 0]) * (X[:, 2] - X[:, 0])
    return int((area > 0).sum()), int((area < 0).sum())


def test_rasterisation_plain_first_arrival_tiny_fan():
    """A tiny fan through a smooth bump: the tables equal the plain
    first-arrival rule applied to every triangle of the mesh."""
    g = W.centred_grid(14, 1e-3, 6, 5e-3, 1500.0)
    X, Y = g.pixel_centres()
    c = 1500.0 + 60.0 * np.exp(-((X - 1e-3) ** 2 + Y ** 2) / (2 * (2e-3) ** 2))
    al = np.full_like(c, 3.0)
    to = W.resolve_trace_opts(g, c, 11)
    to = W.TraceOpts(n_rays=11, dtau=4.0 * to.dtau, tau_max=to.tau_max, j_min=to.j_min)
    e = 2
    fan = rays.trace_fan(g, to, 1.0 / c, al, e)
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / c, al, e, e + 1)
    n_cov, _, near = _check_plain_first_arrival(g, to, fan, np.concatenate([T[0], Tr[0]]),
                                                np.concatenate([A[0], Ar[0]]), np.concatenate([B[0], Br[0]]),
                                                to.dtau * 2.0 ** -20)
    assert n_cov > 60 and near == 0


@pytest.mark.parametrize("case", ["tiny_lens", "ring64_lens"])
def test_rasterisation_plain_first_arrival_through_a_caustic(case):
    """A strong slow lens in front of the element folds its wavefront (mesh
    cells of both orientations; points reached by two branches whose
    arrival times differ by up to a few tenths of a microsecond and whose
    amplitudes differ severalfold).  The first arrival is the branch with
    the smallest travel time (Eq. 6; Discussion, back-propagation of ray
    parameters): the tables equal the plain rule at every point, and no
    point has two branches within 2^-20 of a ray step of each other."""
    if case == "tiny_lens":
        g = W.centred_grid(40, 0.5e-3, 8, 9e-3, 1500.0)
        c, al = W.lens_medium(g, (5e-3, 0.0), 1.5e-3, -400.0)
        nr = 41
    else:
        g = W.centred_grid(128, 0.5e-3, 64, 30e-3, 1500.0)
        c, al = W.lens_medium(g, (25e-3, 0.0), 1.5e-3, -400.0)
        nr = 360
    to = W.resolve_trace_opts(g, c, nr)
    fan = rays.trace_fan(g, to, 1.0 / c, al, 0)
    pos, neg = _fold_counts(fan, nr)
    assert min(pos, neg) > 0.02 * (pos + neg), (pos, neg)
    T, A, B, Tr, Ar, Br = rays.tables(g, to, 1.0 / c, al, 0, 1)
    n_cov, multi, near = _check_plain_first_arrival(g, to, fan, np.concatenate([T[0], Tr[0]]),
                                                    np.concatenate([A[0], Ar[0]]),
                                                    np.concatenate([B[0], Br[0]]), to.dtau * 2.0 ** -20)
    assert multi >= 20, multi
    assert near == 0
