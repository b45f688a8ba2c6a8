"""Pins of the FP64 oracle against things other than itself: closed forms,
independent textbook algorithms (de Boor, de Casteljau, Boehm insertion),
invariances, brute force, and central finite differences.  CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2606_31764_amd import synth

R2 = math.sqrt(2.0) / 2.0


# ---------------------------------------------------------------------------------
# independent evaluators (not the Cox-de Boor recursion of the oracle)
# ---------------------------------------------------------------------------------

def de_boor(U, P, p, u):
    """de Boor's triangular point evaluation of a polynomial B-spline (NURBS Book A3.1 style)."""
    m = len(U) - 1
    k = p
    while k < m - p - 1 and not (U[k] <= u < U[k + 1]):
        k += 1
    if u >= U[m - p]:
        k = m - p - 1
        while U[k] == U[k + 1]:
            k -= 1
    d = [np.array(P[j + k - p], float) for j in range(p + 1)]
    for r in range(1, p + 1):
        for j in range(p, r - 1, -1):
            i = j + k - p
            den = U[i + p + 1 - r] - U[i]
            a = 0.0 if den == 0 else (u - U[i]) / den
            d[j] = (1 - a) * d[j - 1] + a * d[j]
    return d[p]


def de_casteljau_rational(P, w, t):
    """Rational Bezier point by de Casteljau in homogeneous coordinates."""
    H = [np.array([*(np.asarray(P[i], float) * w[i]), w[i]]) for i in range(len(P))]
    n = len(H) - 1
    for r in range(1, n + 1):
        for i in range(n - r + 1):
            H[i] = (1 - t) * H[i] + t * H[i + 1]
    return H[0][:-1] / H[0][-1]


def boehm_insert(U, Pw, p, ubar):
    """Insert knot ubar once (Boehm) into homogeneous control points Pw [n+1, d]."""
    k = max(i for i in range(len(U) - 1) if U[i] <= ubar < U[i + 1])
    Q = []
    for i in range(len(Pw) + 1):
        if i <= k - p:
            Q.append(Pw[i])
        elif i >= k + 1:
            Q.append(Pw[i - 1])
        else:
            a = (ubar - U[i]) / (U[i + p] - U[i])
            Q.append(a * Pw[i] + (1 - a) * Pw[i - 1])
    U2 = np.concatenate([U[:k + 1], [ubar], U[k + 1:]])
    return U2, np.array(Q)


def rand_curve(rng, nk, p, closed=False):
    xy = rng.uniform(0, 100, (nk, 2))
    w = rng.uniform(0.5, 2.0, nk)
    s = rng.uniform(1.0, 4.0, nk)
    tau = rng.uniform(0.2, 1.5, nk if closed else nk - p)
    return xy, w, s, tau


# ---------------------------------------------------------------------------------
# geometry (Sec. 3.1, Eq. 1-3)
# ---------------------------------------------------------------------------------

def test_rational_quadratic_is_exact_circular_arc():
    c, r = np.array([40.0, 30.0]), 25.0
    P = c + r * np.array([[1, 0], [1, 1], [0, 1]], float)
    out = oracle.curve_eval(2, False, P, [1.0, R2, 1.0], [1, 1, 1], [0.7], np.linspace(0, 1, 257))
    rad = np.hypot(out[:, 0] - c[0], out[:, 1] - c[1])
    assert np.abs(rad - r).max() < 1e-12 * r
    # tangent orthogonal to the radius: (C - c) . C' = 0
    dot = (out[:, 0] - c[0]) * out[:, 3] + (out[:, 1] - c[1]) * out[:, 4]
    speed = np.hypot(out[:, 3], out[:, 4])
    assert np.abs(dot / (r * speed)).max() < 1e-12


def test_nine_point_nurbs_circle_with_repeated_knots():
    c, r = np.array([50.0, 50.0]), 20.0
    P = c + r * np.array([(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0)], float)
    w = [1, R2, 1, R2, 1, R2, 1, R2, 1]
    tau = [0.25, 0, 0.25, 0, 0.25, 0, 0.25]
    t = np.concatenate([np.linspace(0, 1, 401), [0.25, 0.5, 0.75, 1.0]])
    out = oracle.curve_eval(2, False, P, w, np.ones(9), tau, t)
    assert np.abs(np.hypot(out[:, 0] - c[0], out[:, 1] - c[1]) - r).max() < 1e-12 * r
    L = oracle.arc_length(2, False, P, w, np.ones(9), tau, 20000)
    assert abs(L - 2 * math.pi * r) < 1e-6 * r


def test_partition_of_unity():
    rng = np.random.default_rng(7)
    for p in range(1, 6):
        for _ in range(6):
            n_int = int(rng.integers(1, 8))
            iv = rng.uniform(0.0, 1.0, n_int) * (rng.uniform(size=n_int) > 0.25)
            iv[0] = max(iv[0], 0.3)
            U = np.concatenate([np.zeros(p + 1), np.cumsum(iv), np.full(p, iv.sum())])
            for u in np.concatenate([np.linspace(0, U[-1], 37), [U[-1]]]):
                N, dN, _ = oracle.basis_all(U, p, u)
                assert abs(N.sum() - 1.0) < 1e-13
                assert abs(dN.sum()) < 1e-11 * (1 + np.abs(dN).max())
                assert N.min() >= -1e-15


def test_span_local_sum_equals_full_sum():
    rng = np.random.default_rng(11)
    for p in (1, 2, 3, 5):
        for closed in (False, True):
            xy, w, s, tau = rand_curve(rng, 9, p, closed)
            t = rng.uniform(0, 1, 50)
            a = oracle.curve_eval(p, closed, xy, w, s, tau, t, full=False)
            b = oracle.curve_eval(p, closed, xy, w, s, tau, t, full=True)
            assert np.abs(a - b).max() < 1e-10


def test_unit_weights_reduce_to_polynomial_bspline():
    rng = np.random.default_rng(3)
    for p in (1, 2, 3, 4, 5):
        xy, _, s, tau = rand_curve(rng, 11, p)
        U = oracle.curve_knots(p, False, tau, 11)
        t = np.concatenate([rng.uniform(0, 1, 40), [0.0, 1.0]])
        out = oracle.curve_eval(p, False, xy, np.ones(11), s, tau, t)
        a, b = U[p], U[-p - 1]
        P3 = np.concatenate([xy, s[:, None]], 1)
        for i, ti in enumerate(t):
            u = b if ti >= 1 else a + ti * (b - a)
            ref = de_boor(U, P3, p, u)
            assert np.abs(out[i, :3] - ref).max() < 1e-12 * 100


def test_single_span_reduces_to_rational_bezier():
    rng = np.random.default_rng(5)
    for p in (1, 2, 3, 4, 5):
        xy, w, s, _ = rand_curve(rng, p + 1, p)
        t = np.linspace(0, 1, 33)
        out = oracle.curve_eval(p, False, xy, w, s, [0.37], t)
        P3 = np.concatenate([xy, s[:, None]], 1)
        for i, ti in enumerate(t):
            assert np.abs(out[i, :3] - de_casteljau_rational(P3, w, ti)).max() < 1e-12 * 100


def test_knot_insertion_leaves_curve_unchanged():
    rng = np.random.default_rng(9)
    for p in (2, 3, 4):
        nk = 8
        xy, w, s, tau = rand_curve(rng, nk, p)
        U = oracle.curve_knots(p, False, tau, nk)
        ubar = 0.5 * (U[p + 1] + U[p + 2]) if U[p + 2] > U[p + 1] else U[p] + 0.37 * (U[-1] - U[p])
        Pw = np.concatenate([xy * w[:, None], (s * w)[:, None], w[:, None]], 1)
        U2, Q = boehm_insert(U, Pw, p, ubar)
        w2 = Q[:, 3]
        xy2, s2 = Q[:, :2] / w2[:, None], Q[:, 2] / w2
        tau2 = np.diff(U2)[p:len(U2) - 1 - p]
        t = np.concatenate([rng.uniform(0, 1, 60), [0, 1]])
        a = oracle.curve_eval(p, False, xy, w, s, tau, t)
        b = oracle.curve_eval(p, False, xy2, w2, s2, tau2, t)
        assert np.abs(a[:, :3] - b[:, :3]).max() < 1e-11


def test_greville_linear_precision_gives_exact_length_and_count():
    rng = np.random.default_rng(2)
    p, nk = 3, 9
    tau = rng.uniform(0.5, 1.5, nk - p)
    U = oracle.curve_knots(p, False, tau, nk)
    grev = np.array([U[i + 1:i + p + 1].mean() for i in range(nk)])
    A, B = np.array([3.0, 7.0]), np.array([53.0, 37.0])
    xy = A + (grev[:, None] - U[p]) / (U[-p - 1] - U[p]) * (B - A)
    L = oracle.arc_length(p, False, xy, np.ones(nk), np.ones(nk), tau, 192)
    assert abs(L - np.hypot(*(B - A))) < 1e-12 * 60
    b = synth._assemble([dict(scene=0, degree=p, flags=0, key_xy=xy, key_w=np.ones(nk), key_s=np.full(nk, 2.0),
                              tau=tau, color=np.zeros(3), opacity=1.0)], [[64, 64]], [[1, 1, 1]], 3)
    # delta_c such that delta_c L is not near an integer
    plan, Lp, G = oracle.plan(b, dict(delta_c=2.0, kappa=4))
    assert plan[0, oracle.P_NSAMP] == math.ceil(2.0 * np.hypot(*(B - A)))
    assert G == plan[0, oracle.P_NSAMP] + 8


def test_closed_wrap_order_and_closure():
    rng = np.random.default_rng(4)
    K = rng.uniform(0, 50, (7, 2))
    # uniform cubic: C(u_p) = (K[n-2] + 4 K[n-1] + K[0]) / 6 (wrap of ceil(3/2) = 2 key points)
    out = oracle.curve_eval(3, True, K, np.ones(7), np.ones(7), np.ones(7), [0.0, 1.0])
    ref = (K[5] + 4 * K[6] + K[0]) / 6
    assert np.abs(out[0, :2] - ref).max() < 1e-12 * 50
    assert np.abs(out[0, :3] - out[1, :3]).max() < 1e-12 * 50          # C(u_p) = C(u_{m-p})
    assert np.abs(out[0, 3:] - out[1, 3:]).max() < 1e-10 * 50          # C' matches too
    # uniform quadratic: C(u_p) = (K[n-1] + K[0]) / 2 (wrap of ceil(2/2) = 1)
    out2 = oracle.curve_eval(2, True, K, np.ones(7), np.ones(7), np.ones(7), [0.0])
    assert np.abs(out2[0, :2] - (K[6] + K[0]) / 2).max() < 1e-12 * 50
    # non-uniform rational closed curves close with matching tangents
    for p in (2, 3, 4, 5):
        xy, w, s, tau = rand_curve(rng, 8, p, closed=True)
        o = oracle.curve_eval(p, True, xy, w, s, tau, [0.0, 1.0])
        assert np.abs(o[0] - o[1]).max() < 1e-9


# ---------------------------------------------------------------------------------
# Gaussians (Sec. 3.2 / 3.3) and invariances
# ---------------------------------------------------------------------------------

def _one_open(rng, p=3, nk=8, size=64):
    xy, w, s, tau = rand_curve(rng, nk, p)
    xy = xy * (size / 100.0)
    return synth._assemble([dict(scene=0, degree=p, flags=0, key_xy=xy, key_w=w, key_s=s, tau=tau,
                                 color=np.array([0.2, 0.3, 0.1]), opacity=0.8)], [[size, size]], [[1, 1, 1]], 3)


def test_endpoint_replication_and_interpolation():
    b = _one_open(np.random.default_rng(1))
    g = oracle.gaussians(b, dict(delta_c=2.0, kappa=4))
    M = g["plan"][0, oracle.P_NSAMP]
    assert len(g["sigma"]) == M + 8
    assert np.all(g["mu"][:5] == g["mu"][4])
    assert np.all(g["mu"][-5:] == g["mu"][-5])
    assert np.abs(g["mu"][0] - b.key_xy[0]).max() < 1e-12 * 64            # clamped ends interpolate
    assert np.abs(g["mu"][-1] - b.key_xy[-1]).max() < 1e-12 * 64
    assert np.abs(g["sigma"][0] - b.key_s[0] / 2.0) < 1e-12                 # sigma = s / rho


def test_convex_hull_and_width_range():
    rng = np.random.default_rng(12)
    b = _one_open(rng, p=3, nk=10)
    g = oracle.gaussians(b, dict(delta_c=3.0, kappa=0))
    assert g["sigma"].min() * 2 >= b.key_s.min() - 1e-12
    assert g["sigma"].max() * 2 <= b.key_s.max() + 1e-12
    # each centre lies in the hull of the p+1 control points of its span
    U = oracle.curve_knots(3, False, b.tau, 10)
    M = g["plan"][0, oracle.P_NSAMP]
    from scipy.spatial import Delaunay
    for j in range(0, M, 7):
        u = U[3] + j * ((U[-4] - U[3]) / (M - 1)) if j < M - 1 else U[-4]
        k = max(i for i in range(3, len(U) - 4) if U[i] <= u) if u < U[-4] else len(U) - 5
        pts = b.key_xy[k - 3:k + 1].astype(np.float64)
        hull = Delaunay(pts + 1e-9 * np.random.default_rng(j).normal(size=pts.shape))
        assert hull.find_simplex(g["mu"][j]) >= 0 or np.min(np.linalg.norm(pts - g["mu"][j], axis=1)) < 1e-9


def _loss_grad(b, tgt, prm, plan):
    return oracle.loss_and_grad(b, tgt, prm, frozen_plan=plan)


def test_weight_and_knot_scale_invariance():
    b = synth.config2(seed=2300, n_curves=4, size=64)
    prm = dict(delta_c=2.0)
    tgt = oracle.render(synth.perturbed(b, 5), prm)[0]
    plan, _, _ = oracle.plan(b, prm)
    L0, g0, gs0, img0 = _loss_grad(b, tgt, prm, plan)
    for attr in ("key_w", "tau"):
        b2 = b.copy()
        setattr(b2, attr, getattr(b, attr).astype(np.float64) * 1.7)
        gs2 = oracle.gaussians(b2, prm, plan)
        assert np.abs(gs2["mu"] - gs0["mu"]).max() < 1e-10
        assert np.abs(gs2["sigma"] - gs0["sigma"]).max() < 1e-12
    # Euler identities: sum_i w_i dL/dw_i = 0 per curve, sum_j tau_j dL/dtau_j = 0 per curve
    for c in range(b.n_curves):
        k0, k1 = b.key_off[c], b.key_off[c + 1]
        t0, t1 = b.tau_off[c], b.tau_off[c + 1]
        sw = np.dot(b.key_w[k0:k1], g0["key_w"][k0:k1])
        st = np.dot(b.tau[t0:t1], g0["tau"][t0:t1])
        assert abs(sw) < 1e-9 * (np.abs(b.key_w[k0:k1] * g0["key_w"][k0:k1]).sum() + 1e-12)
        assert abs(st) < 1e-9 * (np.abs(b.tau[t0:t1] * g0["tau"][t0:t1]).sum() + 1e-12)


def test_translation_moves_centres_and_gradient_identity():
    b = synth.config2(seed=2400, n_curves=3, size=64)
    prm = dict(delta_c=2.0)
    plan, _, _ = oracle.plan(b, prm)
    g0 = oracle.gaussians(b, prm, plan)
    b2 = b.copy()
    b2.key_xy = b.key_xy.astype(np.float64) + np.array([2.5, -1.25])
    g2 = oracle.gaussians(b2, prm, plan)
    assert np.abs(g2["mu"] - g0["mu"] - np.array([2.5, -1.25])).max() < 1e-11
    tgt = oracle.render(synth.perturbed(b, 6), prm)[0]
    img, T = oracle.composite(b, g0, prm)
    _, _, adj = oracle.composite(b, g0, prm, upstream=2 * (img - tgt))
    gr = oracle.param_grad(b, g0, adj, prm)
    assert np.allclose(gr["key_xy"].sum(0), adj[:, :2].sum(0), rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------------------------
# compositing (Sec. 3.4, Eq. 8-9)
# ---------------------------------------------------------------------------------

def _gauss_batch(centres, sigmas, opac, colours, size=8, bg=(0.2, 0.4, 0.6)):
    parts = [dict(scene=0, degree=1, flags=0, key_xy=np.zeros((2, 2)), key_w=np.ones(2), key_s=np.ones(2),
                  tau=[1.0], color=np.asarray(c, float), opacity=1.0) for c in colours]
    b = synth._assemble(parts, [[size, size]], [bg], 3)
    n = len(centres)
    plan = np.zeros((n, 8), np.int32)
    plan[:, oracle.P_COUNT] = 1
    plan[:, oracle.P_GOFF] = np.arange(n)
    g = dict(mu=np.asarray(centres, float), sigma=np.asarray(sigmas, float), opacity=np.asarray(opac, float),
             curve=np.arange(n, dtype=np.int32), local=np.zeros(n, np.int32), plan=plan)
    return b, g


def test_one_and_two_gaussian_closed_forms():
    prm = dict(alpha_max=0.99, eps_T=0.0)
    bg = np.array([0.25, 0.375, 0.625])          # exact in FP32, the batch's storage type
    c1, c2 = np.array([0.875, 0.125, 0.3125]), np.array([0.0, 0.75, 0.5])
    b, g = _gauss_batch([[3.2, 4.1]], [1.3], [0.7], [c1], bg=bg)
    img, T = oracle.composite(b, g, prm, pixels=[[0, 2, 5]])
    a = 0.7 * math.exp(-((5.5 - 3.2) ** 2 + (2.5 - 4.1) ** 2) / (2 * 1.3 ** 2))
    assert np.abs(img[0] - (c1 * a + bg * (1 - a))).max() < 1e-15
    # two: the later one (index 1) is in front
    b, g = _gauss_batch([[3.2, 4.1], [4.0, 3.0]], [1.3, 0.9], [0.7, 0.6], [c1, c2], bg=bg)
    img, T = oracle.composite(b, g, prm, pixels=[[0, 2, 5]])
    a1 = 0.7 * math.exp(-((5.5 - 3.2) ** 2 + (2.5 - 4.1) ** 2) / (2 * 1.3 ** 2))
    a2 = 0.6 * math.exp(-((5.5 - 4.0) ** 2 + (2.5 - 3.0) ** 2) / (2 * 0.9 ** 2))
    ref = c2 * a2 + c1 * a1 * (1 - a2) + bg * (1 - a1) * (1 - a2)
    assert np.abs(img[0] - ref).max() < 1e-15
    assert abs(T[0] - (1 - a1) * (1 - a2)) < 1e-15


def test_clamp_and_termination():
    prm = dict(alpha_max=0.99, eps_T=1e-6)
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [0, 1, 1]]
    b, g = _gauss_batch([[4.5, 4.5]] * 5, [2.0] * 5, [1.0] * 5, cols)
    img, T = oracle.composite(b, g, prm, pixels=[[0, 4, 4]])
    # alpha = min(0.99, 1) at the centre: three layers take T to 1e-6 (< eps only after the 4th)
    assert abs(T[0] - 0.01 ** 4) < 1e-18
    ref = np.zeros(3)
    Tr = 1.0
    for c in cols[::-1][:4]:
        ref += np.array(c) * 0.99 * Tr
        Tr *= 0.01
    ref += Tr * np.array([0.2, 0.4, 0.6], np.float32).astype(np.float64)
    assert np.abs(img[0] - ref).max() < 1e-15


def test_same_colour_permutation_invariance():
    rng = np.random.default_rng(8)
    n = 12
    cent = rng.uniform(0, 8, (n, 2))
    sg = rng.uniform(0.5, 2, n)
    op = rng.uniform(0.2, 0.9, n)
    prm = dict(eps_T=0.0)
    b, g = _gauss_batch(cent, sg, op, [[0.3, 0.6, 0.9]] * n)
    img, _ = oracle.composite(b, g, prm)
    perm = rng.permutation(n)
    b2, g2 = _gauss_batch(cent[perm], sg[perm], op[perm], [[0.3, 0.6, 0.9]] * n)
    img2, _ = oracle.composite(b2, g2, prm)
    assert np.abs(img - img2).max() < 1e-12


def test_all_transparent_gives_background():
    b, g = _gauss_batch([[4, 4]], [1.0], [0.0], [[1, 0, 0]])
    img, T = oracle.composite(b, g, dict())
    assert np.all(T == 1.0)
    np.testing.assert_array_equal(img.reshape(3, 8, 8)[1], float(np.float32(0.4)))


# ---------------------------------------------------------------------------------
# SDF (Suppl. S2) and annealing (Eq. 14)
# ---------------------------------------------------------------------------------

@pytest.mark.parametrize("N", [3, 5, 8, 13])
def test_sdf_regular_polygon(N):
    R, c = 10.0, np.array([20.0, 15.0])
    ang = 2 * np.pi * np.arange(N) / N
    poly = c + R * np.stack([np.cos(ang), np.sin(ang)], 1)
    d, wn, s = oracle.sdf(poly, c)
    assert abs(d - R * math.cos(math.pi / N)) < 1e-12 and abs(wn - 1) < 1e-12 and s > 0
    d, wn, s = oracle.sdf(poly, c + np.array([3 * R, 0.5]))
    assert abs(wn) < 1e-12 and s < 0 and abs(s + d) < 1e-15
    d, wn, s = oracle.sdf(poly[::-1], c)
    assert abs(wn + 1) < 1e-12 and s < 0                 # clockwise: outside by the wn > 1/2 rule
    # a point on an edge midpoint has distance 0
    mid = 0.5 * (poly[0] + poly[1])
    assert oracle.sdf(poly, mid)[0] < 1e-12


def test_fill_opacity_inside_outside():
    b = synth.config3(seed=3400, n_paths=1, size=96)
    b.key_xy[:] = 48 + 30 * np.stack([np.cos(2 * np.pi * np.arange(len(b.key_xy)) / len(b.key_xy)),
                                      np.sin(2 * np.pi * np.arange(len(b.key_xy)) / len(b.key_xy))], 1)
    b.key_w[:] = 1.0
    b.opacity[:] = 0.8
    g = oracle.gaussians(b, dict(h=1.0))
    r = np.hypot(g["mu"][:, 0] - 48, g["mu"][:, 1] - 48)
    assert np.abs(g["opacity"][r < 10] - float(np.float32(0.8))).max() < 1e-12
    far = r > r.max() - 1
    assert g["opacity"][far].max() < 1e-6


def test_annealing_schedule():
    hmax, hmin, tb, te, T = 8.0, 1.0, 0.1, 0.8, 1000
    assert oracle.anneal(0, T, hmax, hmin, tb, te) == hmax
    assert oracle.anneal(100, T, hmax, hmin, tb, te) == hmax
    assert abs(oracle.anneal(450, T, hmax, hmin, tb, te) - 4.5) < 1e-12
    assert abs(oracle.anneal(800, T, hmax, hmin, tb, te) - hmin) < 1e-15
    assert oracle.anneal(1000, T, hmax, hmin, tb, te) == hmin
    hs = [oracle.anneal(t, T, hmax, hmin, tb, te) for t in range(T + 1)]
    assert all(a >= b for a, b in zip(hs, hs[1:]))


# ---------------------------------------------------------------------------------
# binning (Sec. 3.4) vs brute-force rectangle enumeration
# ---------------------------------------------------------------------------------

def test_binning_matches_brute_force():
    b = synth.config2(seed=2500, n_curves=5, size=70)
    prm = dict(delta_c=2.0)
    g = oracle.gaussians(b, prm)
    for tile in (8, 16, 32):
        ranges, idx = oracle.bin_gaussians(b, g, tile=tile, k_sigma=6.0)
        nx, ny = -(-70 // tile), -(-70 // tile)
        for t in range(nx * ny):
            tx, ty = t % nx, t // nx
            want = []
            for k in range(len(g["sigma"])):
                m = g["mu"][k].astype(np.float32)
                r = np.float32(6.0) * np.float32(g["sigma"][k])
                lo, hi = (m - r) - np.float32(1), (m + r) + np.float32(1)
                if (math.floor(lo[0] / tile) <= tx <= math.floor(hi[0] / tile)
                        and math.floor(lo[1] / tile) <= ty <= math.floor(hi[1] / tile)):
                    want.append(k)
            got = idx[ranges[t, 0]:ranges[t, 1]].tolist() if ranges[t, 1] > ranges[t, 0] else []
            assert got == want


# ---------------------------------------------------------------------------------
# analytic gradient vs central finite differences (frozen plan, no termination)
# ---------------------------------------------------------------------------------

def _fd_check(b, prm, tgt, names, nper=3, eps=1e-6, seed=0):
    plan, _, _ = oracle.plan(b, prm)
    _, gr, _, _ = oracle.loss_and_grad(b, tgt, prm, frozen_plan=plan)
    rng = np.random.default_rng(seed)
    worst = 0.0
    scale = max(np.abs(gr[n]).max() for n in names)
    for n in names:
        flat = getattr(b, n).reshape(-1)
        for i in rng.choice(len(flat), min(nper, len(flat)), replace=False):
            h = eps * max(1.0, abs(float(flat[i])))
            vals = []
            for sgn in (1, -1):
                bb = b.copy()
                a = getattr(b, n).astype(np.float64).reshape(-1).copy()
                a[i] += sgn * h
                setattr(bb, n, a.reshape(getattr(b, n).shape))
                vals.append(np.sum((oracle.render(bb, prm, plan)[0] - tgt) ** 2))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = gr[n].reshape(-1)[i]
            worst = max(worst, abs(fd - an) / (1e-6 * scale + 1e-6 * abs(an) + 1e-7))
    return worst


def test_fd_strokes():
    prm = dict(delta_c=1.5, eps_T=0.0)
    b = synth.config1()
    b.opacity[:] = 0.8
    tgt = oracle.render(synth.config1(1001), prm)[0]
    assert _fd_check(b, prm, tgt, ["key_xy", "key_w", "key_s", "tau", "opacity", "color"]) < 1.0


def test_fd_fills():
    prm = dict(h=3.0, eps_T=0.0)
    b = synth.config3(seed=3500, n_paths=4, size=64)
    b.opacity[:] = np.minimum(b.opacity, 0.9)
    tgt = oracle.render(synth.config3(seed=3501, n_paths=4, size=64), prm)[0]
    assert _fd_check(b, prm, tgt, ["key_xy", "key_w", "tau", "opacity", "color"]) < 1.0
