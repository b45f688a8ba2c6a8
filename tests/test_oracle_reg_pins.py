"""Pins of the oracle's geometric regularisers (Sec. 3.5: derivative loss
Eq. 11, bounding-box loss Eq. 12) and of its optimiser step (Adam with the
cosine learning-rate decay and the clamps of the supplementary settings),
against closed forms, an independent derivative formula (Bernstein forward
differences), the independent first-derivative path of Eq. 2 and central
finite differences.  CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2606_31764_amd import synth


def _bernstein(n, i, t):
    return math.comb(n, i) * t ** i * (1.0 - t) ** (n - i)


def _bezier_deriv(P, k, t, span):
    """k-th u-derivative of a polynomial Bezier curve on a domain of length span:
    p!/(p-k)! / span^k * sum_i Delta^k P_i B_{i,p-k}(t)."""
    p = len(P) - 1
    if k > p:
        return np.zeros(2)
    D = np.asarray(P, float)
    for _ in range(k):
        D = D[1:] - D[:-1]
    n = p - k
    s = sum(_bernstein(n, i, t) * D[i] for i in range(n + 1))
    return math.factorial(p) / math.factorial(p - k) / span ** k * s


@pytest.mark.parametrize("p", [3, 5])
def test_polynomial_bezier_derivatives_match_forward_differences(p):
    rng = np.random.default_rng(10 + p)
    P = rng.uniform(-20, 20, (p + 1, 2))
    tau = [rng.uniform(0.5, 2.0)]
    ts = np.array([0.0, 0.17, 0.5, 0.83, 1.0])
    d = oracle.curve_derivs(p, False, P, np.ones(p + 1), np.ones(p + 1), tau, ts, 4)
    for i, t in enumerate(ts):
        for k in range(5):
            ref = _bezier_deriv(P, k, t, tau[0])
            assert np.allclose(d[i, k], ref, rtol=1e-11, atol=1e-9 * (1 + np.abs(ref).max())), (k, t)


def test_cubic_bspline_third_derivative_piecewise_constant():
    rng = np.random.default_rng(21)
    p, nk = 3, 9
    P = rng.uniform(0, 50, (nk, 2))
    tau = rng.uniform(0.5, 1.5, nk - p)
    U = oracle.curve_knots(p, False, tau, nk)
    a, b = U[p], U[-p - 1]
    for s in range(p, len(U) - p - 1):
        if U[s + 1] <= U[s]:
            continue
        ts = (np.linspace(U[s], U[s + 1], 7)[1:-1] - a) / (b - a)
        d3 = oracle.curve_derivs(p, False, P, np.ones(nk), np.ones(nk), tau, ts, 3)[:, 3]
        assert np.abs(d3 - d3[0]).max() <= 1e-9 * (1 + np.abs(d3).max())


@pytest.mark.parametrize("closed", [False, True])
def test_rational_derivatives_match_differences_of_eq2(closed):
    """C'' and C''' of a rational cubic against central differences of C' from
    the Eq. 2 path (a different code path: curve_eval's quotient rule)."""
    rng = np.random.default_rng(31 + closed)
    p, nk = 3, 8
    P = rng.uniform(0, 60, (nk, 2))
    w = rng.uniform(0.5, 2.0, nk)
    tau = rng.uniform(0.5, 1.5, nk if closed else nk - p)
    U = oracle.curve_knots(p, closed, tau, nk)
    a, b = U[p], U[-p - 1]
    # interior points of spans, away from knots
    ts = []
    for s in range(p, len(U) - p - 1):
        if U[s + 1] > U[s]:
            ts += [(U[s] + f * (U[s + 1] - U[s]) - a) / (b - a) for f in (0.3, 0.6)]
    ts = np.array(ts)
    d = oracle.curve_derivs(p, closed, P, w, np.ones(nk), tau, ts, 3)
    h = 1e-4 / (b - a)
    c1 = lambda t: oracle.curve_eval(p, closed, P, w, np.ones(nk), tau, t)[:, 3:5]
    assert np.allclose(d[:, 1], c1(ts), rtol=1e-12, atol=1e-10)
    d2 = (c1(ts + h) - c1(ts - h)) / (2 * h * (b - a))
    d3 = (c1(ts + h) - 2 * c1(ts) + c1(ts - h)) / (h * (b - a)) ** 2
    sc2 = np.abs(d[:, 2]).max()
    sc3 = np.abs(d[:, 3]).max()
    assert np.abs(d[:, 2] - d2).max() <= 1e-6 * sc2
    assert np.abs(d[:, 3] - d3).max() <= 1e-4 * sc3


def _one_curve_batch(xy, w, s, tau, p, closed=False, filled=False, hw=(64, 64)):
    flags = (synth.CLOSED if closed else 0) | (synth.FILLED if filled else 0)
    return synth._assemble([dict(scene=0, degree=p, flags=flags, key_xy=np.asarray(xy, float),
                                 key_w=np.asarray(w, float), key_s=np.asarray(s, float),
                                 tau=np.asarray(tau, float), color=np.zeros(3), opacity=1.0)],
                           [list(hw)], [[1, 1, 1]], 3)


def _greville_line(A, B, p=3, nk=9, seed=2):
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0.5, 1.5, nk - p)
    U = oracle.curve_knots(p, False, tau, nk)
    grev = np.array([U[i + 1:i + p + 1].mean() for i in range(nk)])
    xy = A + (grev[:, None] - U[p]) / (U[-p - 1] - U[p]) * (B - A)
    return xy, tau


def test_derivative_loss_vanishes_on_linearly_parametrised_line():
    xy, tau = _greville_line(np.array([3.0, 7.0]), np.array([53.0, 37.0]))
    b = _one_curve_batch(xy, np.ones(9), np.full(9, 2.0), tau, 3)
    plan, _, _ = oracle.plan(b, dict(delta_c=2.0))
    # the key points are stored in FP32, so the line is linear in u to ~1e-6 px
    bent = b.copy()
    bent.key_xy = b.key_xy + np.array([[0.0, 3.0]]) * np.sin(np.arange(9))[:, None]
    for r in (2, 3):
        v, g = oracle.reg_loss_grad(b, plan, dict(delta_c=2.0), deriv_weight=1.0, deriv_order=r)
        vb, gb = oracle.reg_loss_grad(bent, plan, dict(delta_c=2.0), deriv_weight=1.0, deriv_order=r)
        assert abs(v) < 1e-9 * vb
        # a minimum: every gradient vanishes too
        gs = max(np.abs(gb[n]).max() for n in ("key_xy", "key_w", "tau"))
        assert max(np.abs(g[n]).max() for n in ("key_xy", "key_w", "tau")) < 1e-4 * gs


def test_derivative_loss_of_a_bezier_cubic_is_its_constant_third_derivative():
    rng = np.random.default_rng(41)
    P = rng.uniform(5, 55, (4, 2))
    tau = [1.3]
    b = _one_curve_batch(P, np.ones(4), np.full(4, 2.0), tau, 3)
    prm = dict(delta_c=1.0)
    plan, _, _ = oracle.plan(b, prm)
    v = oracle.reg_loss(b, plan, prm, deriv_weight=2.5, deriv_order=3)
    P = P.astype(np.float32).astype(np.float64)          # the batch stores FP32 values
    t0 = float(np.float32(tau[0]))
    c3 = 6.0 * (P[3] - 3 * P[2] + 3 * P[1] - P[0]) / t0 ** 3
    assert abs(v - 2.5 * float(c3 @ c3)) <= 1e-12 * v


@pytest.mark.parametrize("kind", [0, 1])
def test_bbox_loss_closed_form_on_a_line(kind):
    """Samples of a linearly parametrised line are u-uniform points on it, so the
    penalty sums have a closed form."""
    A, B = np.array([-10.0, 20.0]), np.array([90.0, 30.0])
    xy, tau = _greville_line(A, B, seed=5)
    b = _one_curve_batch(xy, np.ones(9), np.full(9, 2.0), tau, 3, hw=(64, 64))
    prm = dict(delta_c=1.0)
    plan, _, _ = oracle.plan(b, prm)
    M = int(plan[0, oracle.P_NSAMP])
    pts = A + np.linspace(0.0, 1.0, M)[:, None] * (B - A)
    if kind == 0:
        phi = lambda x: np.maximum(x, 0.0)
    else:
        phi = lambda x: np.logaddexp(0.0, x)
    ref = np.sum(phi(0.0 - pts[:, 0]) + phi(pts[:, 0] - 64.0) + phi(0.0 - pts[:, 1]) + phi(pts[:, 1] - 64.0))
    v = oracle.reg_loss(b, plan, prm, bbox_weight=1.5, bbox_kind=kind)
    assert abs(v - 1.5 * ref) <= 1e-7 * (1 + ref)   # FP32-stored key points: ~1e-6 px
    # a custom box per scene
    box = np.array([[5.0, 22.0, 60.0, 26.0]])
    ref = np.sum(phi(5.0 - pts[:, 0]) + phi(pts[:, 0] - 60.0) + phi(22.0 - pts[:, 1]) + phi(pts[:, 1] - 26.0))
    v = oracle.reg_loss(b, plan, prm, bbox_weight=1.0, bbox_kind=kind, bbox=box)
    assert abs(v - ref) <= 1e-7 * (1 + ref)


def test_bbox_loss_zero_inside():
    b = synth.config2(seed=2200, n_curves=4, size=256)
    prm = dict(delta_c=2.0)
    plan, _, _ = oracle.plan(b, prm)
    big = np.array([[-1e4, -1e4, 1e4, 1e4]])
    v, g = oracle.reg_loss_grad(b, plan, prm, bbox_weight=1.0, bbox_kind=0, bbox=big)
    assert v == 0.0 and all(np.all(g[n] == 0.0) for n in g)


def _reg_fd(b, prm, plan, names, reg, nper=4, eps=1e-6, seed=0):
    v0, g = oracle.reg_loss_grad(b, plan, prm, **reg)
    rng = np.random.default_rng(seed)
    scale = max(np.abs(g[n]).max() for n in names)
    worst = 0.0
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
                vals.append(oracle.reg_loss(bb, plan, prm, **reg))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = g[n].reshape(-1)[i]
            worst = max(worst, abs(fd - an) / (1e-6 * scale + 1e-6 * abs(an) + 1e-9))
    return worst


def test_reg_gradient_matches_finite_differences_strokes():
    b = synth.config2(seed=2300, n_curves=3, size=96)
    b.key_xy = b.key_xy + np.array([60.0, -30.0])   # push parts outside the canvas
    prm = dict(delta_c=1.0)
    plan, _, _ = oracle.plan(b, prm)
    reg = dict(bbox_weight=0.7, bbox_kind=1, deriv_weight=0.3, deriv_order=3)
    assert _reg_fd(b, prm, plan, ["key_xy", "key_w", "tau"], reg) < 1.0


def test_reg_gradient_matches_finite_differences_fills():
    b = synth.config3(seed=2400, n_paths=3, size=64)
    b.key_xy = b.key_xy * 1.3 - 5.0
    prm = dict(h=4.0)
    plan, _, _ = oracle.plan(b, prm)
    reg = dict(bbox_weight=1.0, bbox_kind=1, deriv_weight=0.5, deriv_order=3)
    assert _reg_fd(b, prm, plan, ["key_xy", "key_w", "tau"], reg) < 1.0


def test_cosine_learning_rate_ends():
    assert oracle.cosine_lr(2.0, 0, 100, 0.1) == 2.0
    assert abs(oracle.cosine_lr(2.0, 50, 100, 0.1) - 1.1) < 1e-15
    assert abs(oracle.cosine_lr(2.0, 100, 100, 0.1) - 0.2) < 1e-15
    assert abs(oracle.cosine_lr(2.0, 250, 100, 0.1) - 0.2) < 1e-15


def test_adam_constant_gradient_moves_by_lr_each_step():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2,
    so every step moves a parameter by lr_t * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    shapes = dict(key_xy=(5, 2), key_w=(5,), key_s=(5,), tau=(2,), color=(1, 3), opacity=(1,))
    prm = {n: rng.uniform(0.5, 1.5, s) for n, s in shapes.items()}
    grd = {n: rng.normal(0, 1, s) for n, s in shapes.items()}
    m = {n: np.zeros(s) for n, s in shapes.items()}
    v = {n: np.zeros(s) for n, s in shapes.items()}
    lr = [1.5, 0.1, 0.2, 0.1, 0.01, 0.01]
    x = {n: a.copy() for n, a in prm.items()}
    for t in range(1, 6):
        before = {n: a.copy() for n, a in x.items()}
        oracle.adam_step(x, grd, m, v, t, lr, total=10, final_ratio=0.1, w_range=(-1e9, 1e9),
                         tau_range=(-1e9, 1e9))
        for i, n in enumerate(oracle.GROUPS):
            step = oracle.cosine_lr(lr[i], t - 1, 10, 0.1) * grd[n] / (np.abs(grd[n]) + 1e-8)
            assert np.allclose(before[n] - x[n], step, rtol=1e-9, atol=1e-15), (n, t)


def test_adam_clamps_weights_and_intervals():
    shapes = dict(key_xy=(2, 2), key_w=(2,), key_s=(2,), tau=(2,), color=(1, 3), opacity=(1,))
    x = {n: np.full(s, 0.5) for n, s in shapes.items()}
    x["key_w"][:] = [0.011, 9.99]
    x["tau"][:] = [0.001, 1.999]
    g = {n: np.zeros(s) for n, s in shapes.items()}
    g["key_w"][:] = [1.0, -1.0]      # pushes 0.011 down and 9.99 up
    g["tau"][:] = [1.0, -1.0]
    m = {n: np.zeros(s) for n, s in shapes.items()}
    v = {n: np.zeros(s) for n, s in shapes.items()}
    oracle.adam_step(x, g, m, v, 1, [1.0] * 6)
    assert np.array_equal(x["key_w"], [0.01, 10.0])
    assert np.array_equal(x["tau"], [0.0, 2.0])


def test_derivative_loss_approximates_the_integral_within_the_trapezoid_bound():
    """Quintic Bezier: ||C'''(u)||^2 is a degree-4 polynomial whose domain average
    is integrated exactly here; the sample-based value of Eq. 11 must be within
    the composite trapezoid error bound (b - a)^2 / (12 (M-1)^2) max|f''|."""
    rng = np.random.default_rng(51)
    p = 5
    P = rng.uniform(5, 55, (p + 1, 2)).astype(np.float32).astype(np.float64)
    tau = [float(np.float32(2.0))]
    b = _one_curve_batch(P, np.ones(p + 1), np.full(p + 1, 2.0), tau, p)
    prm = dict(delta_c=0.5)
    plan, _, _ = oracle.plan(b, prm)
    M = int(plan[0, oracle.P_NSAMP])
    v = oracle.reg_loss(b, plan, prm, deriv_weight=1.0, deriv_order=3)
    # f(t) = ||C'''(t tau)||^2 on t in [0, 1], from the Bernstein forward differences
    ts = np.linspace(0.0, 1.0, 401)
    c3 = np.array([_bezier_deriv(P, 3, t, tau[0]) for t in ts])
    f = np.sum(c3 ** 2, axis=1)
    coef = np.polyfit(ts, f, 4)
    exact = np.polyval(np.polyint(coef), 1.0) - np.polyval(np.polyint(coef), 0.0)
    f2 = np.abs(np.polyval(np.polyder(coef, 2), ts)).max()
    bound = f2 / (12.0 * (M - 1) ** 2)
    assert abs(v - exact) <= bound + 1e-9 * exact
    assert abs(v - exact) > 0.0 or f2 == 0.0


def _seg_dist_np(q, A, B):
    """Distance from points q [n, 2] to segments A->B [m, 2] (numpy, vectorised)."""
    e = B - A
    ee = np.sum(e * e, axis=1)
    r = q[:, None, :] - A[None, :, :]
    t = np.where(ee > 0, np.sum(r * e[None], axis=2) / np.where(ee > 0, ee, 1.0), 0.0)
    t = np.clip(t, 0.0, 1.0)
    pnt = A[None] + t[..., None] * e[None] - q[:, None, :]
    return np.sqrt(np.sum(pnt * pnt, axis=2)).min(axis=1)


def test_udf_weights_against_a_numpy_brute_force():
    """Distances to the boundary polyline (boundary points taken from the
    separate curve_eval path, distances by a vectorised numpy projection),
    weights max(0, tau - d) normalised per scene, loss and dL/dI."""
    b = synth.config3(seed=5800, n_paths=3, size=40)
    prm = dict(h=2.0)
    plan, _, _ = oracle.plan(b, prm)
    rng = np.random.default_rng(3)
    n_img = 3 * 40 * 40
    img, tgt = rng.uniform(0, 1, n_img), rng.uniform(0, 1, n_img)
    sel = np.array([1, 0, 1], np.int32)
    tau = 6.0
    v, dL, dist = oracle.udf_loss(b, plan, img, tgt, tau, sel=sel, params=prm)
    ys, xs = np.mgrid[0:40, 0:40]
    q = np.stack([xs.ravel() + 0.5, ys.ravel() + 0.5], 1).astype(np.float64)
    d = np.full(len(q), np.inf)
    for c in np.nonzero(sel)[0]:
        k0, k1 = b.key_off[c], b.key_off[c + 1]
        t0, t1 = b.tau_off[c], b.tau_off[c + 1]
        nb = int(plan[c, oracle.P_NSAMP])
        pts = oracle.curve_eval(int(b.degree[c]), True, b.key_xy[k0:k1], b.key_w[k0:k1], b.key_s[k0:k1],
                                b.tau[t0:t1], np.arange(nb) / nb)[:, :2]
        d = np.minimum(d, _seg_dist_np(q, pts, np.roll(pts, -1, axis=0)))
    assert np.allclose(dist, d, rtol=0, atol=1e-9)
    wq = np.maximum(0.0, tau - d)
    wn = wq / wq.sum()
    e = (img - tgt).reshape(3, -1)
    assert abs(v - np.sum(wn * np.sum(e * e, axis=0) / 3)) <= 1e-12
    assert np.allclose(dL.reshape(3, -1), 2 * wn * e / 3, rtol=0, atol=1e-15)


def test_udf_weights_sum_to_one_and_vanish_beyond_tau():
    b = synth.concat([synth.config3(seed=5900, n_paths=2, size=32), synth.config3(seed=5901, n_paths=2, size=24)])
    prm = dict(h=2.0)
    plan, _, _ = oracle.plan(b, prm)
    n_img = 3 * (32 * 32 + 24 * 24)
    img = np.full(n_img, 0.75)
    tgt = np.full(n_img, 0.25)
    v, dL, dist = oracle.udf_loss(b, plan, img, tgt, 4.0, params=prm)
    # a constant error e per channel: L = sum_s sum_q w (e^2) = (number of scenes) e^2
    assert abs(v - 2 * 0.25) <= 1e-12
    # zero gradient wherever d >= tau
    far = np.concatenate([np.tile(dist[:32 * 32] >= 4.0, 3), np.tile(dist[32 * 32:] >= 4.0, 3)])
    assert np.all(dL[far] == 0.0) and np.any(dL != 0.0)
