"""Pins of the oracle's tangent-aligned (anisotropic) contour Gaussians, the
variant of Eq. 5 the paper contrasts its isotropic sampling with (Sec. 3.2;
the early prototype with Bezier Splatting's contour sampling, supplementary
S4.5).  Reading: sigma_across = s / rho, sigma_along = max(sigma_across,
|C'(u_j)| du / rho) along t = C' / |C'|, du the sample spacing in u, and the
count M = ceil(delta_a L).  Pinned by the reduction to Eq. 5, a closed form on
a straight segment, rotation by 90 degrees, and central finite differences.
CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2606_31764_amd import synth

A = oracle.ANISO


def _stroke(xy, flags=0, p=3, w=None, s=None, tau=None, colour=(0.2, 0.5, 0.8), o=0.9, seed=0):
    rng = np.random.default_rng(seed)
    xy = np.asarray(xy, float)
    nk = len(xy)
    closed = bool(flags & synth.CLOSED)
    nt = nk if closed else nk - p
    return dict(scene=0, degree=p, flags=flags, key_xy=xy,
                key_w=rng.uniform(0.6, 1.6, nk) if w is None else np.asarray(w, float),
                key_s=rng.uniform(1.0, 2.0, nk) if s is None else np.asarray(s, float),
                tau=rng.uniform(0.5, 1.5, nt) if tau is None else np.asarray(tau, float), color=colour, opacity=o)


def _batch(parts, size=48):
    return synth._assemble(parts, [[size, size]], [[1.0, 1.0, 1.0]], 3)


def test_dense_sampling_reduces_to_eq5():
    """Where the sample spacing |C'| du / rho stays below s / rho, both axes
    equal s / rho and the Gaussians, hence the image, are those of Eq. 5."""
    rng = np.random.default_rng(3)
    xy = rng.uniform(8, 40, (7, 2))
    kw = dict(w=np.ones(7), tau=np.ones(4), seed=1)   # unit weights, uniform knots: a near-uniform speed
    iso = _batch([_stroke(xy, **kw)])
    ani = _batch([_stroke(xy, flags=A, **kw)])
    prm = dict(delta_c=16.0, delta_a=16.0)   # spacing ~0.06 px against widths of 1-2 px
    gi = oracle.gaussians(iso, prm)
    ga = oracle.gaussians(ani, prm)
    np.testing.assert_array_equal(gi["plan"], ga["plan"])
    assert np.all(ga["sigma"] == ga["sp"])   # the axis across won everywhere
    assert np.abs(ga["mu"] - gi["mu"]).max() < 1e-13
    assert np.abs(ga["sigma"] - gi["sigma"]).max() < 1e-13
    assert np.abs(ga["sp"] - gi["sigma"]).max() < 1e-13
    ii, _ = oracle.composite(iso, gi, prm)
    ia, _ = oracle.composite(ani, ga, prm)
    assert np.abs(ia - ii).max() < 1e-12
    # and the tangents are unit vectors along C'
    assert np.abs(np.hypot(ga["tdir"][:, 0], ga["tdir"][:, 1]) - 1.0).max() < 1e-12


@pytest.mark.parametrize("angle", [0.0, 0.7, 2.3])
def test_straight_segment_closed_form(angle):
    """A degree-1 segment from P to Q: C' is constant, so every Gaussian has
    t = (Q - P) / |Q - P|, sigma_along = |Q - P| / ((M - 1) rho) and
    sigma_across = s / rho; with M = 2 and no endpoint copies the image is the
    two-layer compositing of Eq. 8 with the elliptical Eq. 9, written out here."""
    c = np.array([24.0, 24.0])
    d = np.array([math.cos(angle), math.sin(angle)])
    P, Q = c - 9.0 * d, c + 9.0 * d
    s = 1.5
    part = _stroke([P, Q], flags=A, p=1, w=[1.0, 1.0], s=[s, s], tau=[1.0], o=0.7, colour=(0.1, 0.6, 0.3))
    b = _batch([part])
    P, Q = b.key_xy.astype(np.float64)          # the FP32 inputs the renderer sees
    length = float(np.hypot(*(Q - P)))
    d = (Q - P) / length
    prm = dict(delta_a=0.05, kappa=0, rho=2.0)   # M = max(2, ceil(0.05 * 18)) = 2
    g = oracle.gaussians(b, prm)
    assert g["plan"][0, oracle.P_NSAMP] == 2 and len(g["sigma"]) == 2
    np.testing.assert_allclose(g["mu"], np.stack([P, Q]), atol=1e-12)
    np.testing.assert_allclose(g["tdir"], np.stack([d, d]), atol=1e-12)
    np.testing.assert_allclose(g["sigma"], length / 1 / 2.0, rtol=1e-12)     # |Q - P| / ((M - 1) rho)
    np.testing.assert_allclose(g["sp"], s / 2.0, rtol=1e-12)
    img, T = oracle.composite(b, g, dict(prm, cutoff=0.0))
    img = img.reshape(3, 48, 48)
    yy, xx = np.mgrid[0:48, 0:48]
    px, py = xx + 0.5, yy + 0.5

    def alpha(m):
        dx, dy = px - m[0], py - m[1]
        dp = dx * d[0] + dy * d[1]
        dq = -dx * d[1] + dy * d[0]
        o = float(np.float32(0.7))  # the batch holds FP32 inputs
        return np.minimum(0.99, o * np.exp(-0.5 * (dp ** 2 / (length / 2.0) ** 2 + dq ** 2 / (s / 2.0) ** 2)))

    aP, aQ = alpha(P), alpha(Q)
    for ch, col in enumerate(np.float32([0.1, 0.6, 0.3]).astype(np.float64)):
        # Q is the later Gaussian: in front
        want = col * aQ + (1 - aQ) * (col * aP + (1 - aP) * 1.0)
        assert np.abs(img[ch] - want).max() < 1e-12


def test_rotation_by_90_degrees():
    """Rotating every key point by 90 degrees about the centre of a square
    canvas maps pixel centres onto pixel centres, so the image rotates with it
    (the tangents and the two axes follow the curve)."""
    rng = np.random.default_rng(7)
    xy = np.round(rng.uniform(10, 38, (8, 2)) * 64) / 64   # exact in FP32, before and after the rotation
    W = 48
    rot = np.stack([W - xy[:, 1], xy[:, 0]], 1)         # (x, y) -> (W - y, x)
    prm = dict(delta_a=0.3)
    b0 = _batch([_stroke(xy, flags=A, s=np.full(8, 1.2), seed=2)], W)
    b1 = _batch([_stroke(rot, flags=A, s=np.full(8, 1.2), seed=2)], W)
    i0, _, g0 = oracle.render(b0, prm)
    i1, _, g1 = oracle.render(b1, prm)
    assert np.sum(g0["sigma"] > g0["sp"] * 1.5) > 10        # genuinely anisotropic
    i0 = i0.reshape(3, W, W)
    i1 = i1.reshape(3, W, W)
    # pixel (x, y) of the original lands on (W - 1 - y, x)
    y, x = np.mgrid[0:W, 0:W]
    assert np.abs(i1[:, x, W - 1 - y] - i0[:, y, x]).max() < 1e-10


def _fd(b, prm, tgt, names, nper=4, seed=0):
    plan, _, _ = oracle.plan(b, prm)
    _, gr, _, _ = oracle.loss_and_grad(b, tgt, prm, frozen_plan=plan)
    rng = np.random.default_rng(seed)
    worst = 0.0
    scale = max(np.abs(gr[n]).max() for n in names)
    for n in names:
        flat = getattr(b, n).reshape(-1)
        for i in rng.choice(len(flat), min(nper, len(flat)), replace=False):
            h = 1e-6 * max(1.0, abs(float(flat[i])))
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


@pytest.mark.parametrize("closed", [False, True])
def test_finite_differences(closed):
    """The analytic gradient (forward mode through t, both axes and the sample
    spacing; per-pixel adjoint of the elliptical Eq. 9) against central
    differences of the oracle's own loss at a frozen plan."""
    rng = np.random.default_rng(11 if closed else 12)
    parts = []
    for k in range(3):
        if closed:
            nk = 7
            ang = 2 * np.pi * np.arange(nk) / nk
            xy = np.stack([16 + 8 * k + 7 * np.cos(ang), 18 + 6 * k + 7 * np.sin(ang)], 1)
            parts.append(_stroke(xy, flags=A | synth.CLOSED, s=rng.uniform(0.8, 1.4, nk), seed=20 + k,
                                 colour=tuple(rng.uniform(0, 1, 3)), o=0.8))
        else:
            xy = rng.uniform(8, 40, (6, 2))
            parts.append(_stroke(xy, flags=A, s=rng.uniform(0.8, 1.4, 6), seed=20 + k,
                                 colour=tuple(rng.uniform(0, 1, 3)), o=0.8))
    b = _batch(parts)
    prm = dict(delta_a=0.35, eps_T=0.0, cutoff=8.0)
    g = oracle.gaussians(b, prm)
    assert np.sum(g["sigma"] > g["sp"] * 1.2) > 10
    tgt = oracle.render(synth.perturbed(b, 3), prm)[0]
    assert _fd(b, prm, tgt, ["key_xy", "key_w", "key_s", "tau", "opacity", "color"]) < 1.0
