"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle of the NURBS Splatting render path.

A plain, slow, brute-force reference (``nsplat_oracle.cpp``) that follows the
paper step by step (Sec. 3.1-3.4, Eq. 1-9, Suppl. S2 Eq. S1-S3, Eq. 14, and the
regularisers of Sec. 3.5, Eq. 11-12) and composites every Gaussian at every
pixel; the optimiser step (Adam with the cosine learning-rate decay and the
clamps of the supplementary settings) is written out in numpy below.  Only ``tests/``, the smoke check and
the CPU-baseline leg of the benchmark may import it.  It shares no code with
the GPU library and the GPU library never calls it.

Inputs are "curve batches": any object with the numpy attributes
``scene, degree, flags, key_off, tau_off, key_xy, key_w, key_s, tau, color,
opacity, hw, bg, channels`` (see ``paper_2606_31764_amd.synth``), converted
here to FP64 (exactly: they are FP32 values).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsplat_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

# Table S1 defaults, plus the readings the paper leaves open: alpha clamp,
# termination threshold, fill padding, and the support radius (alpha = 0 beyond
# cutoff * sigma; Eq. 9 itself has infinite support, cutoff <= 0 restores it).
DEFAULTS = dict(delta_c=10.0, delta_b=0.5, rho=2.0, eta=1.5, gamma=5.0, nl_factor=3.0,
                fill_pad=0.1, h=1.0, alpha_max=0.99, eps_T=1e-6, cutoff=6.0, delta_a=0.25, kappa=4)
ANISO = 4  # curve flag: tangent-aligned (anisotropic) contour Gaussians
NADJ = 9   # per-Gaussian adjoint slots: mx, my, sigma, opacity, colour (3), sp, theta

P_COUNT, P_NSAMP, P_IX0, P_IY0, P_NX, P_NY, P_GOFF, P_FLAG = range(8)
FLAG_NEAR_INT, FLAG_INVALID = 1, 2
KIND = dict(key_x=1, key_y=2, key_w=3, key_s=4, tau=5, opacity=6, color0=7, color1=8, color2=9)


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Curves(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("channels", ctypes.c_int32)] + [
        (n, ctypes.c_void_p) for n in ("scene", "degree", "flags", "key_off", "tau_off",
                                        "key_xy", "key_w", "key_s", "tau", "color", "opacity")]


class _Scenes(ctypes.Structure):
    _fields_ = [("n_scenes", ctypes.c_int32), ("hw", ctypes.c_void_p), ("bg", ctypes.c_void_p)]


_PARAM_NAMES = ("delta_c", "delta_b", "rho", "eta", "gamma", "nl_factor", "fill_pad", "h", "alpha_max", "eps_T",
                "cutoff", "delta_a")


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _PARAM_NAMES] + [("kappa", ctypes.c_int32)]


class _Reg(ctypes.Structure):
    _fields_ = [("bbox_weight", ctypes.c_double), ("bbox_kind", ctypes.c_int32), ("bbox", ctypes.c_void_p),
                ("deriv_weight", ctypes.c_double), ("deriv_order", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # NSPLAT_ORACLE_LIB: a separately built copy (e.g. with AddressSanitizer)
        _lib = ctypes.CDLL(os.environ.get("NSPLAT_ORACLE_LIB") or build())
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "or_plan": (i64, [vp, vp, vp, vp, vp]),
            "or_gaussians": (i64, [vp] * 11),
            "or_bin": (i64, [i64, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, i64]),
            "or_composite": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, vp]),
            "or_param_grad_seeds": (i32, [vp, vp, vp, vp, vp, i64, vp, vp]),
            "or_param_grad_seeds_scaled": (i32, [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp]),
            "or_param_grad_full": (i32, [vp] * 18),
            "or_curve_knots": (i32, [i32, i32, i32, i32, vp, vp]),
            "or_curve_eval": (i32, [i32, i32, i32, i32, vp, vp, vp, vp, i32, vp, i32, vp]),
            "or_basis_all": (i32, [i32, i32, vp, dbl, vp, vp]),
            "or_arc_length": (dbl, [i32, i32, i32, i32, vp, vp, vp, vp, i32]),
            "or_sdf": (i32, [i32, vp, dbl, dbl, vp]),
            "or_anneal": (dbl, [dbl, dbl, dbl, dbl, dbl, dbl]),
            "or_num_threads": (i32, []),
            "or_reg_loss": (dbl, [vp, vp, vp, vp, vp, i64, vp, vp]),
            "or_reg_grad_full": (dbl, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "or_curve_derivs": (i32, [i32, i32, i32, i32, vp, vp, vp, vp, i32, vp, i32, vp]),
            "or_udf_loss": (dbl, [vp, vp, vp, vp, vp, dbl, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype, f.argtypes = res, args
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _plan_rows(pl, n_curves):
    """A plan in the oracle's own layout: int32 [n_curves][8]."""
    pl = np.ascontiguousarray(pl, np.int32)
    if pl.shape != (n_curves, 8):
        raise ValueError("oracle plan must be int32 [%d][8] (got %s)" % (n_curves, pl.shape))
    return pl


class _Batch:
    """FP64 / int32 copies of a curve batch, kept alive with the ctypes views."""

    def __init__(self, b, params):
        self.keep = dict(
            scene=np.ascontiguousarray(b.scene, np.int32), degree=np.ascontiguousarray(b.degree, np.int32),
            flags=np.ascontiguousarray(b.flags, np.int32), key_off=np.ascontiguousarray(b.key_off, np.int32),
            tau_off=np.ascontiguousarray(b.tau_off, np.int32),
            key_xy=np.ascontiguousarray(b.key_xy, np.float64), key_w=np.ascontiguousarray(b.key_w, np.float64),
            key_s=np.ascontiguousarray(b.key_s, np.float64), tau=np.ascontiguousarray(b.tau, np.float64),
            color=np.ascontiguousarray(b.color, np.float64), opacity=np.ascontiguousarray(b.opacity, np.float64),
            hw=np.ascontiguousarray(b.hw, np.int32), bg=np.ascontiguousarray(b.bg, np.float64))
        k = self.keep
        self.n_curves = int(len(k["degree"]))
        self.channels = int(b.channels)
        self.curves = _Curves(self.n_curves, self.channels, *[_p(k[n]) for n in (
            "scene", "degree", "flags", "key_off", "tau_off", "key_xy", "key_w", "key_s", "tau", "color", "opacity")])
        self.scenes = _Scenes(int(len(k["hw"])), _p(k["hw"]), _p(k["bg"]))
        pr = dict(DEFAULTS)
        pr.update({n: v for n, v in (params or {}).items() if n in DEFAULTS})
        self.pdict = pr
        self.params = _Params(*[float(pr[n]) for n in _PARAM_NAMES], int(pr["kappa"]))

    def refs(self):
        return ctypes.byref(self.curves), ctypes.byref(self.scenes), ctypes.byref(self.params)


def plan(batch, params=None):
    """Per-curve plan [N][8] (count, n_samples, ix0, iy0, nx, ny, g_offset, flags:
    1 = delta L within 1e-9 of an integer, 2 = values outside the domain of
    Sec. 3.1, no Gaussians), arc lengths L [N], and the total number of Gaussians."""
    B = _Batch(batch, params)
    pl = np.zeros((B.n_curves, 8), np.int32)
    L = np.zeros(B.n_curves, np.float64)
    G = lib().or_plan(*B.refs(), _p(pl), _p(L))
    return pl, L, int(G)


def gaussians(batch, params=None, frozen_plan=None):
    """Gaussians in emission order: dict(mu [G,2], sigma, opacity, curve, local, plan, L,
    sp, tdir [G,2]); sigma is the axis along the tangent of a tangent-aligned
    Gaussian (curve flag ANISO), sp the axis across it and tdir its tangent
    (isotropic Gaussians: sp = sigma, tdir = (1, 0))."""
    B = _Batch(batch, params)
    if frozen_plan is None:
        pl, L, G = plan(batch, params)
    else:
        pl = _plan_rows(frozen_plan, B.n_curves)
        L = None
        G = int(pl[:, P_COUNT].sum())
    mu = np.zeros((G, 2)); sg = np.zeros(G); op = np.zeros(G)
    cv = np.zeros(G, np.int32); lc = np.zeros(G, np.int32)
    sp = np.zeros(G); td = np.zeros((G, 2))
    lib().or_gaussians(*B.refs(), _p(pl), _p(mu), _p(sg), _p(op), _p(cv), _p(lc), _p(sp), _p(td))
    return dict(mu=mu, sigma=sg, opacity=op, curve=cv, local=lc, plan=pl, L=L, sp=sp, tdir=td)


def tile_key_count(hw, tile):
    hw = np.asarray(hw)
    return int(sum(((h + tile - 1) // tile) * ((w + tile - 1) // tile) for h, w in hw))


def bin_gaussians(batch, g, tile=16, k_sigma=6.0):
    """Sec. 3.4 binning emulated in FP32 from the oracle's own centres: returns
    (ranges [n_tiles, 2] int32, idx [pairs] int32)."""
    hw = np.ascontiguousarray(batch.hw, np.int32)
    sc = _Scenes(int(len(hw)), _p(hw), None)
    gscene = np.ascontiguousarray(np.asarray(batch.scene, np.int32)[g["curve"]], np.int32)
    mu = np.ascontiguousarray(g["mu"], np.float64)
    sg = np.ascontiguousarray(g["sigma"], np.float64)
    nt = tile_key_count(hw, tile)
    ranges = np.zeros((nt, 2), np.int32)
    n = lib().or_bin(len(sg), _p(mu), _p(sg), _p(gscene), ctypes.byref(sc), tile, float(k_sigma),
                     _p(ranges), None, 0)
    idx = np.zeros(max(n, 1), np.int32)
    lib().or_bin(len(sg), _p(mu), _p(sg), _p(gscene), ctypes.byref(sc), tile, float(k_sigma),
                 _p(ranges), _p(idx), n)
    return ranges, idx[:n]


def _image_layout(batch):
    C = int(batch.channels)
    hw = np.asarray(batch.hw)
    n_img = int(sum(C * h * w for h, w in hw))
    n_t = int(sum(h * w for h, w in hw))
    return C, n_img, n_t


def composite(batch, g, params=None, pixels=None, upstream=None, with_abs=False):
    """Eq. 8-9 by brute force.  pixels None: full images, returned flat
    (per scene [C][H][W] concatenated) with T_final flat ([H][W] per scene).
    pixels [n,3] (scene, y, x): values [n, C] and T [n].  With upstream (same
    layout as the image) also returns adj [G, 7]: the gradient of
    sum(upstream * I) w.r.t. (mx, my, sigma, opacity, colour[0..2], sp, theta)
    per Gaussian ([G, 9]), and with with_abs adjabs [G, 9]: the same sums taken
    over the absolute values of every term (the scale of any evaluation's
    rounding error)."""
    B = _Batch(batch, params)
    C, n_img, n_t = _image_layout(batch)
    G = len(g["sigma"])
    mu = np.ascontiguousarray(g["mu"], np.float64)
    sg = np.ascontiguousarray(g["sigma"], np.float64)
    op = np.ascontiguousarray(g["opacity"], np.float64)
    cv = np.ascontiguousarray(g["curve"], np.int32)
    if pixels is None:
        img = np.zeros(n_img); T = np.zeros(n_t); pix = None; npix = 0
    else:
        pix = np.ascontiguousarray(pixels, np.int32).reshape(-1, 3)
        npix = len(pix)
        img = np.zeros((npix, C)); T = np.zeros(npix)
    up = None if upstream is None else np.ascontiguousarray(upstream, np.float64)
    adj = np.zeros((G, NADJ)) if up is not None else None
    adjabs = np.zeros((G, NADJ)) if (up is not None and with_abs) else None
    sp = g.get("sp")
    td = g.get("tdir")
    sp = None if sp is None else np.ascontiguousarray(sp, np.float64)
    td = None if td is None else np.ascontiguousarray(td, np.float64)
    lib().or_composite(*B.refs(), _p(np.ascontiguousarray(g["plan"], np.int32)), _p(mu), _p(sg), _p(op), _p(sp),
                       _p(td), _p(cv), G, npix, _p(pix), _p(img), _p(T), _p(up), _p(adj), _p(adjabs))
    if up is None:
        return img, T
    if with_abs:
        return img, T, adj, adjabs
    return img, T, adj


def param_grad(batch, g, adj, params=None, adjabs=None):
    """Gradient of the loss w.r.t. every curve parameter, given per-Gaussian
    adjoints.  With adjabs (composite(..., with_abs=True)) also returns the
    error scale of every component: sum_g adjabs_g . |d gaussian_g / d theta|."""
    B = _Batch(batch, params)
    k = B.keep
    names = ("key_xy", "key_w", "key_s", "tau", "color", "opacity")
    out = {n: np.zeros_like(k[n]) for n in names}
    scl = {n: np.zeros_like(k[n]) for n in names} if adjabs is not None else None
    ab = None if adjabs is None else np.ascontiguousarray(adjabs, np.float64)
    lib().or_param_grad_full(*B.refs(), _p(np.ascontiguousarray(g["plan"], np.int32)),
                             _p(np.ascontiguousarray(adj, np.float64)), *[_p(out[n]) for n in names], _p(ab),
                             *[(_p(scl[n]) if scl is not None else None) for n in names])
    if adjabs is None:
        return out
    return out, scl


def param_grad_seeds(batch, g, adj, seeds, params=None, adjabs=None):
    """Selected gradient components; seeds [n, 3] = (curve, kind, local index).
    With adjabs also returns their error scales (see param_grad)."""
    B = _Batch(batch, params)
    sd = np.ascontiguousarray(seeds, np.int32).reshape(-1, 3)
    out = np.zeros(len(sd))
    if adjabs is None:
        lib().or_param_grad_seeds(*B.refs(), _p(np.ascontiguousarray(g["plan"], np.int32)),
                                  _p(np.ascontiguousarray(adj, np.float64)), len(sd), _p(sd), _p(out))
        return out
    scale = np.zeros(len(sd))
    lib().or_param_grad_seeds_scaled(*B.refs(), _p(np.ascontiguousarray(g["plan"], np.int32)),
                                     _p(np.ascontiguousarray(adj, np.float64)),
                                     _p(np.ascontiguousarray(adjabs, np.float64)), len(sd), _p(sd), _p(out),
                                     _p(scale))
    return out, scale


def render(batch, params=None, frozen_plan=None):
    g = gaussians(batch, params, frozen_plan)
    img, T = composite(batch, g, params)
    return img, T, g


def loss_and_grad(batch, target, params=None, frozen_plan=None, with_scale=False):
    """L = sum (I - I*)^2 and its gradient w.r.t. every curve parameter (FP64).
    with_scale: the gradient is a pair (values, error scales), see param_grad."""
    g = gaussians(batch, params, frozen_plan)
    img, T = composite(batch, g, params)
    up = 2.0 * (img - target)
    if with_scale:
        _, _, adj, adjabs = composite(batch, g, params, upstream=up, with_abs=True)
        return float(np.sum((img - target) ** 2)), param_grad(batch, g, adj, params, adjabs), g, img
    _, _, adj = composite(batch, g, params, upstream=up)
    return float(np.sum((img - target) ** 2)), param_grad(batch, g, adj, params), g, img


# --- single-curve geometry (closed-form tests) --------------------------------------

def curve_knots(p, closed, tau, nk):
    tau = np.ascontiguousarray(tau, np.float64)
    U = np.zeros(len(tau) + 2 * p + 2)
    n = lib().or_curve_knots(p, int(closed), nk, len(tau), _p(tau), _p(U))
    return U[:n]


def curve_eval(p, closed, key_xy, key_w, key_s, tau, t, full=False):
    """(x, y, s, dx/du, dy/du, ds/du) at u = a + t (b - a)."""
    kx = np.ascontiguousarray(key_xy, np.float64).reshape(-1, 2)
    kw = np.ascontiguousarray(key_w, np.float64)
    ks = np.ascontiguousarray(key_s, np.float64)
    tu = np.ascontiguousarray(tau, np.float64)
    t = np.ascontiguousarray(np.atleast_1d(t), np.float64)
    out = np.zeros((len(t), 6))
    lib().or_curve_eval(p, int(closed), len(kx), len(tu), _p(kx), _p(kw), _p(ks), _p(tu), len(t), _p(t),
                        int(full), _p(out))
    return out


def basis_all(U, p, u):
    U = np.ascontiguousarray(U, np.float64)
    m = len(U) - 1
    N = np.zeros(m - p); dN = np.zeros(m - p)
    span = lib().or_basis_all(m, p, _p(U), float(u), _p(N), _p(dN))
    return N, dN, span


def arc_length(p, closed, key_xy, key_w, key_s, tau, n_L):
    kx = np.ascontiguousarray(key_xy, np.float64).reshape(-1, 2)
    kw = np.ascontiguousarray(key_w, np.float64)
    ks = np.ascontiguousarray(key_s, np.float64)
    tu = np.ascontiguousarray(tau, np.float64)
    return lib().or_arc_length(p, int(closed), len(kx), len(tu), _p(kx), _p(kw), _p(ks), _p(tu), int(n_L))


def sdf(poly, q):
    b = np.ascontiguousarray(poly, np.float64).reshape(-1, 2)
    out = np.zeros(3)
    lib().or_sdf(len(b), _p(b), float(q[0]), float(q[1]), _p(out))
    return out  # (d, wn, sdf)


def anneal(t, T, hmax, hmin, tb, te):
    return lib().or_anneal(float(t), float(T), float(hmax), float(hmin), float(tb), float(te))


def num_threads():
    return lib().or_num_threads()


# --- geometric regularisers (Sec. 3.5) and the optimiser step ------------------------

def _reg(bbox_weight=0.0, bbox_kind=0, bbox=None, deriv_weight=0.0, deriv_order=3):
    bb = None if bbox is None else np.ascontiguousarray(bbox, np.float64).reshape(-1, 4)
    return _Reg(float(bbox_weight), int(bbox_kind), _p(bb), float(deriv_weight), int(deriv_order)), bb


def reg_loss_grad(batch, plan_rows, params=None, **reg):
    """Value of lambda_bbox L_bbox (Eq. 12) + lambda_deriv L_deriv^r (Eq. 11, averaged over
    each scene's curves) at the samples of the given plan, and its gradient w.r.t. every
    key point, weight, width and interval (dict in the input layout)."""
    B = _Batch(batch, params)
    k = B.keep
    rg, keep_bb = _reg(**reg)
    out = dict(key_xy=np.zeros_like(k["key_xy"]), key_w=np.zeros_like(k["key_w"]),
               key_s=np.zeros_like(k["key_s"]), tau=np.zeros_like(k["tau"]),
               color=np.zeros_like(k["color"]), opacity=np.zeros_like(k["opacity"]))
    total = lib().or_reg_grad_full(*B.refs(), _p(_plan_rows(plan_rows, B.n_curves)), ctypes.byref(rg),
                                   *[_p(out[n]) for n in ("key_xy", "key_w", "key_s", "tau")])
    del keep_bb
    return float(total), out


def reg_loss(batch, plan_rows, params=None, **reg):
    """Value only (no gradient seeds)."""
    B = _Batch(batch, params)
    rg, keep_bb = _reg(**reg)
    v = lib().or_reg_loss(*B.refs(), _p(_plan_rows(plan_rows, B.n_curves)), ctypes.byref(rg), 0,
                          None, None)
    del keep_bb
    return float(v)


def curve_derivs(p, closed, key_xy, key_w, key_s, tau, t, r):
    """u-derivatives of order 0..r of (x, y) at u = a + t (b - a): array [len(t), r + 1, 2]."""
    kx = np.ascontiguousarray(key_xy, np.float64).reshape(-1, 2)
    kw = np.ascontiguousarray(key_w, np.float64)
    ks = np.ascontiguousarray(key_s, np.float64)
    tu = np.ascontiguousarray(tau, np.float64)
    t = np.ascontiguousarray(np.atleast_1d(t), np.float64)
    out = np.zeros((len(t), r + 1, 2))
    lib().or_curve_derivs(p, int(closed), len(kx), len(tu), _p(kx), _p(kw), _p(ks), _p(tu), len(t), _p(t),
                          int(r), _p(out))
    return out


def udf_loss(batch, plan_rows, image, target, tau, sel=None, params=None):
    """Distance-weighted image loss (LIVE's unsigned-distance weights): value,
    dL/dImage (image layout) and the per-pixel distance d."""
    B = _Batch(batch, params)
    img = np.ascontiguousarray(image, np.float64).ravel()
    tgt = np.ascontiguousarray(target, np.float64).ravel()
    dL = np.zeros_like(img)
    npix = int(sum(int(h) * int(w) for h, w in batch.hw))
    dist = np.zeros(npix)
    sl = None if sel is None else np.ascontiguousarray(sel, np.int32)
    v = lib().or_udf_loss(*B.refs(), _p(_plan_rows(plan_rows, B.n_curves)), _p(sl), float(tau), _p(img),
                          _p(tgt), _p(dL), _p(dist))
    return float(v), dL, dist


GROUPS = ("key_xy", "key_w", "key_s", "tau", "color", "opacity")


def cosine_lr(lr0, t, total, final_ratio):
    """Cosine decay from lr0 at t = 0 to final_ratio * lr0 at t = total (held after)."""
    x = min(max(t / total, 0.0), 1.0)
    lo = final_ratio * lr0
    return lo + (lr0 - lo) * 0.5 * (1.0 + np.cos(np.pi * x))


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, total=1000, final_ratio=0.1,
              w_range=(0.01, 10.0), tau_range=(0.0, 2.0)):
    """One Adam step (Kingma & Ba, Alg. 1; eps added to the bias-corrected root)
    on every parameter group, at step t >= 1 with the learning rate of group
    g = cosine_lr(lr[g], t - 1, total, final_ratio), then the clamps of the
    supplementary settings (rational weights to w_range, knot intervals to
    tau_range).  Updates params, m, v in place (FP64)."""
    for i, g in enumerate(GROUPS):
        x, d = params[g], grads[g]
        m[g][...] = beta1 * m[g] + (1.0 - beta1) * d
        v[g][...] = beta2 * v[g] + (1.0 - beta2) * d * d
        mh = m[g] / (1.0 - beta1 ** t)
        vh = v[g] / (1.0 - beta2 ** t)
        x -= cosine_lr(lr[i], t - 1, total, final_ratio) * mh / (np.sqrt(vh) + eps)
        if g == "key_w":
            np.clip(x, w_range[0], w_range[1], out=x)
        if g == "tau":
            np.clip(x, tau_range[0], tau_range[1], out=x)


def timed(fn, *a, **kw):
    t0 = time.perf_counter()
    r = fn(*a, **kw)
    return r, time.perf_counter() - t0
