"""Seeded synthetic curve batches shaped like the paper's workloads.

This module only draws random inputs (key points, weights, knot intervals,
widths, colours, opacities, canvases).  It holds none of the render path's
arithmetic, so both the GPU path and the CPU oracle may take their inputs from
it.  The paper's own data (calligraphy fonts, Noto Emoji) is not available;
the generators reproduce the shapes the paper describes: calligraphy-like open
strokes with per-control-point widths (Sec. 4.1 / 5.2), star-shaped filled
closed paths as in layer-wise vectorisation (Sec. 4.2 / 5.3), and long
smoothing splines as in the efficiency study (Suppl. S4.1).

All arrays are numpy, FP32 for real values and int32 for indices; curves are
grouped by scene in ascending scene order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

CLOSED = 1
FILLED = 2
ANISO = 4      # tangent-aligned contour Gaussians (strokes only)


@dataclasses.dataclass
class CurveBatch:
    """CSR over curves.  key_off / tau_off have n_curves + 1 entries.  Open
    curves store n_k - p knot intervals, closed curves n_k (Sec. 3.1)."""
    scene: np.ndarray      # [N] int32
    degree: np.ndarray     # [N] int32
    flags: np.ndarray      # [N] int32 (CLOSED | FILLED | ANISO)
    key_off: np.ndarray    # [N+1] int32
    tau_off: np.ndarray    # [N+1] int32
    key_xy: np.ndarray     # [K, 2] float32, pixels (y down)
    key_w: np.ndarray      # [K] float32 rational weights
    key_s: np.ndarray      # [K] float32 stroke widths (px)
    tau: np.ndarray        # [T] float32 knot intervals
    color: np.ndarray      # [N, C] float32
    opacity: np.ndarray    # [N] float32
    hw: np.ndarray         # [S, 2] int32 (height, width)
    bg: np.ndarray         # [S, C] float32
    channels: int = 3

    @property
    def n_curves(self) -> int:
        return int(len(self.degree))

    @property
    def n_scenes(self) -> int:
        return int(len(self.hw))

    def copy(self) -> "CurveBatch":
        return dataclasses.replace(self, **{f.name: np.array(getattr(self, f.name)) for f in dataclasses.fields(self)
                                            if isinstance(getattr(self, f.name), np.ndarray)})

    def select_scene(self, s: int) -> "CurveBatch":
        """The curves of scene s as a one-scene batch."""
        idx = np.nonzero(self.scene == s)[0]
        return _gather(self, idx, new_scene_of=lambda c: 0, hw=self.hw[s:s + 1], bg=self.bg[s:s + 1])


def _gather(b: CurveBatch, idx, new_scene_of, hw, bg) -> CurveBatch:
    parts = []
    for c in idx:
        k0, k1 = b.key_off[c], b.key_off[c + 1]
        t0, t1 = b.tau_off[c], b.tau_off[c + 1]
        parts.append(dict(scene=new_scene_of(c), degree=int(b.degree[c]), flags=int(b.flags[c]),
                          key_xy=b.key_xy[k0:k1], key_w=b.key_w[k0:k1], key_s=b.key_s[k0:k1],
                          tau=b.tau[t0:t1], color=b.color[c], opacity=float(b.opacity[c])))
    return _assemble(parts, hw, bg, b.channels)


def _assemble(parts, hw, bg, channels) -> CurveBatch:
    nk = [len(p["key_xy"]) for p in parts]
    nt = [len(p["tau"]) for p in parts]
    cat = lambda name, dim: (np.concatenate([np.asarray(p[name], np.float32).reshape(-1, *dim) for p in parts])
                             if parts else np.zeros((0,) + dim, np.float32))
    return CurveBatch(
        scene=np.array([p["scene"] for p in parts], np.int32),
        degree=np.array([p["degree"] for p in parts], np.int32),
        flags=np.array([p["flags"] for p in parts], np.int32),
        key_off=np.concatenate([[0], np.cumsum(nk)]).astype(np.int32),
        tau_off=np.concatenate([[0], np.cumsum(nt)]).astype(np.int32),
        key_xy=cat("key_xy", (2,)), key_w=cat("key_w", ()), key_s=cat("key_s", ()), tau=cat("tau", ()),
        color=np.array([np.asarray(p["color"], np.float32).reshape(channels) for p in parts], np.float32).reshape(-1, channels),
        opacity=np.array([p["opacity"] for p in parts], np.float32),
        hw=np.asarray(hw, np.int32).reshape(-1, 2), bg=np.asarray(bg, np.float32).reshape(-1, channels),
        channels=channels)


def concat(batches: List[CurveBatch]) -> CurveBatch:
    """Scenes of several batches, one after another."""
    parts, hw, bg = [], [], []
    base = 0
    ch = batches[0].channels
    for b in batches:
        assert b.channels == ch
        for c in range(b.n_curves):
            k0, k1 = b.key_off[c], b.key_off[c + 1]
            t0, t1 = b.tau_off[c], b.tau_off[c + 1]
            parts.append(dict(scene=base + int(b.scene[c]), degree=int(b.degree[c]), flags=int(b.flags[c]),
                              key_xy=b.key_xy[k0:k1], key_w=b.key_w[k0:k1], key_s=b.key_s[k0:k1],
                              tau=b.tau[t0:t1], color=b.color[c], opacity=float(b.opacity[c])))
        hw.append(b.hw)
        bg.append(b.bg)
        base += b.n_scenes
    return _assemble(parts, np.concatenate(hw), np.concatenate(bg), ch)


def _taus(rng, n, normalise=True):
    t = rng.uniform(0.5, 1.5, n)
    return t / t.sum() if normalise else t


# ---------------------------------------------------------------------------------
# Open strokes: calligraphy-like random walks (configs 1 and 2)
# ---------------------------------------------------------------------------------

def strokes(seed, n_curves=32, size=256, nk_range=(12, 40), step=8.0, width=(1.0, 8.0), degree=3,
            weights=(0.3, 3.0), channels=3, margin=None, scene=0, flags=0) -> List[dict]:
    rng = np.random.default_rng(seed)
    margin = size * 0.1 if margin is None else margin
    parts = []
    for _ in range(n_curves):
        nk = int(rng.integers(nk_range[0], nk_range[1] + 1))
        nk = max(nk, degree + 1)
        p0 = rng.uniform(margin, size - margin, 2)
        walk = np.cumsum(rng.normal(0.0, step, (nk, 2)), axis=0)
        walk[0] = 0.0
        xy = np.clip(p0 + walk - walk[0], 1.0, size - 1.0)
        parts.append(dict(scene=scene, degree=degree, flags=flags, key_xy=xy,
                          key_w=np.exp(rng.uniform(math.log(weights[0]), math.log(weights[1]), nk)),
                          key_s=rng.uniform(width[0], width[1], nk), tau=_taus(rng, nk - degree),
                          color=np.zeros(channels), opacity=1.0))
    return parts


def config1(seed=1000):
    """One open cubic, 8 control points in a 64x64 canvas, width 2, black on white."""
    rng = np.random.default_rng(seed)
    nk = 8
    part = dict(scene=0, degree=3, flags=0, key_xy=rng.uniform(0.0, 64.0, (nk, 2)),
                key_w=rng.uniform(0.5, 2.0, nk), key_s=np.full(nk, 2.0), tau=_taus(rng, nk - 3),
                color=np.zeros(3), opacity=1.0)
    return _assemble([part], [[64, 64]], [[1.0, 1.0, 1.0]], 3)


def config2(seed=2000, n_curves=32, size=256):
    return _assemble(strokes(seed, n_curves=n_curves, size=size), [[size, size]], [[1.0, 1.0, 1.0]], 3)


# ---------------------------------------------------------------------------------
# Filled closed paths: star-shaped around random centres (config 3)
# ---------------------------------------------------------------------------------

def fills(seed, n_paths=256, size=512, nk_range=(6, 24), radius=(5.0, 80.0), degrees=(2, 3), channels=3,
          scene=0) -> List[dict]:
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(n_paths):
        p = int(rng.choice(degrees))
        nk = int(rng.integers(nk_range[0], nk_range[1] + 1))
        nk = max(nk, p + 1)
        c = rng.uniform(0.0, size, 2)
        R = math.exp(rng.uniform(math.log(radius[0]), math.log(radius[1])))
        ang = 2 * np.pi * np.arange(nk) / nk + rng.uniform(-0.3, 0.3, nk) * 2 * np.pi / nk
        rad = R * rng.uniform(0.6, 1.0, nk)
        xy = c + np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)   # increasing angle: positive winding
        col = rng.uniform(0.0, 1.0, channels)
        parts.append(dict(scene=scene, degree=p, flags=CLOSED | FILLED, key_xy=xy,
                          key_w=rng.uniform(0.5, 2.0, nk), key_s=np.ones(nk), tau=rng.uniform(0.5, 1.5, nk),
                          color=col, opacity=float(rng.uniform(0.5, 1.0))))
    return parts


def config3(seed=3000, n_paths=256, size=512):
    return _assemble(fills(seed, n_paths=n_paths, size=size), [[size, size]], [[1.0, 1.0, 1.0]], 3)


# ---------------------------------------------------------------------------------
# Long smoothing splines (config 4)
# ---------------------------------------------------------------------------------

def long_splines(seed, n_curves=16, n_cp=2000, size=1024, width=(1.0, 3.0), channels=1, scene=0) -> List[dict]:
    rng = np.random.default_rng(seed)
    parts = []
    lo, hi = 0.1953 * size, 0.8047 * size          # [200, 824] at 1024
    for _ in range(n_curves):
        pos = rng.uniform(lo, hi, 2)
        v = np.zeros(2)
        xy = np.zeros((n_cp, 2))
        for i in range(n_cp):
            xy[i] = pos
            v = 0.9 * v + rng.normal(0.0, 2.0, 2)
            pos = pos + v
            for a in range(2):                      # reflect at the canvas edge
                if pos[a] < 1.0:
                    pos[a] = 2.0 - pos[a]; v[a] = -v[a]
                if pos[a] > size - 1.0:
                    pos[a] = 2.0 * (size - 1.0) - pos[a]; v[a] = -v[a]
        w = rng.uniform(0.5, 2.0, n_cp)
        w[0] = 1.0
        parts.append(dict(scene=scene, degree=3, flags=0, key_xy=xy, key_w=w,
                          key_s=rng.uniform(width[0], width[1], n_cp), tau=_taus(rng, n_cp - 3),
                          color=np.zeros(channels), opacity=1.0))
    return parts


def config4(seed=4000, n_curves=16, n_cp=2000, size=1024):
    return _assemble(long_splines(seed, n_curves=n_curves, n_cp=n_cp, size=size), [[size, size]], [[1.0]], 1)


# ---------------------------------------------------------------------------------
# Many uneven scenes (config 5)
# ---------------------------------------------------------------------------------

def config5(seed=5000, n_scenes=64, sides=None, channels=3):
    """Scenes drawn from the stroke, fill and long-spline kinds, canvas sides
    128..1024 px, 4..256 paths (long splines capped at 16 curves of 150-600
    control points so that no scene exceeds ~2M Gaussians)."""
    rng = np.random.default_rng(seed)
    sides = list(range(128, 1025, 64)) if sides is None else sides
    parts, hw, bg, kinds = [], [], [], []
    for s in range(n_scenes):
        kind = int(rng.integers(0, 3))
        side = int(rng.choice(sides))
        sub = int(rng.integers(0, 2 ** 31 - 1))
        if kind == 0:
            n = int(rng.integers(4, 257))
            ps = strokes(sub, n_curves=n, size=side, step=8.0 * side / 256.0, nk_range=(12, 40),
                         channels=channels, scene=s)
        elif kind == 1:
            n = int(rng.integers(4, 257))
            ps = fills(sub, n_paths=n, size=side, radius=(5.0 * side / 512.0, 80.0 * side / 512.0),
                       channels=channels, scene=s)
        else:
            n = int(rng.integers(4, 17))
            ps = long_splines(sub, n_curves=n, n_cp=int(rng.integers(150, 601)), size=side,
                              channels=channels, scene=s)
            for p in ps:
                p["color"] = np.zeros(channels)
        parts += ps
        hw.append([side, side])
        bg.append(np.ones(channels))
        kinds.append(kind)
    b = _assemble(parts, hw, bg, channels)
    return b, kinds


# ---------------------------------------------------------------------------------
# Targets and perturbations
# ---------------------------------------------------------------------------------

def perturbed(b: CurveBatch, seed, pos=2.0, w=0.2, tau=0.1, width=0.1) -> CurveBatch:
    """Ground truth perturbed for the optimisation start: P + N(0, pos^2),
    w e^N(0, w^2), tau e^N(0, tau^2), width e^N(0, width^2)."""
    rng = np.random.default_rng(seed)
    o = b.copy()
    o.key_xy = (b.key_xy + rng.normal(0.0, pos, b.key_xy.shape)).astype(np.float32)
    o.key_w = (b.key_w * np.exp(rng.normal(0.0, w, b.key_w.shape))).astype(np.float32)
    o.tau = (b.tau * np.exp(rng.normal(0.0, tau, b.tau.shape))).astype(np.float32)
    o.key_s = (b.key_s * np.exp(rng.normal(0.0, width, b.key_s.shape))).astype(np.float32)
    return o


CONFIG_PARAMS = {
    1: dict(delta_c=1.5),
    2: dict(delta_c=3.0),
    3: dict(h=1.0),
    4: dict(delta_c=10.0),
    5: dict(delta_c=3.0, h=1.0),
}
