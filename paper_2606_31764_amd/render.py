"""PyTorch-facing wrapper of the NURBS Splatting C ABI.

Only argument marshalling lives here: every step of the render path and of
its adjoint runs in the HIP kernels of libnsplat.so.  PyTorch supplies device
memory and the current stream.  There is no CPU fallback: without the built
library or without a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_vp = ctypes.c_void_p


def _ptr(t: Optional[torch.Tensor]):
    return _vp(t.data_ptr()) if t is not None else None


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


@dataclasses.dataclass
class Params:
    """Method constants (Table S1 of the paper) and rasteriser settings."""
    delta_c: float = 10.0
    delta_b: float = 0.5
    rho: float = 2.0
    eta: float = 1.5
    gamma: float = 5.0
    nl_factor: float = 3.0
    fill_pad: float = 0.1
    h: float = 1.0
    k_sigma: float = 6.0
    alpha_max: float = 0.99
    eps_T: float = 1e-6
    delta_a: float = 0.25
    kappa: int = 4
    tile: int = 16
    batch: int = 64
    chunk: int = 0

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)

    def cstruct(self, h_dev: Optional[torch.Tensor] = None) -> L.Params:
        return L.Params(self.delta_c, self.delta_b, self.rho, self.eta, self.gamma, self.nl_factor, self.fill_pad,
                        self.h, self.k_sigma, self.alpha_max, self.eps_T, self.delta_a, int(self.kappa),
                        int(self.tile), int(self.batch), int(self.chunk), _ptr(h_dev))


class Context:
    """Owns one nsplat_ctx bound to a HIP device."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("nsplat needs a HIP device; none is visible")
        self.lib = L.load()
        self.device = device
        h = _vp()
        rc = self.lib.nsplat_create(ctypes.byref(h), device)
        self.h = h
        L.check(h, rc)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.nsplat_destroy(self.h)
        except Exception:
            pass

    def check(self, rc):
        return L.check(self.h, rc)


class Meta:
    """Device copies of the integer layout of a curve batch plus host sizes."""

    def __init__(self, batch, device="cuda"):
        dev = torch.device(device)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32), device=dev)
        self.scene = i32(batch.scene)
        self.degree = i32(batch.degree)
        self.flags = i32(batch.flags)
        self.key_off = i32(batch.key_off)
        self.tau_off = i32(batch.tau_off)
        self.hw_host = np.ascontiguousarray(batch.hw, np.int32)
        self.hw = i32(self.hw_host)
        self.bg = torch.as_tensor(np.ascontiguousarray(batch.bg, np.float32), device=dev)
        self.channels = int(batch.channels)
        self.n_curves = int(len(batch.degree))
        self.n_keys = int(batch.key_off[-1]) if self.n_curves else 0
        self.n_taus = int(batch.tau_off[-1]) if self.n_curves else 0
        # the degree bound handed to the library (0: its own maximum)
        self.max_degree = int(np.max(batch.degree)) if self.n_curves else 0
        self.any_flags = int(np.bitwise_or.reduce(np.asarray(batch.flags, np.int64))) if self.n_curves else 0
        self.all_flags = int(np.bitwise_and.reduce(np.asarray(batch.flags, np.int64))) if self.n_curves else 0
        if not 1 <= self.max_degree <= L.MAX_DEGREE:
            self.max_degree = 0
        self.n_scenes = int(len(self.hw_host))
        self.n_pixels = int(sum(int(h) * int(w) for h, w in self.hw_host))
        self.scenes_c = L.Scenes(self.n_scenes, _vp(self.hw_host.ctypes.data), _ptr(self.hw), _ptr(self.bg))

    def curves_c(self, key_xy, key_w, key_s, tau, color, opacity) -> L.Curves:
        return L.Curves(self.n_curves, self.channels, self.n_keys, self.n_taus, self.max_degree, self.any_flags,
                        self.all_flags,
                        _ptr(self.scene),
                        _ptr(self.degree),
                        _ptr(self.flags), _ptr(self.key_off), _ptr(self.tau_off), _ptr(key_xy), _ptr(key_w),
                        _ptr(key_s), _ptr(tau), _ptr(color), _ptr(opacity))

    def split_image(self, flat: torch.Tensor):
        out, off = [], 0
        for h, w in self.hw_host:
            n = self.channels * int(h) * int(w)
            out.append(flat[off:off + n].view(self.channels, int(h), int(w)))
            off += n
        return out


def param_tensors(batch, device="cuda", requires_grad=False):
    """FP32 device tensors (key_xy, key_w, key_s, tau, color, opacity)."""
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device).requires_grad_(requires_grad)
    return (f32(batch.key_xy), f32(batch.key_w), f32(batch.key_s), f32(batch.tau), f32(batch.color),
            f32(batch.opacity))


class Renderer:
    """One render state (plan, Gaussians, tile lists, workspace) for a curve
    batch of fixed layout.  A forward call must be followed by its backward
    before the next forward (the state is reused)."""

    def __init__(self, batch, params: Params = None, device: str = "cuda", caps=None, ctx: Context = None,
                 persistent: bool = False, h_dev: Optional[torch.Tensor] = None):
        self.ctx = ctx or Context(torch.device(device).index or 0)
        self.dev = torch.device(device)
        self.params = params or Params()
        self.meta = Meta(batch, device)
        self.persistent = bool(persistent)
        self.h_dev = h_dev
        # counts forward() calls: the adjoint reads the state the last forward
        # left (Gaussians, tile lists, T, n_last, checkpoints), so an autograd
        # node remembers the generation it was recorded at
        self.generation = 0
        self.caps = dict(gauss=4096, pairs=16384, boundary=1024) if caps is None else dict(caps)
        self.n_tiles_alloc = 0
        self._alloc()
        self.image = torch.empty(self.meta.channels * self.meta.n_pixels, device=self.dev)
        self.T = torch.empty(self.meta.n_pixels, device=self.dev)
        self.n_last = torch.empty(self.meta.n_pixels, dtype=torch.int32, device=self.dev)

    # -- buffers -------------------------------------------------------------------
    def _alloc(self):
        m, d = self.meta, self.dev
        self.plan = torch.zeros((max(m.n_curves, 1), L.PLAN_STRIDE), dtype=torch.int32, device=d)
        self.gauss = torch.empty((max(self.caps["gauss"], 1), 4), dtype=torch.float64, device=d)
        n_tiles = max(int(self.ctx.lib.nsplat_num_tiles(ctypes.byref(m.scenes_c), 8)), 1)
        self.n_tiles_alloc = n_tiles
        self.ranges = torch.zeros((n_tiles, 2), dtype=torch.int32, device=d)
        self.idx = torch.empty(max(self.caps["pairs"], 1), dtype=torch.int32, device=d)
        self.counters = torch.zeros(L.NUM_COUNTERS, dtype=torch.int32, device=d)
        self.caps_c = L.Caps(self.caps["gauss"], self.caps["pairs"], self.caps["boundary"])
        dummy = self.meta.curves_c(*[None] * 6)
        ws_bytes = int(self.ctx.lib.nsplat_workspace_size(ctypes.byref(dummy), ctypes.byref(m.scenes_c), None,
                                                          ctypes.byref(self.caps_c)))
        self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=d)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.bufs = L.Buffers(_ptr(self.plan), _ptr(self.gauss), _ptr(self.ranges), _ptr(self.idx),
                              _ptr(self.counters), _vp(self.ws_ptr), ws_bytes, self.caps_c)

    def grow(self, gauss=None, pairs=None, boundary=None):
        changed = False
        for k, v in (("gauss", gauss), ("pairs", pairs), ("boundary", boundary)):
            if v is not None and v > self.caps[k]:
                self.caps[k] = int(v * 1.25) + 1024
                changed = True
        if changed:
            plan = self.plan.clone()
            self._alloc()
            self.plan.copy_(plan)
        return changed

    def read_counters(self):
        out = (ctypes.c_int32 * L.NUM_COUNTERS)()
        self.ctx.check(self.ctx.lib.nsplat_read_counters(self.ctx.h, ctypes.byref(self.bufs), out, _stream()))
        return list(out)

    # -- the four steps --------------------------------------------------------------
    def _structs(self, tensors, params=None):
        p = params or self.params
        cv = self.meta.curves_c(*tensors)
        pr = p.cstruct(self.h_dev)
        return cv, pr

    def sample(self, tensors, frozen=False, sync=True, params=None):
        """nsplat_sample; with sync, returns the counters (a host synchronisation)."""
        cv, pr = self._structs(tensors, params)
        c = self.ctx
        c.check(c.lib.nsplat_sample(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c), ctypes.byref(pr),
                                    ctypes.byref(self.bufs), int(bool(frozen)), _stream()))
        return self.read_counters() if sync else None

    def bin(self, tensors, sync=True, params=None):
        """nsplat_bin; with sync, returns the counters (a host synchronisation)."""
        cv, pr = self._structs(tensors, params)
        c = self.ctx
        c.check(c.lib.nsplat_bin(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c), ctypes.byref(pr),
                                 ctypes.byref(self.bufs), _stream()))
        return self.read_counters() if sync else None

    def forward(self, tensors, params=None):
        cv, pr = self._structs(tensors, params)
        c = self.ctx
        self.generation += 1
        c.check(c.lib.nsplat_forward(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c), ctypes.byref(pr),
                                     ctypes.byref(self.bufs), _ptr(self.image), _ptr(self.T), _ptr(self.n_last),
                                     int(self.persistent), _stream()))
        return self.image

    def backward(self, tensors, dL: torch.Tensor, params=None, reg: "Reg" = None, grads=None, want=None):
        """Parameter gradients of the image loss (upstream dL) plus, with `reg`,
        the geometric regularisers (Eq. 11-12).  `grads` may pass preallocated
        output tensors (e.g. for graph capture); `want` (six booleans, default
        all) selects the groups to compute; a group not wanted is returned as
        None and the library leaves it out."""
        cv, pr = self._structs(tensors, params)
        if grads is None:
            grads = [torch.empty_like(t) if w else None for t, w in zip(tensors, want or (True,) * 6)]
        gc = L.Grads(*[_ptr(g) for g in grads])
        c = self.ctx
        dL = dL.contiguous()
        if reg is None:
            c.check(c.lib.nsplat_backward(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c),
                                          ctypes.byref(pr), ctypes.byref(self.bufs), _ptr(dL), _ptr(self.T),
                                          _ptr(self.n_last), ctypes.byref(gc), int(self.persistent), _stream()))
        else:
            rc = reg.struct()
            c.check(c.lib.nsplat_backward_reg(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c),
                                              ctypes.byref(pr), ctypes.byref(self.bufs), _ptr(dL), _ptr(self.T),
                                              _ptr(self.n_last), ctypes.byref(rc), ctypes.byref(gc),
                                              int(self.persistent), _stream()))
        return grads

    def udf_loss(self, tensors, image: torch.Tensor, target: torch.Tensor, tau: float, sel=None, loss=None,
                 params=None, out=None, noalloc=False):
        """dL/dImage of the distance-weighted image loss (LIVE's unsigned-distance
        weights around the selected filled curves; sel: device int32 [n_curves] or
        None for every filled curve) for this step's boundaries; the loss value
        is added to `loss` (device [1]) when given.  noalloc selects
        nsplat_udf_loss_noalloc (scratch in the library's static device array)."""
        cv, pr = self._structs(tensors, params)
        dL = torch.empty_like(image) if out is None else out
        c = self.ctx
        fn = c.lib.nsplat_udf_loss_noalloc if noalloc else c.lib.nsplat_udf_loss
        c.check(fn(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c), ctypes.byref(pr),
                                      ctypes.byref(self.bufs), _ptr(sel), float(tau), _ptr(image.contiguous()),
                                      _ptr(target.contiguous()), _ptr(dL), _ptr(loss), _stream()))
        return dL

    def run_forward(self, tensors, frozen=False, sync=True, params=None):
        """sample -> bin -> forward.  With sync, any capacity overflow grows the
        buffers and re-runs from sampling (growing reallocates the workspace)."""
        if not sync:
            self.sample(tensors, frozen=frozen, sync=False, params=params)
            self.bin(tensors, sync=False, params=params)
            return self.forward(tensors, params=params)
        for _ in range(4):
            cnt = self.sample(tensors, frozen=frozen, params=params)
            if self.grow(gauss=cnt[L.CNT_GAUSS_REQ], boundary=cnt[L.CNT_BOUND_REQ]):
                continue
            cnt = self.bin(tensors, params=params)
            if self.grow(pairs=cnt[L.CNT_PAIRS_REQ]):
                continue
            return self.forward(tensors, params=params)
        raise RuntimeError("nsplat: buffers kept overflowing")

    def autotune(self, tensors, dL):
        cv, pr = self._structs(tensors)
        grads = [torch.empty_like(t) for t in tensors]
        gc = L.Grads(*[_ptr(g) for g in grads])
        bt, bb = ctypes.c_int32(), ctypes.c_int32()
        times = (ctypes.c_float * 12)()
        c = self.ctx
        c.check(c.lib.nsplat_autotune(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c), ctypes.byref(pr),
                                      ctypes.byref(self.bufs), _ptr(self.image), _ptr(self.T), _ptr(self.n_last),
                                      _ptr(dL.contiguous()), ctypes.byref(gc), int(self.persistent),
                                      ctypes.byref(bt), ctypes.byref(bb), times, _stream()))
        return int(bt.value), int(bb.value), list(times)

    # -- views for tests ------------------------------------------------------------------
    def gaussians(self):
        """Records as numpy: dict(mu [G,2] f64, sigma, opacity (f32), curve, local (i32))."""
        G = self.read_counters()[L.CNT_GAUSS]
        raw = self.gauss[:G].cpu().numpy()
        u8 = raw.view(np.uint8).reshape(G, 32)
        return dict(mu=raw[:, :2].copy(), sigma=u8[:, 16:20].copy().view(np.float32)[:, 0],
                    opacity=u8[:, 20:24].copy().view(np.float32)[:, 0], curve=u8[:, 24:28].copy().view(np.int32)[:, 0],
                    local=u8[:, 28:32].copy().view(np.int32)[:, 0])

    def gauss_frame(self, tensors):
        """Tangent and cross-axis width of the tangent-aligned stroke Gaussians
        of the last sample: dict(tdir [G,2], sp [G], ratio [G]) as numpy (FP32);
        rows of other kinds are unspecified."""
        G = self.read_counters()[L.CNT_GAUSS]
        out = torch.empty((max(G, 1), 4), dtype=torch.float32, device=self.gauss.device)
        cv = self.meta.curves_c(*tensors)
        c = self.ctx
        c.check(c.lib.nsplat_gauss_frame(c.h, ctypes.byref(cv), ctypes.byref(self.meta.scenes_c),
                                         ctypes.byref(self.bufs), _ptr(out), int(G), _stream()))
        a = out[:G].cpu().numpy()
        return dict(tdir=a[:, :2].copy(), sp=a[:, 2].copy(), ratio=a[:, 3].copy())

    def tiles(self, tile=None):
        tile = tile or self.params.tile
        n_tiles = int(self.ctx.lib.nsplat_num_tiles(ctypes.byref(self.meta.scenes_c), int(tile)))
        P = self.read_counters()[L.CNT_PAIRS]
        return self.ranges[:n_tiles].cpu().numpy(), self.idx[:P].cpu().numpy()

    def plan_np(self):
        return self.plan[:self.meta.n_curves].cpu().numpy()


class NSplatFunction(torch.autograd.Function):
    """image = render(key_xy, key_w, key_s, tau, color, opacity); the backward
    runs the library's adjoint.  The adjoint reads the Renderer's state from
    the forward that recorded this node, so the backward raises if the same
    Renderer has run another forward since.  Inputs that need no gradient
    (e.g. weights or knot intervals held fixed, the ablations of Table 1) get
    None, and the library does not write them."""

    @staticmethod
    def forward(ctx, key_xy, key_w, key_s, tau, color, opacity, renderer: Renderer, frozen: bool, sync: bool):
        tensors = tuple(t.detach().contiguous() for t in (key_xy, key_w, key_s, tau, color, opacity))
        img = renderer.run_forward(tensors, frozen=frozen, sync=sync)
        ctx.renderer = renderer
        ctx.tensors = tensors
        ctx.generation = renderer.generation
        return img.clone()

    @staticmethod
    def backward(ctx, grad_img):
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("nsplat: this Renderer has run another forward since the one this backward belongs "
                               "to; its state (Gaussians, tile lists, per-pixel state) no longer matches")
        want = tuple(bool(x) for x in ctx.needs_input_grad[:6])
        if not any(want):
            return (None,) * 9
        grads = r.backward(ctx.tensors, grad_img, want=want)
        return (*grads, None, None, None)


@dataclasses.dataclass
class Reg:
    """Geometric regularisers of Sec. 3.5 for Renderer.backward: bounding-box
    penalty (Eq. 12; kind 0 ReLU, 1 softplus; bbox [S][4] device tensor or None
    for the canvas) and derivative loss of order r (Eq. 11).  `loss` (device
    [2]) accumulates the two values."""
    bbox_weight: float = 0.0
    bbox_kind: int = 0
    bbox: Optional[torch.Tensor] = None
    deriv_weight: float = 0.0
    deriv_order: int = 3
    loss: Optional[torch.Tensor] = None

    def struct(self):
        return L.Reg(float(self.bbox_weight), int(self.bbox_kind),
                     _ptr(self.bbox) if self.bbox is not None else None, float(self.deriv_weight),
                     int(self.deriv_order), _ptr(self.loss) if self.loss is not None else None)


class Adam:
    """Device Adam over the six parameter groups with the supplementary
    settings: per-group learning rates (key_xy, key_w, key_s, tau, color,
    opacity), cosine decay to final_ratio over total_steps, clamps w in
    [0.01, 10] and tau in [0, 2].  The step counter lives on the device, so a
    captured graph advances it."""

    def __init__(self, tensors, lr=(1.5, 0.1, 0.2, 0.1, 0.01, 0.01), betas=(0.9, 0.999), eps=1e-8,
                 total_steps=1000, final_ratio=0.1, w_range=(0.01, 10.0), tau_range=(0.0, 2.0), ctx=None):
        self.ctx = ctx or Context(tensors[0].device.index or 0)
        self.tensors = tensors
        n = sum(t.numel() for t in tensors)
        self.m = torch.zeros(n, device=tensors[0].device)
        self.v = torch.zeros(n, device=tensors[0].device)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=tensors[0].device)
        self.cfg = L.Adam((ctypes.c_float * 6)(*lr), betas[0], betas[1], eps, final_ratio, int(total_steps),
                          w_range[0], w_range[1], tau_range[0], tau_range[1])
        key_xy, key_w, key_s, tau, color, opacity = tensors
        self.vals = L.Values(int(opacity.numel()), int(color.numel() // max(opacity.numel(), 1)),
                             int(key_w.numel()), int(tau.numel()), *[_ptr(t) for t in tensors])

    def step(self, grads):
        gc = L.Grads(*[_ptr(g) for g in grads])
        c = self.ctx
        c.check(c.lib.nsplat_adam_step(c.h, ctypes.byref(self.cfg), ctypes.byref(self.vals), ctypes.byref(gc),
                                       _ptr(self.m), _ptr(self.v), _ptr(self.step_dev), _stream()))


def render(renderer: Renderer, key_xy, key_w, key_s, tau, color, opacity, frozen=False, sync=True):
    """Differentiable render of all scenes; returns the flat image (per scene [C][H][W] concatenated)."""
    return NSplatFunction.apply(key_xy, key_w, key_s, tau, color, opacity, renderer, frozen, sync)
