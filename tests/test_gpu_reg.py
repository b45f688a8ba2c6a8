"""Geometric regularisers (Sec. 3.5: derivative loss Eq. 11, bounding-box
loss Eq. 12) in the backward pass, and the device Adam step, against the FP64
oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from helpers import PARAM_NAMES, grad_check_fp64, grad_close, oracle_params
from paper_2606_31764_amd import synth
from paper_2606_31764_amd.render import Params

pytestmark = pytest.mark.gpu


def _gpu_reg(b, p, reg_kw, box=None):
    """GPU gradients and loss values of the regularisers alone (zero image gradient)."""
    import torch
    from paper_2606_31764_amd.render import Reg, Renderer, param_tensors
    r = Renderer(b, p)
    t = param_tensors(b)
    img = r.run_forward(t)
    loss = torch.zeros(2, device="cuda")
    bb = None if box is None else torch.as_tensor(np.asarray(box, np.float32), device="cuda")
    reg = Reg(loss=loss, bbox=bb, **reg_kw)
    grads = r.backward(t, torch.zeros_like(img), reg=reg)
    torch.cuda.synchronize()
    g = {n: x.cpu().numpy().astype(np.float64) for n, x in zip(PARAM_NAMES, grads)}
    return g, loss.cpu().numpy().astype(np.float64)


def _oracle_reg(b, p, reg_kw, box=None):
    op = oracle_params(p)
    plan, _, _ = oracle.plan(b, op)
    kw = dict(reg_kw)
    if box is not None:
        kw["bbox"] = np.asarray(box, np.float64)
    return oracle.reg_loss_grad(b, plan, op, **kw)


def _check(b, p, reg_kw, box=None, loss_rtol=2e-5):
    g, loss = _gpu_reg(b, p, reg_kw, box)
    v, gref = _oracle_reg(b, p, reg_kw, box)
    worst, rep = grad_check_fp64(g, gref)
    assert worst <= 1.0, rep
    assert abs(loss.sum() - v) <= loss_rtol * abs(v) + 1e-6, (loss, v)
    return g, gref


def _strokes(seed, n=4, size=96, degrees=(3,)):
    b = synth.config2(seed=seed, n_curves=n, size=size)
    rng = np.random.default_rng(seed)
    b.degree = np.asarray(rng.choice(degrees, len(b.degree)), np.int32)
    # open curves need n_k - p intervals
    parts = []
    for c in range(b.n_curves):
        k0, k1 = b.key_off[c], b.key_off[c + 1]
        p_ = int(b.degree[c])
        parts.append(dict(scene=0, degree=p_, flags=0, key_xy=b.key_xy[k0:k1], key_w=b.key_w[k0:k1],
                          key_s=b.key_s[k0:k1], tau=rng.uniform(0.5, 1.5, (k1 - k0) - p_), color=b.color[c],
                          opacity=float(b.opacity[c])))
    return synth._assemble(parts, [[size, size]], [[1, 1, 1]], 3)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_derivative_loss_strokes(order):
    b = _strokes(5100 + order, degrees=(2, 3, 5))
    _check(b, Params().replace(delta_c=1.0), dict(deriv_weight=0.7, deriv_order=order))


def test_derivative_loss_closed_strokes_and_fills():
    rng = np.random.default_rng(5200)
    parts = []
    for k, p_ in enumerate((2, 3, 4)):
        nk = 7 + k
        ang = np.sort(rng.uniform(0, 2 * np.pi, nk))
        xy = np.stack([48 + 20 * np.cos(ang), 48 + 18 * np.sin(ang)], 1)
        parts.append(dict(scene=0, degree=p_, flags=synth.CLOSED | (synth.FILLED if k == 1 else 0), key_xy=xy,
                          key_w=rng.uniform(0.5, 2.0, nk), key_s=rng.uniform(1, 3, nk),
                          tau=rng.uniform(0.5, 1.5, nk), color=rng.uniform(0, 1, 3), opacity=0.8))
    b = synth._assemble(parts, [[96, 96]], [[1, 1, 1]], 3)
    _check(b, Params().replace(delta_c=1.0, h=2.0), dict(deriv_weight=1.3, deriv_order=3))


@pytest.mark.parametrize("kind", [0, 1])
def test_bbox_loss_strokes_and_fills(kind):
    b1 = _strokes(5300, n=3, size=80)
    b1.key_xy = b1.key_xy + np.array([50.0, -25.0], np.float32)      # partly outside the canvas
    b2 = synth.config3(seed=5301, n_paths=3, size=80)
    b2.key_xy = (b2.key_xy * 1.4 - 10.0).astype(np.float32)
    b2.scene[:] = 0
    b = synth.concat([b1, b2])
    _check(b, Params().replace(delta_c=1.0, h=2.0), dict(bbox_weight=2.0, bbox_kind=kind))


def test_bbox_custom_boxes_in_a_batch_and_both_terms():
    b = synth.concat([_strokes(5400, n=3, size=64), synth.config3(seed=5401, n_paths=3, size=72)])
    box = [[5.0, 5.0, 50.0, 60.0], [10.0, 0.0, 72.0, 40.0]]
    _check(b, Params().replace(delta_c=1.0, h=2.0),
           dict(bbox_weight=1.0, bbox_kind=1, deriv_weight=0.5, deriv_order=3), box=box)


def test_reg_adds_to_the_image_gradient():
    """backward with regularisers = image-only backward + regulariser-only backward."""
    import torch
    from paper_2606_31764_amd.render import Reg, Renderer, param_tensors
    b = _strokes(5500, n=4, size=96)
    b.key_xy = b.key_xy + np.array([30.0, 0.0], np.float32)
    p = Params().replace(delta_c=1.0)
    r = Renderer(b, p)
    t = param_tensors(b)
    img = r.run_forward(t).clone()
    dL = 2.0 * (img - 0.5)
    reg = dict(bbox_weight=1.0, bbox_kind=0, deriv_weight=0.2, deriv_order=3)
    g_img = r.backward(t, dL)
    g_reg = r.backward(t, torch.zeros_like(dL), reg=Reg(**reg))
    g_all = r.backward(t, dL, reg=Reg(**reg))
    torch.cuda.synchronize()
    a = {n: x.cpu().numpy().astype(np.float64) for n, x in zip(PARAM_NAMES, g_all)}
    s = {n: (x.cpu().numpy().astype(np.float64) + y.cpu().numpy().astype(np.float64))
         for n, x, y in zip(PARAM_NAMES, g_img, g_reg)}
    assert grad_close(a, s, rtol=1e-5, atol=1e-6) <= 1.0


def test_adam_step_matches_oracle():
    import torch
    from paper_2606_31764_amd.render import Adam, param_tensors
    b = synth.concat([_strokes(5600, n=3, size=64), synth.config3(seed=5601, n_paths=3, size=64)])
    t = list(param_tensors(b))
    gen0 = torch.Generator(device="cuda").manual_seed(2)
    t[1].uniform_(0.005, 10.5, generator=gen0)      # weights near and beyond the clamp range
    t[3].uniform_(-0.1, 2.1, generator=gen0)
    lr = (1.5, 0.1, 0.2, 0.1, 0.01, 0.01)
    opt = Adam(t, lr=lr, total_steps=7, final_ratio=0.1)
    x = {n: a.detach().cpu().numpy().astype(np.float64) for n, a in zip(oracle.GROUPS, t)}
    m = {n: np.zeros_like(a) for n, a in x.items()}
    v = {n: np.zeros_like(a) for n, a in x.items()}
    gen = torch.Generator(device="cuda").manual_seed(3)
    for step in range(1, 10):
        grads = [torch.randn(a.shape, device="cuda", generator=gen) for a in t]
        opt.step(grads)
        g = {n: a.cpu().numpy().astype(np.float64) for n, a in zip(oracle.GROUPS, grads)}
        oracle.adam_step(x, g, m, v, step, lr, total=7, final_ratio=0.1)
        torch.cuda.synchronize()
        for n, a in zip(oracle.GROUPS, t):
            got = a.cpu().numpy().astype(np.float64)
            assert np.abs(got - x[n]).max() <= 2e-5 * (1.0 + np.abs(x[n]).max()), (n, step)
    assert int(opt.step_dev.item()) == 9
    # the clamps hold in FP32 (0.01 is not representable: its FP32 rounding is the bound)
    assert t[1].min().item() >= float(np.float32(0.01)) and t[1].max().item() <= 10.0
    assert t[3].min().item() >= 0.0 and t[3].max().item() <= 2.0


def test_full_step_in_a_graph():
    """sample -> bin -> forward -> L2 -> backward with regularisers -> Adam captured
    once and replayed: every replay matches the same step run eagerly from the
    same parameters."""
    import torch
    from paper_2606_31764_amd.render import Adam, Reg, Renderer, param_tensors
    b = synth.concat([_strokes(5700, n=3, size=64), synth.config3(seed=5701, n_paths=3, size=64)])
    p = Params().replace(delta_c=1.0, h=2.0)
    t_ref = [x.clone() for x in param_tensors(b)]
    sizer = Renderer(b, p)
    sizer.run_forward(t_ref)
    cnt = sizer.read_counters()
    caps = dict(gauss=int(cnt[3] * 1.5) + 256, pairs=int(cnt[4] * 1.5) + 1024, boundary=int(cnt[5] * 1.5) + 64)
    # two 64 x 64 scenes: the target and dL cover every pixel of both
    n_img = 3 * sum(int(h) * int(w) for h, w in b.hw)
    assert n_img == sizer.image.numel()
    target = torch.full((n_img,), 0.7, device="cuda")

    def make():
        t = [x.clone() for x in t_ref]
        r = Renderer(b, p, caps=caps)
        # eps = 1 keeps the update linear in small gradients, so that the FP32
        # atomic order (which differs between runs) cannot flip a noise-level step
        opt = Adam(t, total_steps=20, eps=1.0)
        dL = torch.empty_like(target)
        grads = [torch.empty_like(x) for x in t]
        reg = Reg(bbox_weight=1.0, bbox_kind=1, deriv_weight=0.1, deriv_order=3)
        lib, h = r.ctx.lib, r.ctx.h

        def step():
            img = r.run_forward(t, sync=False)
            assert img.numel() == target.numel() == dL.numel()
            import ctypes
            r.ctx.check(lib.nsplat_l2_grad(h, ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                           ctypes.c_void_p(dL.data_ptr()), None, img.numel(),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
            r.backward(t, dL, reg=reg, grads=grads)
            opt.step(grads)
        return t, step

    t_e, step_e = make()
    t_g, step_g = make()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step_g()            # warm-up eager step (also advances t_g once)
    torch.cuda.current_stream().wait_stream(s)
    step_e()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step_g()
    for k in range(3):
        graph.replay()
        step_e()
        torch.cuda.synchronize()
        for a, e in zip(t_g, t_e):
            d = (a - e).abs().max().item()
            assert d <= 1e-4 * (1.0 + e.abs().max().item()), (k, d)
        _ = (torch.randn(100, device="cuda") * 3).sum().item()


@pytest.mark.parametrize("selected", [False, True])
def test_udf_loss_matches_oracle(selected):
    import torch
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.concat([synth.config3(seed=6000, n_paths=5, size=72),
                      synth.config2(seed=6001, n_curves=2, size=40), synth.config3(seed=6002, n_paths=3, size=48)])
    p = Params().replace(delta_c=2.0, h=2.0)
    r = Renderer(b, p)
    t = param_tensors(b)
    img = r.run_forward(t).clone()
    rng = np.random.default_rng(6003)
    tgt = torch.as_tensor(rng.uniform(0, 1, img.numel()).astype(np.float32), device="cuda")
    sel_np = (rng.uniform(size=b.n_curves) < 0.5).astype(np.int32) if selected else None
    sel = None if sel_np is None else torch.as_tensor(sel_np, device="cuda")
    loss = torch.zeros(1, device="cuda")
    dL = r.udf_loss(t, img, tgt, tau=8.0, sel=sel, loss=loss)
    torch.cuda.synchronize()
    op = oracle_params(p)
    plan, _, _ = oracle.plan(b, op)
    v, dref, _ = oracle.udf_loss(b, plan, img.cpu().numpy(), tgt.cpu().numpy(), 8.0, sel=sel_np, params=op)
    got = dL.cpu().numpy().astype(np.float64)
    assert np.abs(got - dref).max() <= 1e-5 * np.abs(dref).max() + 1e-12
    assert abs(float(loss.item()) - v) <= 1e-5 * abs(v) + 1e-9
