"""Edge cases of the GPU path, each against the oracle or an exact property."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from helpers import (IMG_TOL, grad_check, grad_close, grad_report, gpu_run, gpu_vs_oracle, oracle_params,
                     oracle_plan, oracle_reference, plans_equal)
from paper_2606_31764_amd import synth
from paper_2606_31764_amd.render import Params

pytestmark = pytest.mark.gpu

R2 = math.sqrt(2.0) / 2.0


def _batch(parts, hw=(48, 40), bg=(1.0, 1.0, 1.0), channels=3):
    return synth._assemble(parts, [list(hw)], [list(bg)], channels)


def _part(xy, p=3, closed=False, filled=False, w=None, s=None, tau=None, color=(0.2, 0.4, 0.6), o=0.8, seed=0):
    rng = np.random.default_rng(seed)
    xy = np.asarray(xy, float)
    nk = len(xy)
    nt = nk if closed else nk - p
    return dict(scene=0, degree=p, flags=(synth.CLOSED if closed else 0) | (synth.FILLED if filled else 0),
                key_xy=xy, key_w=rng.uniform(0.5, 2.0, nk) if w is None else np.asarray(w, float),
                key_s=rng.uniform(1.0, 3.0, nk) if s is None else np.asarray(s, float),
                tau=rng.uniform(0.5, 1.5, nt) if tau is None else np.asarray(tau, float), color=color, opacity=o)


def _full_parity(b, p, target_seed=5):
    op = oracle_params(p)
    tb = synth.perturbed(b, seed=target_seed)
    target = oracle.render(tb, op)[0]
    out, _, _ = gpu_vs_oracle(b, p, target)
    ref_g = oracle.gaussians(b, op)
    plans_equal(out["plan"], ref_g["plan"])
    return out


def test_no_curves_gives_background():
    b = synth._assemble([], [[20, 30]], [[0.25, 0.5, 0.75]], 3)
    out = gpu_run(b, Params(), target=np.zeros(3 * 20 * 30, np.float32))
    img = out["image"].reshape(3, 20, 30)
    for c, v in enumerate((0.25, 0.5, 0.75)):
        assert np.all(img[c] == np.float32(v))
    assert out["counters"][0] == 0 and out["counters"][1] == 0
    assert all(g.size == 0 for g in out["grads"].values())


def test_scene_without_curves_inside_a_batch():
    b1 = synth.config2(seed=2601, n_curves=3, size=40)
    empty = synth._assemble([], [[24, 24]], [[1.0, 1.0, 1.0]], 3)
    b = synth.concat([b1, empty, synth.config2(seed=2602, n_curves=2, size=36)])
    p = Params().replace(delta_c=2.0)
    op = oracle_params(p)
    out = gpu_run(b, p, backward=False)
    img_ref, _, _ = oracle.render(b, op)
    assert np.abs(out["image"] - img_ref).max() <= IMG_TOL
    off = 3 * 40 * 40
    assert np.all(out["image"][off:off + 3 * 24 * 24] == 1.0)


def test_curve_outside_the_canvas():
    b = _batch([_part([[200, 200], [210, 205], [220, 200], [230, 210]])])
    out = gpu_run(b, Params(), target=np.zeros(3 * 48 * 40, np.float32))
    assert out["counters"][1] == 0
    assert np.all(out["image"] == 1.0)
    for n, g in out["grads"].items():
        assert np.all(g == 0.0), n


def test_degenerate_point_curve():
    b = _batch([_part([[20.3, 17.6]] * 5, p=3)])
    out = _full_parity(b, Params().replace(delta_c=2.0))
    assert out["plan"][0, 1] == 2          # M = max(2, ceil(0))


def test_repeated_knots_nine_point_circle_stroke():
    c, r = np.array([24.0, 20.0]), 12.0
    P = c + r * np.array([(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0)], float)
    w = [1, R2, 1, R2, 1, R2, 1, R2, 1]
    b = _batch([_part(P, p=2, w=w, s=np.full(9, 2.0), tau=[0.25, 0, 0.25, 0, 0.25, 0, 0.25])])
    p = Params().replace(delta_c=2.0)
    out = _full_parity(b, p)
    mu = out["gauss"]["mu"]
    ref = oracle.gaussians(b, oracle_params(p))["mu"]
    assert np.abs(mu - ref).max() < 1e-9
    # FP32-stored weights (sqrt(2)/2 rounded) keep the circle to ~1e-7 of r
    assert np.abs(np.hypot(mu[:, 0] - c[0], mu[:, 1] - c[1]) - r).max() < 1e-6


def test_all_degrees_open_and_closed_strokes():
    rng = np.random.default_rng(3)
    parts = []
    for p in range(1, 6):
        parts.append(_part(rng.uniform(5, 43, (p + 4, 2)), p=p, seed=p, color=rng.uniform(0, 1, 3)))
        parts.append(_part(rng.uniform(5, 43, (p + 3, 2)), p=p, closed=True, seed=10 + p,
                           color=rng.uniform(0, 1, 3)))
    b = _batch(parts, hw=(48, 48))
    _full_parity(b, Params().replace(delta_c=2.0))


def test_invalid_curves_set_status_and_are_skipped():
    good = _part([[5, 5], [20, 30], [35, 10], [40, 40]], p=3)
    bad = [
        dict(_part([[5, 5], [20, 30], [35, 10], [40, 40]], p=3), degree=6),   # degree too high
        _part([[5, 5], [20, 30]], p=3, tau=[1.0]),                            # too few key points
        _part([[5, 5], [20, 30], [35, 10], [40, 40]], p=3, filled=True),      # filled but open
    ]
    for b_ in bad:
        b_["tau"] = np.asarray(b_["tau"], float)
    b = _batch([good] + bad)
    out = gpu_run(b, Params().replace(delta_c=2.0), backward=False)
    assert out["counters"][2] & 8           # NSPLAT_STATUS_DATA
    assert np.all(out["plan"][1:, 0] == 0)
    ref = gpu_run(_batch([good]), Params().replace(delta_c=2.0), backward=False)
    np.testing.assert_array_equal(out["image"], ref["image"])


def test_declared_degree_bound_rejects_higher_degrees():
    # a batch that declares degree <= 3 but holds a degree-4 curve: that curve
    # is invalid data (no Gaussians, status bit), the rest renders and
    # differentiates as without it, through the degree-3 adjoint kernels
    import torch
    from paper_2606_31764_amd.render import Renderer, param_tensors
    rng = np.random.default_rng(41)
    good = [_part(rng.uniform(6, 42, (6, 2)), p=3, seed=1, color=(0.9, 0.2, 0.1)),
            _part(rng.uniform(6, 42, (5, 2)), p=2, closed=True, seed=2, color=(0.1, 0.3, 0.8))]
    high = _part(rng.uniform(6, 42, (7, 2)), p=4, seed=3)
    p = Params().replace(delta_c=2.0)
    b_good = _batch(good)
    b_all = _batch(good + [high])
    op = oracle_params(p)
    target = oracle.render(synth.perturbed(b_good, seed=8), op)[0]
    r = Renderer(b_all, p)
    assert r.meta.max_degree == 4
    r.meta.max_degree = 3
    t = param_tensors(b_all)
    img = r.run_forward(t).clone()
    counters = r.read_counters()
    plan = r.plan_np()
    assert counters[2] & 8  # NSPLAT_STATUS_DATA
    assert plan[2, 0] == 0 and plan[0, 0] > 0 and plan[1, 0] > 0
    img_ref, up, gref, scale = oracle_reference(b_good, target, op)
    assert np.abs(img.cpu().numpy() - img_ref).max() <= IMG_TOL
    grads = r.backward(t, torch.as_tensor(up.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    from helpers import PARAM_NAMES
    g = {n: x.cpu().numpy().astype(np.float64) for n, x in zip(PARAM_NAMES, grads)}
    nk, nt = int(b_good.key_off[-1]), int(b_good.tau_off[-1])
    cut = dict(key_xy=2 * nk, key_w=nk, key_s=nk, tau=nt, color=3 * len(good), opacity=len(good))
    mine = {n: g[n].ravel()[:cut[n]] for n in PARAM_NAMES}
    worst, rep = grad_check(mine, gref, scale)
    assert worst <= 1.0, rep
    for n in PARAM_NAMES:
        assert np.all(g[n].ravel()[cut[n]:] == 0.0), n


def test_capacity_growth_gives_same_result():
    b = synth.config3(seed=3700, n_paths=5, size=64)
    p = Params().replace(h=2.0)
    a = gpu_run(b, p, backward=False, caps=dict(gauss=16, pairs=16, boundary=8))
    c = gpu_run(b, p, backward=False, caps=dict(gauss=1 << 16, pairs=1 << 18, boundary=1 << 12))
    np.testing.assert_array_equal(a["image"], c["image"])
    np.testing.assert_array_equal(a["idx"], c["idx"])


def test_frozen_plan_keeps_counts():
    import torch
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.config3(seed=3800, n_paths=4, size=64)
    p = Params().replace(h=2.0)
    r = Renderer(b, p)
    t = param_tensors(b)
    r.run_forward(t)
    plan0 = r.plan_np().copy()
    b2 = b.copy()
    b2.key_xy = b.key_xy * 1.03          # would change arc lengths and windows
    t2 = param_tensors(b2)
    r.run_forward(t2, frozen=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.plan_np()[:, :7], plan0[:, :7])
    ref = oracle.gaussians(b2, oracle_params(p), frozen_plan=oracle_plan(plan0))
    g = r.gaussians()
    assert np.abs(g["mu"] - ref["mu"]).max() < 1e-9
    assert np.abs(g["opacity"] - ref["opacity"]).max() < 2e-7


def test_device_annealing_matches_eq14():
    import ctypes
    import torch
    from paper_2606_31764_amd.render import Context
    ctx = Context(0)
    h = torch.zeros(1, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    vals = []
    for t in range(0, 1001, 50):
        ctx.check(ctx.lib.nsplat_anneal_h(ctx.h, ctypes.c_void_p(h.data_ptr()), None, t, 1000, 8.0, 1.0, 0.1, 0.8,
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        vals.append((t, float(h.item())))
    for t, v in vals:
        assert v == np.float32(oracle.anneal(t, 1000, 8.0, 1.0, np.float32(0.1), np.float32(0.8)))
    # device step counter form: reads and increments the counter
    for t in range(3):
        ctx.check(ctx.lib.nsplat_anneal_h(ctx.h, ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(step.data_ptr()), 0,
                                          1000, 8.0, 1.0, 0.1, 0.8,
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    assert int(step.item()) == 3


@pytest.mark.parametrize("name", ["strokes", "fills"])
def test_tile_sizes_agree(name):
    if name == "strokes":
        b, p = synth.config2(seed=2700, n_curves=6, size=72), Params().replace(delta_c=2.0)
    else:
        b, p = synth.config3(seed=3900, n_paths=6, size=72), Params().replace(h=2.0)
    target = oracle.render(synth.perturbed(b, seed=1), oracle_params(p))[0]
    outs = {t: gpu_run(b, p.replace(tile=t), target=target) for t in (8, 16, 32)}
    for t in (8, 32):
        assert np.abs(outs[t]["image"] - outs[16]["image"]).max() < 2e-6
        assert grad_close(outs[t]["grads"], outs[16]["grads"], rtol=2e-5, atol=1e-7) <= 1.0


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_batch_depths_agree(tile):
    """The per-pixel order of operations does not depend on the batch depth,
    so images are bit-identical across depths; gradients agree up to the
    order of FP32 atomics."""
    b, p = synth.config3(seed=3950, n_paths=8, size=88), Params().replace(h=2.0, tile=tile)
    target = oracle.render(synth.perturbed(b, seed=2), oracle_params(p))[0]
    outs = {d: gpu_run(b, p.replace(batch=d), target=target) for d in (32, 64, 128, 256)}
    for d in (32, 128, 256):
        np.testing.assert_array_equal(outs[d]["image"], outs[64]["image"])
        np.testing.assert_array_equal(outs[d]["n_last"], outs[64]["n_last"])
        assert grad_close(outs[d]["grads"], outs[64]["grads"], rtol=1e-5, atol=1e-7) <= 1.0


def test_capacity_overflow_without_growth_is_flagged_and_consistent():
    """A step that overflows the Gaussian capacity with no host check in between
    (as inside a captured graph) sets the status bit and still leaves every record
    below the cap written (the fill lattice then goes row-major), so the later
    kernels of the step read only valid records."""
    import torch
    from paper_2606_31764_amd import _lib as Lb
    from paper_2606_31764_amd.render import Reg, Renderer, param_tensors
    b = synth.concat([synth.config2(seed=2900, n_curves=3, size=64), synth.config3(seed=2901, n_paths=4, size=64)])
    p = Params().replace(delta_c=2.0, h=2.0)
    sizer = Renderer(b, p)
    t = param_tensors(b)
    sizer.run_forward(t)
    cnt = sizer.read_counters()
    G_full = cnt[Lb.CNT_GAUSS]
    caps = dict(gauss=G_full // 2, pairs=4 * cnt[Lb.CNT_PAIRS] + 1024, boundary=2 * cnt[Lb.CNT_BOUND_REQ] + 64)
    r = Renderer(b, p, caps=caps)
    r.sample(t, sync=False)
    r.bin(t, sync=False)
    img = r.forward(t)
    grads = r.backward(t, 2.0 * (img - 0.5), reg=Reg(bbox_weight=1.0, deriv_weight=0.1))
    torch.cuda.synchronize()
    cnt2 = r.read_counters()
    assert cnt2[Lb.CNT_STATUS] & Lb.STATUS_GAUSS_CAP
    assert cnt2[Lb.CNT_GAUSS] == caps["gauss"] and cnt2[Lb.CNT_GAUSS_REQ] == G_full
    rec = r.gaussians()
    plan = r.plan_np()
    assert np.all((rec["curve"] >= 0) & (rec["curve"] < b.n_curves))
    assert np.all(rec["local"] >= 0) and np.all(rec["local"] < plan[rec["curve"], 0])
    # the records below the cap are exactly the full run's first records
    ref = sizer.gaussians()
    n = caps["gauss"]
    np.testing.assert_array_equal(rec["curve"], ref["curve"][:n])
    np.testing.assert_array_equal(rec["local"], ref["local"][:n])
    assert np.array_equal(rec["mu"], ref["mu"][:n])
    assert all(torch.isfinite(g).all().item() for g in grads)


@pytest.mark.parametrize("n_paths,size,tile", [(6, 72, 16), (24, 560, 8)])
def test_pair_overflow_leaves_every_list_empty(n_paths, size, tile):
    """With fewer pair slots than pairs no pair is written, whether the
    pairs are emitted and radix-sorted (the small scene) or placed straight
    at their sorted positions by the low digit of a wider key (4900 tiles,
    then one radix pass): the status bit and the required count are set, the
    pair count is 0, every tile list is empty, the image is the background
    and the step stays finite."""
    import torch
    from paper_2606_31764_amd import _lib as Lb
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.config3(seed=2903, n_paths=n_paths, size=size)  # 114,491 Gaussians at 560^2
    p = Params().replace(h=1.0, tile=tile)
    sizer = Renderer(b, p)
    t = param_tensors(b)
    sizer.run_forward(t)
    full = sizer.read_counters()
    caps = dict(gauss=full[Lb.CNT_GAUSS] + 64, pairs=full[Lb.CNT_PAIRS] // 2, boundary=2 * full[Lb.CNT_BOUND_REQ] + 64)
    r = Renderer(b, p, caps=caps)
    r.sample(t, sync=False)
    r.bin(t, sync=False)
    img = r.forward(t)
    grads = r.backward(t, 2.0 * (img - 0.5))
    torch.cuda.synchronize()
    cnt = r.read_counters()
    assert cnt[Lb.CNT_STATUS] & Lb.STATUS_PAIR_CAP
    assert cnt[Lb.CNT_PAIRS_REQ] == full[Lb.CNT_PAIRS] and cnt[Lb.CNT_PAIRS] == 0
    ranges, _ = r.tiles()
    assert np.all(ranges[:, 1] == ranges[:, 0])
    H, W = b.hw[0]
    bg = np.repeat(np.asarray(b.bg[0], np.float32), H * W)
    np.testing.assert_array_equal(img.cpu().numpy(), bg)
    assert all(torch.isfinite(g).all().item() for g in grads)


def test_timing_mask_records_only_selected_phases():
    """nsplat_timing with NSPLAT_TIMING_ONLY | mask records event pairs around the
    masked phases alone; plain enable records every phase of the step."""
    import ctypes
    import torch
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.config3(seed=2950, n_paths=6, size=64)
    p = Params().replace(h=2.0)
    r = Renderer(b, p)
    t = param_tensors(b)
    img = r.run_forward(t)
    c = r.ctx
    only, bwd_id, n_timers = 0x40000000, 6, 11

    def step_counts(enable):
        c.check(c.lib.nsplat_timing(c.h, enable))
        r.sample(t, sync=False)
        r.bin(t, sync=False)
        im = r.forward(t)
        r.backward(t, 2.0 * (im - 0.5))
        torch.cuda.synchronize()
        ms = (ctypes.c_double * n_timers)()
        n = (ctypes.c_int64 * n_timers)()
        c.check(c.lib.nsplat_timing_read(c.h, ms, n))
        c.check(c.lib.nsplat_timing(c.h, 0))
        return list(n), list(ms)

    n_all, _ = step_counts(1)
    assert all(n_all[i] >= 1 for i in range(10))  # every phase but the regulariser
    n_one, ms_one = step_counts(only | (1 << bwd_id))
    assert n_one[bwd_id] == 1 and ms_one[bwd_id] > 0.0
    assert sum(n_one) == 1
    assert bool(torch.isfinite(img).all())


@pytest.mark.parametrize("persistent", [False, True])
def test_many_tiles_agree(persistent):
    """An 800x800 canvas has 10,000 tiles at tile 8 (the multi-block path of the
    tile order and of the chunk and item offsets) and 2,500 at tile 16 (the
    single-block path); both give the same image and gradients."""
    b = synth.config2(seed=2750, n_curves=8, size=800)
    p = Params().replace(delta_c=1.0)
    tb = synth.perturbed(b, seed=3)
    target = gpu_run(tb, p.replace(tile=16), backward=False)["image"]
    outs = {t: gpu_run(b, p.replace(tile=t), target=target, persistent=persistent) for t in (8, 16)}
    assert outs[8]["ranges"].shape[0] == 10000 and outs[16]["ranges"].shape[0] == 2500
    assert np.abs(outs[8]["image"] - outs[16]["image"]).max() < 2e-6
    assert grad_close(outs[8]["grads"], outs[16]["grads"], rtol=2e-5, atol=1e-7) <= 1.0


def test_wide_radix_digit_lists_are_sorted_and_agree():
    """900 tiles (a 240x240 canvas at tile 8) take one radix pass with a
    10-bit digit (the wavefront-ranked scatter): every tile list must hold
    ascending Gaussian indices, and the render must agree with the 225-tile
    form (8-bit digit)."""
    b = synth.config3(seed=3960, n_paths=10, size=240)
    p = Params().replace(h=2.0)
    tb = synth.perturbed(b, seed=4)
    target = gpu_run(tb, p.replace(tile=16), backward=False)["image"]
    outs = {t: gpu_run(b, p.replace(tile=t), target=target) for t in (8, 16)}
    ranges, idx = outs[8]["ranges"], outs[8]["idx"]
    assert ranges.shape[0] == 900
    n_pairs = 0
    for s, e in ranges:
        if e > s:
            assert np.all(np.diff(idx[s:e]) > 0)
            n_pairs += e - s
    assert n_pairs == len(idx)
    assert np.abs(outs[8]["image"] - outs[16]["image"]).max() < 2e-6
    assert grad_close(outs[8]["grads"], outs[16]["grads"], rtol=2e-5, atol=1e-7) <= 1.0


def test_transmittance_threshold_range():
    # a high threshold stops pixels after a few layers: images and gradients
    # against the oracle; eps_T = 1 (each pixel stops at its first Gaussian
    # with alpha > 0) is accepted, a threshold above 1 is rejected on the host
    from paper_2606_31764_amd._lib import NSplatError
    rng = np.random.default_rng(43)
    parts = [_part(rng.uniform(6, 42, (6, 2)), p=3, seed=1, color=(0.9, 0.2, 0.1)),
             _part(rng.uniform(6, 42, (5, 2)), p=2, closed=True, filled=True, seed=2, color=(0.1, 0.3, 0.8)),
             _part(rng.uniform(6, 42, (6, 2)), p=3, closed=True, seed=3, color=(0.2, 0.7, 0.3))]
    b = _batch(parts)
    _full_parity(b, Params().replace(delta_c=2.0, eps_T=0.5))
    p1 = Params().replace(delta_c=2.0, eps_T=1.0)
    one = gpu_run(b, p1, backward=False)
    # one Gaussian at most per pixel: T >= 1 - alpha_max everywhere
    assert one["T"].min() >= 1.0 - p1.alpha_max - 1e-6
    assert one["T"].min() < 0.5  # and the curves do cover pixels
    with pytest.raises(NSplatError, match="eps_T"):
        gpu_run(b, Params().replace(delta_c=2.0, eps_T=1.5), backward=False)


# ---------------------------------------------------------------------------------
# values outside the domain of Sec. 3.1: the curve is skipped, the status says so
# ---------------------------------------------------------------------------------

_GOOD_A = [[3, 20], [9, 25], [14, 18], [22, 24], [28, 20]]
_GOOD_B = [[4, 6], [10, 3], [17, 9], [24, 4], [30, 8]]
_BAD_XY = [[5, 12], [10, 16], [15, 10], [20, 14], [25, 11]]
BAD_VALUES = {
    "zero_weight": dict(w=[1, 0, 1, 1, 1]),
    "negative_weight": dict(w=[1, 1, -0.5, 1, 1]),
    "zero_width": dict(s=[2, 2, 0, 2, 2]),
    "negative_interval": dict(tau=[1.0, -0.25]),
    "empty_domain": dict(tau=[0.0, 0.0]),
    "nan_key": dict(xy=[[5, 12], [10, float("nan")], [15, 10], [20, 14], [25, 11]]),
    "inf_weight": dict(w=[1, 1, float("inf"), 1, 1]),
    "nan_opacity": dict(o=float("nan")),
    "inf_colour": dict(color=(0.1, float("inf"), 0.3)),
}


@pytest.mark.parametrize("case", sorted(BAD_VALUES))
def test_invalid_values_skip_the_curve(case):
    kw = dict(BAD_VALUES[case])
    xy = kw.pop("xy", _BAD_XY)
    kw.setdefault("w", [1, 1.5, 0.8, 1, 1.2])
    kw.setdefault("s", [2, 2.5, 3, 2, 2])
    kw.setdefault("tau", [1.0, 0.7])
    good_a = _part(_GOOD_A, seed=1)
    good_b = _part(_GOOD_B, seed=2, color=(0.7, 0.1, 0.2))
    bad = _part(xy, **kw)
    p = Params(delta_c=1.5, tile=16)
    with_bad = _batch([good_a, bad, good_b], hw=(32, 36))
    without = _batch([good_a, good_b], hw=(32, 36))
    target = oracle.render(synth.perturbed(without, seed=3), oracle_params(p))[0]
    out = gpu_run(with_bad, p, target=target)
    ref = gpu_run(without, p, target=target)
    from paper_2606_31764_amd import _lib as L
    assert out["counters"][L.CNT_STATUS] == L.STATUS_VALUE
    assert out["plan"][1, 0] == 0 and out["plan"][1, L.PLAN_FLAGS] & L.PLAN_INVALID
    assert not out["plan"][0, L.PLAN_FLAGS] & L.PLAN_INVALID and not out["plan"][2, L.PLAN_FLAGS] & L.PLAN_INVALID
    plans_equal(out["plan"], oracle.plan(with_bad, oracle_params(p))[0])
    np.testing.assert_array_equal(out["image"], ref["image"])  # bit for bit
    for n in ("key_xy", "key_w", "key_s", "tau", "color", "opacity"):
        assert np.all(np.isfinite(out["grads"][n])), n
    k0, k1 = with_bad.key_off[1], with_bad.key_off[2]
    assert np.all(out["grads"]["key_xy"][k0:k1] == 0) and np.all(out["grads"]["key_w"][k0:k1] == 0)
    assert np.all(out["grads"]["tau"][with_bad.tau_off[1]:with_bad.tau_off[2]] == 0)
    assert out["grads"]["opacity"][1] == 0 and np.all(out["grads"]["color"][1] == 0)
    # the other curves' gradients are those of the batch without the bad curve
    keep = np.r_[0:k0, k1:len(with_bad.key_w)]
    np.testing.assert_allclose(out["grads"]["key_xy"][keep], ref["grads"]["key_xy"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(out["grads"]["opacity"][[0, 2]], ref["grads"]["opacity"], rtol=1e-5, atol=1e-6)


def test_invalid_values_under_a_frozen_plan():
    """A curve whose weight becomes 0 between two calls is skipped also when
    the second call keeps the first call's plan."""
    import torch
    from paper_2606_31764_amd import _lib as L
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = _batch([_part(_GOOD_A, seed=1), _part(_BAD_XY, seed=4), _part(_GOOD_B, seed=2)], hw=(32, 36))
    r = Renderer(b, Params(delta_c=1.5))
    t = param_tensors(b)
    r.run_forward(t)
    assert r.read_counters()[L.CNT_STATUS] == 0 and r.plan_np()[1, 0] > 0
    t[1][b.key_off[1] + 2] = 0.0
    r.run_forward(t, frozen=True)
    torch.cuda.synchronize()
    cnt = r.read_counters()
    plan = r.plan_np()
    assert cnt[L.CNT_STATUS] == L.STATUS_VALUE and plan[1, 0] == 0 and plan[1, L.PLAN_FLAGS] & L.PLAN_INVALID
    assert cnt[L.CNT_GAUSS] == plan[0, 0] + plan[2, 0]
    assert np.all(np.isfinite(r.image.cpu().numpy()))


def test_forward_and_backward_refuse_another_tile_than_bin():
    """Tile lists are laid out for the tile side nsplat_bin used; a forward or
    backward with another params.tile is an argument error, not wrong output."""
    import torch
    from paper_2606_31764_amd import _lib as L
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.config2(seed=2801, n_curves=4, size=64)
    p = Params(delta_c=3.0, tile=16)
    r = Renderer(b, p)
    t = param_tensors(b)
    r.run_forward(t)
    with pytest.raises(L.NSplatError, match="tile 16"):
        r.forward(t, params=p.replace(tile=32))
    dL = torch.ones_like(r.image)
    with pytest.raises(L.NSplatError, match="tile 16"):
        r.backward(t, dL, params=p.replace(tile=8))
    r.bin(t, params=p.replace(tile=32))
    r.forward(t, params=p.replace(tile=32))  # consistent again
    r.backward(t, dL, params=p.replace(tile=32))
    torch.cuda.synchronize()


def test_backward_refuses_items_of_another_fill_split():
    """At 32 x 32 tiles nsplat_bin lays out the adjoint items of scenes with
    fills per 8 x 8 block; a backward whose curves differ in NSPLAT_FILLED
    (so it would read them per quadrant) is an argument error."""
    import torch
    from paper_2606_31764_amd import _lib as L
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.config3(seed=3960, n_paths=4, size=64)
    p = Params().replace(h=1.0, tile=32)
    r = Renderer(b, p)
    t = param_tensors(b)
    r.run_forward(t)
    dL = torch.ones_like(r.image)
    m = r.meta
    declared = (m.any_flags, m.all_flags)
    m.any_flags, m.all_flags = declared[0] & ~synth.FILLED, declared[1] & ~synth.FILLED
    with pytest.raises(L.NSplatError, match="pixel blocks"):
        r.backward(t, dL)
    m.any_flags, m.all_flags = declared
    r.backward(t, dL)  # consistent again
    torch.cuda.synchronize()


def test_declared_flag_intersection():
    """nsplat_curves.all_flags declares flags every curve carries: with
    NSPLAT_FILLED declared the stroke adjoint is not launched and a stroke
    in the batch is invalid data (no Gaussians, status bit, plan flag) while
    the fills render and differentiate as without it; the binding's own
    intersection (fills and strokes: nothing) leaves both adjoints on."""
    import torch
    from paper_2606_31764_amd import _lib as Lb
    from paper_2606_31764_amd.render import Renderer, param_tensors
    fills = synth.fills(3300, n_paths=3, size=64, radius=(6.0, 16.0))
    strokes = synth.strokes(3301, n_curves=2, size=64, nk_range=(5, 7))
    b = synth._assemble(fills + strokes, [[64, 64]], [[1.0, 1.0, 1.0]], 3)
    p = Params().replace(h=1.0, delta_c=3.0)
    r = Renderer(b, p)
    assert r.meta.all_flags & synth.FILLED == 0
    r.meta.all_flags = synth.FILLED | synth.CLOSED
    t = param_tensors(b)
    img = r.run_forward(t)
    grads = r.backward(t, 2.0 * (img - 0.5))
    torch.cuda.synchronize()
    cnt = r.read_counters()
    plan = r.plan_np()
    filled = (b.flags & synth.FILLED) != 0
    assert cnt[Lb.CNT_STATUS] & 8
    assert np.all(plan[~filled, 0] == 0) and np.all(plan[~filled, Lb.PLAN_FLAGS] & Lb.PLAN_INVALID)
    sub = synth._gather(b, np.flatnonzero(filled), lambda c: 0, b.hw, b.bg)
    ref = oracle.render(sub, oracle_params(p))[0]
    assert np.abs(img.cpu().numpy().astype(np.float64) - ref).max() <= IMG_TOL
    ko = int(b.key_off[int(np.flatnonzero(~filled)[0])])
    assert torch.all(grads[0].view(-1, 2)[ko:] == 0)  # no gradient reaches the invalid strokes
    assert all(torch.isfinite(g).all().item() for g in grads)


@pytest.mark.parametrize("chunk", [512, 1024, 4096, 8192])
def test_chunk_lengths_against_oracle(chunk):
    """Every chunk length the adjoint's split of the tile lists allows gives
    the oracle's image and gradients, on lists of a few chunks at 512."""
    b = synth.config3(seed=3960, n_paths=12, size=96)
    p = Params().replace(h=1.0, tile=16, chunk=chunk)
    out = _full_parity(b, p)
    lens = out["ranges"][:, 1] - out["ranges"][:, 0]
    print("chunk", chunk, "longest list", int(lens.max()), flush=True)
    assert lens.max() > 2 * 512


def test_chunk_length_is_checked():
    """params.chunk must be 0 or a power of two in [512, 8192], and the
    forward and backward refuse a chunk length other than the one nsplat_bin
    laid the lists out for."""
    import torch
    from paper_2606_31764_amd import _lib as L
    from paper_2606_31764_amd.render import Renderer, param_tensors
    b = synth.config2(seed=2802, n_curves=4, size=64)
    p = Params(delta_c=3.0, chunk=1024)
    r = Renderer(b, p)
    t = param_tensors(b)
    r.run_forward(t)
    for bad in (256, 1000, 16384, -512):
        with pytest.raises(L.NSplatError, match="chunk must be"):
            r.bin(t, params=p.replace(chunk=bad))
    with pytest.raises(L.NSplatError, match="chunk 1024"):
        r.forward(t, params=p.replace(chunk=2048))
    dL = torch.ones_like(r.image)
    with pytest.raises(L.NSplatError, match="chunk 1024"):
        r.backward(t, dL, params=p.replace(chunk=512))
    r.bin(t, params=p.replace(chunk=2048))
    r.forward(t, params=p.replace(chunk=2048))  # consistent again
    r.backward(t, dL, params=p.replace(chunk=2048))
    torch.cuda.synchronize()


@pytest.mark.parametrize("p_deg", [1, 4, 5])
def test_fill_of_other_degrees(p_deg):
    """Filled closed curves of degree 1 (a polygon), 4 and 5, against the oracle."""
    rng = np.random.default_rng(40 + p_deg)
    parts = []
    for k in range(3):
        nk = 9 + k
        ang = 2 * np.pi * np.arange(nk) / nk + rng.uniform(-0.2, 0.2, nk)
        rad = rng.uniform(9.0, 15.0, nk)
        c = (14 + 12 * k, 16 + 6 * k)
        xy = np.stack([c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang)], 1)
        parts.append(_part(xy, p=p_deg, closed=True, filled=True, color=tuple(rng.uniform(0, 1, 3)),
                           o=0.85, seed=50 + k))
    b = _batch(parts, hw=(44, 52))
    _full_parity(b, Params(h=1.0))


def test_clockwise_fill():
    """A fill whose boundary runs clockwise has winding -1 inside, so its SDF
    sign is -1 everywhere (R11): the interior is not filled, only a band
    around the boundary shows (opacity o sigmoid(-gamma d / h)).  GPU and
    oracle agree, and pixels far inside keep the background."""
    nk = 12
    ang = -2 * np.pi * np.arange(nk) / nk          # decreasing angle: clockwise in y-down pixels
    xy = np.stack([24 + 15 * np.cos(ang), 22 + 15 * np.sin(ang)], 1)
    b = _batch([_part(xy, p=3, closed=True, filled=True, color=(0.9, 0.1, 0.1), o=0.9, seed=7)], hw=(44, 48))
    out = _full_parity(b, Params(h=1.0))
    img = out["image"].reshape(3, 44, 48)
    # the centre (9 px or more from the boundary): background
    assert np.all(np.abs(img[:, 18:27, 20:29] - 1.0) < 1e-4)
    # the same path counter-clockwise fills the centre
    xy_ccw = xy[::-1].copy()
    b2 = _batch([_part(xy_ccw, p=3, closed=True, filled=True, color=(0.9, 0.1, 0.1), o=0.9, seed=7)], hw=(44, 48))
    img2 = gpu_run(b2, Params(h=1.0), backward=False)["image"].reshape(3, 44, 48)
    assert np.all(np.abs(img2[0, 18:27, 20:29] - (0.9 * 0.9 + 0.1 * 1.0)) < 2e-2)


@pytest.mark.parametrize("n_cp,delta_c", [(6000, 3.0), (3000, 0.02)])
def test_stroke_span_search_long_and_sparse(n_cp, delta_c):
    """Stroke samples of a wavefront on one curve find their knot spans
    cooperatively: over 6000 key points (three search rounds, more than 4096
    knots) and, with very sparse sampling, windows wider than the 64 spans a
    wavefront stages (the per-sample fallback).  Plan, curve and sample
    indices bit-exact, centres within 1e-9 px of the oracle."""
    b = synth._assemble(synth.long_splines(4300, n_curves=1, n_cp=n_cp, size=512, channels=3), [[512, 512]],
                        [[1.0, 1.0, 1.0]], 3)
    p = Params().replace(delta_c=delta_c)
    ref = oracle.gaussians(b, oracle_params(p))
    out = gpu_run(b, p, backward=False)
    assert out["counters"][2] == 0
    plans_equal(out["plan"], ref["plan"])
    g = out["gauss"]
    print("n_cp", n_cp, "delta_c", delta_c, "Gaussians", len(g["sigma"]), flush=True)
    np.testing.assert_array_equal(g["curve"], ref["curve"])
    np.testing.assert_array_equal(g["local"], ref["local"])
    assert np.abs(g["mu"] - ref["mu"]).max() < 1e-9
    np.testing.assert_allclose(g["sigma"], ref["sigma"].astype(np.float32), rtol=2e-7, atol=0)
