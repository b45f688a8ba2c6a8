"""Benchmark of the NURBS Splatting render path on one MI355X.

A step is one pass of the whole path over one batch: nsplat_sample ->
nsplat_bin -> nsplat_forward -> L2 loss gradient -> nsplat_backward.
Workload: 256 filled closed degree-2/3 paths (6-24 key points, radii 5-80 px)
on a 512x512 RGB canvas at fill grid step h = 1 (about 1M Gaussians), seeded
synthetic data.  Prints one JSON line.

Also measured (same JSON line): the batched form (64 uneven scenes, one
persistent launch sequence captured in a HIP graph) against per-scene plain
launches, and the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = dict(hbm_gbs=8000.0, fp32_tflops=157.3, fp64_tflops=78.6)
PHASES = ["plan", "emit", "bin", "sort", "ranges", "blend_fwd", "blend_bwd", "adj_gauss", "adj_bound", "fold",
          "reg"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-optim", action="store_true", help="skip the full optimisation-step measurement")
    ap.add_argument("--optim-steps", type=int, default=10)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-aniso", action="store_true", help="skip the tangent-aligned contour measurement")
    ap.add_argument("--only", choices=["batched", "optim", "aniso"], default=None,
                    help="run one secondary leg alone (for profiling); prints its result as JSON")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


class Step:
    """Pre-sized render state + the device-side L2 gradient of one workload."""

    def __init__(self, batch, params, target, persistent=False, ctx=None):
        import torch
        from paper_2606_31764_amd.render import Renderer, param_tensors
        self.torch = torch
        self.r = Renderer(batch, params, persistent=persistent, ctx=ctx)
        self.t = param_tensors(batch)
        self.target = torch.as_tensor(np.asarray(target, np.float32), device="cuda")
        self.dL = torch.empty_like(self.target)
        self.loss = torch.zeros(1, device="cuda")
        self.r.run_forward(self.t)                      # sizes every buffer (synchronising)
        cnt = self.r.read_counters()
        self.G, self.pairs = cnt[0], cnt[1]

    def run(self):
        """One step, no host synchronisation."""
        r, c = self.r, self.r.ctx
        r.sample(self.t, sync=False)
        r.bin(self.t, sync=False)
        img = r.forward(self.t)
        c.check(c.lib.nsplat_l2_grad(c.h, ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(self.target.data_ptr()),
                                     ctypes.c_void_p(self.dL.data_ptr()), ctypes.c_void_p(self.loss.data_ptr()),
                                     img.numel(), ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)))
        return r.backward(self.t, self.dL)


TIMING_ONLY = 0x40000000  # nsplat_timing: record only the phases of the mask


def timing_on(ctx, on):
    ctx.check(ctx.lib.nsplat_timing(ctx.h, int(on)))


def timing_read(ctx):
    ms = (ctypes.c_double * len(PHASES))()
    n = (ctypes.c_int64 * len(PHASES))()
    ctx.check(ctx.lib.nsplat_timing_read(ctx.h, ms, n))
    return {PHASES[i]: (ms[i], n[i]) for i in range(len(PHASES))}


def blend_work(step, tile, frame=None):
    """Algorithmic work of one forward blend launch, counted with torch on the
    GPU from the launch's own tile lists and stopping positions: evaluated
    (pixel, Gaussian) pairs, in-support pairs, and in-support pairs of fill
    Gaussians.  With the tangent-aligned frame ([G, 4] device tensor of
    (t, sp, ratio)), the support of a tangent-aligned Gaussian is its ellipse
    (the fill count then counts those pairs instead)."""
    import torch
    r = step.r
    G = step.G
    raw = r.gauss[:G]
    u8 = raw.view(torch.uint8).view(G, 32)
    mx, my = raw[:, 0], raw[:, 1]
    sigma = u8[:, 16:20].contiguous().view(torch.float32).view(G).double()
    ranges, idx = r.ranges, r.idx
    H, W = int(r.meta.hw_host[0][0]), int(r.meta.hw_host[0][1])
    tx_n = (W + tile - 1) // tile
    n_tiles = tx_n * ((H + tile - 1) // tile)
    rg = ranges[:n_tiles].long()
    lens = rg[:, 1] - rg[:, 0]
    P = int(lens.sum().item())
    tile_of = torch.repeat_interleave(torch.arange(n_tiles, device="cuda"), lens)
    pos = torch.arange(P, device="cuda")
    gidx = idx[:P].long()
    stop = r.n_last.view(H, W).long()
    curve = u8[:, 24:28].contiguous().view(torch.int32).view(G).long()
    is_fill = ((r.meta.flags.long() & 2) != 0)[curve][gidx]
    if frame is not None:
        is_fill = ((r.meta.flags.long() & 4) != 0)[curve][gidx]
        fr = frame[:G].double()[gidx]
    ev = 0
    hit = 0
    hit_fill = 0
    ks = r.params.k_sigma
    for ly in range(tile):
        for lx in range(tile):
            x = (tile_of % tx_n) * tile + lx
            y = (tile_of // tx_n) * tile + ly
            ok = (x < W) & (y < H)
            xs, ys = x.clamp(max=W - 1), y.clamp(max=H - 1)
            st = stop[ys, xs]
            e = ok & (pos >= st)
            dx = xs.double() + 0.5 - mx[gidx]
            dy = ys.double() + 0.5 - my[gidx]
            if frame is None:
                h = e & (dx * dx + dy * dy <= (ks * sigma[gidx]) ** 2)
            else:
                dp = dx * fr[:, 0] + dy * fr[:, 1]
                dq = dy * fr[:, 0] - dx * fr[:, 1]
                m2 = (dp / sigma[gidx]) ** 2 + (dq / fr[:, 2]) ** 2
                h = e & torch.where(is_fill, m2 <= ks * ks, dx * dx + dy * dy <= (ks * sigma[gidx]) ** 2)
            ev += int(e.sum().item())
            hit += int(h.sum().item())
            hit_fill += int((h & is_fill).sum().item())
    return ev, hit, hit_fill


# Algorithmic FP32 operations per in-support (pixel, Gaussian) pair of the
# formulation the kernels compute; an FMA counts 2.  Forward: d^2 (2 sub,
# mul, fma) 5, exp2 argument and exp2 2, o G and the alpha_max clamp 2,
# 1 - alpha and T (1 - alpha) 2, termination test 1 = 12 (the colour is added
# once per run of one curve's entries, as col (T at the run's start - T), not
# per pair).  Adjoint of a fill Gaussian (back to front inside a chunk): d^2 5,
# exp2 2, o G and clamp 2, 1 - alpha 1, r = rcp(1 - alpha) 1, dL/dalpha =
# -W r 1, T = T' r 1, the run's sum of alpha T (FMA) 2, dL/do_j (FMA) 2 = 17
# (K, W and the colour gradient are per curve run, not per pair); a stroke
# Gaussian adds dL/do_j o 1, the d^2 factor G a ln 2 3, dL/dmu 2 x 3 and
# dL/dsigma 4 = 32.  Tangent-aligned strokes: forward 2 subs, a = d . u 3,
# b = r (d x u) 4, a^2 + b^2 3, exp2 1, o G and clamp 2, 1 - alpha and
# T (1 - alpha) 2, termination test 1 = 18; adjoint the same geometry 12,
# exp2 1, clamp 2, 1 - alpha, rcp, dL/dalpha, T' r 4, sum alpha T 2,
# dL/do_j 2, h = dL/dalpha o G 2 ln 2 3, dL/dmu 2 x 5, dL/dsigma, dL/dsp,
# dL/dtheta 11 = 47.
FWD_HIT_FLOPS, BWD_FILL_HIT_FLOPS, BWD_STROKE_HIT_FLOPS = 12, 17, 32
FWD_ANISO_HIT_FLOPS, BWD_ANISO_HIT_FLOPS = 18, 47
# The build disables packed FP32 instructions, so the FP32 vector peak is
# 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s, not the
# packed 157.3.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def source_digest():
    """SHA-256 of the blend kernel sources (identifies the build that counters were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("blend.hip", "nsplat_internal.h"):
        with open(os.path.join(ROOT, "paper_2606_31764_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summary under
    profiles/, or None when that summary was taken on other kernel sources."""
    import re
    path = os.path.join(ROOT, "profiles", "blend_bwd_c3_512_fills.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    m_b = re.search(r"traffic_bytes_per_launch\[%s\]:\s*([0-9.eE+]+)" % re.escape(kernel), txt)
    if not m_sha or not m_b or m_sha.group(1) != source_digest():
        return None
    return float(m_b.group(1))


FB_ITEMS = 4096  # Gaussians per block of the binning by placement (the library's constant)


def phase_bytes(step, tile):
    """Algorithmic HBM bytes of one step's sample / bin / sort / ranges phases.
    emit writes the 32 B record of every Gaussian (+4 B argmin of a fill
    Gaussian).  Binning by placement (the library's choice for at least 65,536
    Gaussian slots and at most 8 pair slots each): bin reads every record and
    writes the per-block counts of the low key digit, which the scan reads and
    writes; sort reads the records again and writes each pair's 4 B index
    (+4 B key when more digits follow), then 20 B per pair for every further
    radix pass; ranges reads the scanned counts (one digit) or the keys and
    writes 8 B per tile.  Otherwise: bin reads the records twice (count,
    emit), writes and rescans the 4 B counts and writes the 8 B (key, index)
    pairs; every radix pass reads the keys for its histogram, then reads and
    writes keys and indices (20 B per pair); ranges as above."""
    r = step.r
    cnt = r.read_counters()
    G, P = int(cnt[0]), int(cnt[1])
    plan = r.plan_np()
    fill = (r.meta.flags.cpu().numpy() & 2) != 0
    n_fill = int(plan[fill, 0].astype(np.int64).sum())
    n_tiles = int(r.ctx.lib.nsplat_num_tiles(ctypes.byref(r.meta.scenes_c), int(tile)))
    bits = 0
    while bits < 31 and (1 << bits) < n_tiles:
        bits += 1
    passes = (bits + 9) // 10
    gcap, pcap = int(r.caps["gauss"]), int(r.caps["pairs"])
    placed = passes >= 1 and gcap >= 65536 and pcap <= 8 * gcap
    emit = 32 * G + 4 * n_fill
    if placed:
        digit = (bits + passes - 1) // passes
        nb = max((gcap + FB_ITEMS - 1) // FB_ITEMS, 1)
        counts = 4 * ((1 << digit) + 1) * nb
        out = dict(emit=emit, bin=32 * G + 3 * counts,
                   sort=32 * G + (4 if passes == 1 else 8) * P + (passes - 1) * 20 * P,
                   ranges=(8 * n_tiles if passes == 1 else 4 * P + 8 * n_tiles))
    else:
        out = dict(emit=emit, bin=64 * G + 12 * G + 8 * P, sort=passes * 20 * P, ranges=4 * P + 8 * n_tiles)
    return out, passes


def hbm_table(nbytes, phases):
    out = {}
    for k, b in nbytes.items():
        ms = phases.get(k)
        if ms:
            gbs = b / (ms * 1e-3) / 1e9
            out[k] = dict(bytes=b, ms=ms, gbs=gbs, frac=gbs / PEAK["hbm_gbs"])
    return out


def bench_main(args):
    import torch
    from paper_2606_31764_amd import synth
    from paper_2606_31764_amd.render import Params, Renderer, param_tensors

    torch.cuda.init()
    b = synth.config3()
    p = Params().replace(h=1.0, tile=args.tile, batch=args.batch)
    log("workload: 256 filled paths, 512x512, h=1")
    # target: the same generator's ground truth, perturbed (P + N(0, 2^2), ...)
    tr = Renderer(synth.perturbed(b, seed=3999), p)
    target = tr.run_forward(param_tensors(synth.perturbed(b, seed=3999))).clone().cpu().numpy()
    del tr
    st = Step(b, p, target)
    log("G = %d, pairs = %d" % (st.G, st.pairs))
    for _ in range(args.warmup):
        st.run()
    torch.cuda.synchronize()
    ctx = st.r.ctx
    # per-phase breakdown (an event pair around every phase) outside the timed region
    timing_on(ctx, True)
    for _ in range(min(args.steps, 10)):
        st.run()
    torch.cuda.synchronize()
    phases = timing_read(ctx)
    timing_on(ctx, False)
    for k, (ms, n) in phases.items():
        if n:
            log("  %-10s %8.4f ms/launch  (%d launches)" % (k, ms / n, n))
    # dominant single-kernel phase; in the timed region only its launches carry events
    single = ["emit", "blend_fwd", "blend_bwd", "adj_gauss", "adj_bound"]
    dom = max(single, key=lambda k: phases[k][0])
    timing_on(ctx, TIMING_ONLY | (1 << PHASES.index(dom)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        st.run()
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    dom_t = timing_read(ctx)[dom]
    timing_on(ctx, False)
    ms_step = total_ms / args.steps
    dom_ms = dom_t[0] / max(dom_t[1], 1)
    log("ms/step %.4f (%s %.4f ms/launch over the timed steps)" % (ms_step, dom, dom_ms))
    roof = roofline(st, dom, dom_ms, p)
    out = dict(metric="fwd+bwd Gaussians/s (512x512, ~1M splats)", value=st.G / (ms_step * 1e-3),
               unit="Gaussians/s", n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms_step,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32 (FP64 curve evaluation)",
               data="synthetic",
               config=dict(workload="256 filled closed NURBS paths (p 2/3, 6-24 key points, radii 5-80 px), "
                                    "512x512 RGB, fill grid h=1, L2 loss vs perturbed target",
                           gaussians=st.G, pairs=st.pairs, tile=p.tile, batch=p.batch),
               phases_ms={k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()},
               roofline=roof)
    nbytes, passes = phase_bytes(st, p.tile)
    out["hbm_phases"] = hbm_table(nbytes, out["phases_ms"])
    out["hbm_phases"]["radix_passes"] = passes
    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if not args.no_batched:
        out["batched"] = bench_batched(args)
    if not args.no_optim:
        out["optim_step"] = bench_optim(args)
    if not args.no_aniso:
        out["tangent_aligned"] = bench_aniso(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b, p, target)
    return out


def roofline(st, dom, dom_ms, p):
    """Roofline entry of the dominant kernel: algorithmic FP32 operations of
    its in-support pairs over its measured average launch time, against the
    non-packed FP32 vector peak; HBM traffic from the profiled counters."""
    if dom in ("blend_fwd", "blend_bwd"):
        ev, hit, hit_fill = blend_work(st, p.tile)
        if dom == "blend_fwd":
            flops, kernel = FWD_HIT_FLOPS * hit, "k_blend_fwd"
        else:
            flops = BWD_FILL_HIT_FLOPS * hit_fill + BWD_STROKE_HIT_FLOPS * (hit - hit_fill)
            kernel = "k_blend_bwd"
        ach = flops / (dom_ms * 1e-3) / 1e12
        return dict(kernel=kernel, bound="alu", achieved=ach, peak=ALU_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / ALU_PEAK_TFLOPS, traffic=profiled_traffic(kernel), in_support_pairs=hit,
                    in_support_fill_pairs=hit_fill, evaluated_pairs=ev, flops_per_launch=flops,
                    ms_per_launch=dom_ms)
    return dict(kernel=dom, bound="alu", achieved=None, peak=None, unit=None, frac=None, traffic=None,
                ms_per_launch=dom_ms)


def bench_batched(args):
    """64 uneven scenes: per-scene plain launches vs one batched persistent
    launch sequence replayed from a HIP graph."""
    import torch
    from paper_2606_31764_amd import synth
    from paper_2606_31764_amd.render import Context, Params
    b5, kinds = synth.config5()
    p = Params().replace(**synth.CONFIG_PARAMS[5])
    ctx = Context(0)
    log("batched: %d scenes, %d curves" % (b5.n_scenes, b5.n_curves))
    # targets: each scene's perturbed ground truth, rendered once by the plain path
    pert = synth.perturbed(b5, seed=5999)
    scenes = [b5.select_scene(s) for s in range(b5.n_scenes)]
    plain = []
    tgt_all = []
    for s in range(b5.n_scenes):
        from paper_2606_31764_amd.render import Renderer, param_tensors
        ps = pert.select_scene(s)
        tr = Renderer(ps, p, ctx=ctx)
        tg = tr.run_forward(param_tensors(ps)).clone()
        tgt_all.append(tg)
        del tr
        plain.append(Step(scenes[s], p, tg.cpu().numpy(), ctx=ctx))
    G_plain = sum(s.G for s in plain)
    target = torch.cat(tgt_all).cpu().numpy()
    bat = Step(b5, p, target, persistent=True, ctx=ctx)
    log("batched G = %d (plain sum %d), pairs = %d" % (bat.G, G_plain, bat.pairs))
    # autotune tile size and batch depth for the batched form (pair buffers
    # sized for the smallest tile first)
    bat.r.run_forward(bat.t, params=p.replace(tile=8))
    bat.run()
    torch.cuda.synchronize()
    tile, depth, tune_ms = bat.r.autotune(bat.t, bat.dL)
    log("autotune: tile %d, batch depth %d (%s)" % (tile, depth, " ".join("%.2f" % x for x in tune_ms)))
    tuned = bat if (tile, depth) == (p.tile, p.batch) else \
        Step(b5, p.replace(tile=tile, batch=depth), target, persistent=True, ctx=ctx)
    K = args.batched_steps
    for _ in range(2):
        for s in plain:
            s.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        for s in plain:
            s.run()
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / K

    def graph_ms(st):
        """Capture one step of st into a graph; time K replays; check a replay against an eager step."""
        s_cap = torch.cuda.Stream()
        s_cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_cap):
            for _ in range(2):
                st.run()
        torch.cuda.current_stream().wait_stream(s_cap)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            grads = st.run()
        torch.cuda.synchronize()
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        eager = [x.clone() for x in st.run()]
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ok = all(float((a - b_).abs().max()) <= 1e-4 * float(a.abs().max() + 1e-6) for a, b_ in zip(eager, grads))
        del g
        return ms, ok

    bat_ms, same = graph_ms(tuned)
    same_cfg_ms = bat_ms if tuned is bat else graph_ms(bat)[0]
    bat = tuned
    # diagnostic (outside the timed regions): per-phase times of one eager step of each form
    def phase_pass(steps, runs):
        c = steps[0].r.ctx
        timing_on(c, True)
        for st_ in steps:
            for _ in range(runs):
                st_.run()
        torch.cuda.synchronize()
        ph = timing_read(c)
        timing_on(c, False)
        return {k: v[0] / runs for k, v in ph.items()}
    ph_plain = phase_pass(plain, 2)
    ph_bat = phase_pass([bat], 2)
    log("phase ms per step   plain   batched")
    for k in PHASES:
        log("  %-10s %8.3f %8.3f" % (k, ph_plain[k], ph_bat[k]))
    res = dict(scenes=b5.n_scenes, gaussians=bat.G, plain_ms_per_step=plain_ms, batched_ms_per_step=bat_ms,
               plain_gaussians_per_s=G_plain / (plain_ms * 1e-3), batched_gaussians_per_s=bat.G / (bat_ms * 1e-3),
               speedup=plain_ms / bat_ms, graph_replay_matches_eager=bool(same),
               tile=tile, batch_depth=depth, autotune_ms=tune_ms,
               batched_ms_at_plain_config=same_cfg_ms, speedup_at_plain_config=plain_ms / same_cfg_ms,
               phases_ms_plain=ph_plain, phases_ms_batched=ph_bat)
    nbytes, passes = phase_bytes(bat, tile)
    res["hbm_phases_batched"] = hbm_table(nbytes, ph_bat)
    res["hbm_phases_batched"]["radix_passes"] = passes
    res["pairs"] = int(bat.r.read_counters()[1])
    log("batched: plain %.3f ms, batched %.3f ms, speedup %.2fx" % (plain_ms, bat_ms, plain_ms / bat_ms))
    res["per_kind"] = batched_per_kind(args, b5, kinds, plain, tgt_all, p.replace(tile=tile, batch=depth), ctx)
    return res


def batched_per_kind(args, b5, kinds, plain, tgt_all, p, ctx):
    """Where the batched step's time goes by scene kind: the scenes of each
    kind (strokes, fills, long splines) as a batch of their own at the tuned
    setting, eager steps timed with events, their phases and sizes, and the
    same scenes' plain per-scene steps."""
    import torch
    from paper_2606_31764_amd import synth
    names = ("strokes", "fills", "long_splines")
    out = {}
    K = args.batched_steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for k, name in enumerate(names):
        idx = [s for s in range(b5.n_scenes) if kinds[s] == k]
        if not idx:
            continue
        sub = synth.concat([b5.select_scene(s) for s in idx])
        tgt = torch.cat([tgt_all[s] for s in idx]).cpu().numpy()
        st = Step(sub, p, tgt, persistent=True, ctx=ctx)
        for _ in range(2):
            st.run()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            st.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        timing_on(ctx, True)
        for _ in range(2):
            st.run()
        torch.cuda.synchronize()
        ph = timing_read(ctx)
        timing_on(ctx, False)
        steps = [plain[s] for s in idx]
        e0.record()
        for _ in range(K):
            for s_ in steps:
                s_.run()
        e1.record()
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / K
        out[name] = dict(scenes=len(idx), gaussians=int(st.G), pairs=int(st.pairs),
                         pixels=int(sum(int(h) * int(w) for h, w in sub.hw)), batched_ms=ms, plain_ms=pms,
                         phases_ms={kk: v[0] / 2 for kk, v in ph.items()})
        log("  kind %-12s %2d scenes, G %8d, pairs %9d: batched %.3f ms (fwd %.3f, bwd %.3f), plain %.3f ms" % (
            name, len(idx), st.G, st.pairs, ms, ph["blend_fwd"][0] / 2, ph["blend_bwd"][0] / 2, pms))
        del st
    return out


def bench_aniso(args):
    """Tangent-aligned contour Gaussians (the prototype variant of Eq. 5)
    next to the paper's isotropic ones on the calligraphy workload (32 open
    cubic strokes, 256x256, delta_c 3 / delta_a 0.25): fwd + L2 bwd per step,
    and the blend kernels' algorithmic rates."""
    import torch
    from paper_2606_31764_amd import synth
    from paper_2606_31764_amd.render import Context, Params, Renderer, param_tensors
    p = Params().replace(**synth.CONFIG_PARAMS[2])
    ctx = Context(0)
    res = {}
    K = args.steps
    for name, flags in (("isotropic", 0), ("tangent_aligned", synth.ANISO)):
        b = synth._assemble(synth.strokes(2000, flags=flags), [[256, 256]], [[1.0, 1.0, 1.0]], 3)
        pert = synth.perturbed(b, seed=2999)
        tr = Renderer(pert, p, ctx=ctx)
        target = tr.run_forward(param_tensors(pert)).clone().cpu().numpy()
        del tr
        st = Step(b, p, target, ctx=ctx)
        for _ in range(args.warmup):
            st.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            st.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        timing_on(ctx, True)
        for _ in range(min(K, 10)):
            st.run()
        torch.cuda.synchronize()
        ph = timing_read(ctx)
        timing_on(ctx, False)
        phm = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in ph.items()}
        frame = None
        if flags:
            frame = torch.empty((max(st.G, 1), 4), dtype=torch.float32, device="cuda")
            cv = st.r.meta.curves_c(*st.t)
            ctx.check(ctx.lib.nsplat_gauss_frame(ctx.h, ctypes.byref(cv), ctypes.byref(st.r.meta.scenes_c),
                                                 ctypes.byref(st.r.bufs), ctypes.c_void_p(frame.data_ptr()),
                                                 int(st.G), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        ev, hit, hit_k = blend_work(st, p.tile, frame)
        if flags:
            f_fwd, f_bwd = FWD_ANISO_HIT_FLOPS * hit_k, BWD_ANISO_HIT_FLOPS * hit_k
        else:
            f_fwd, f_bwd = FWD_HIT_FLOPS * hit, BWD_STROKE_HIT_FLOPS * hit
        ach_f = f_fwd / (phm["blend_fwd"] * 1e-3) / 1e12 if phm["blend_fwd"] else None
        ach_b = f_bwd / (phm["blend_bwd"] * 1e-3) / 1e12 if phm["blend_bwd"] else None
        res[name] = dict(gaussians=int(st.G), pairs=int(st.pairs), ms_per_step=ms,
                         gaussians_per_s=st.G / (ms * 1e-3), in_support_pairs=hit, evaluated_pairs=ev,
                         blend_fwd_tflops=ach_f, blend_bwd_tflops=ach_b,
                         blend_fwd_frac=(ach_f / ALU_PEAK_TFLOPS) if ach_f else None,
                         blend_bwd_frac=(ach_b / ALU_PEAK_TFLOPS) if ach_b else None, phases_ms=phm)
        log("%s strokes: G %d, %.4f ms/step (fwd %.4f, bwd %.4f, adj %.4f ms)" % (
            name, st.G, ms, phm["blend_fwd"], phm["blend_bwd"], phm["adj_gauss"]))
        del st
    res["workload"] = "32 open cubic strokes (12-40 key points, widths 1-8 px), 256x256 RGB, L2 vs perturbed target"
    return res


def bench_optim(args):
    """One full optimisation step on the long-spline workload (16 open cubics x
    2000 key points, 1024^2 grayscale): sample, bin, forward, L2 gradient,
    backward with the derivative loss (r = 3) and the bounding-box loss at the
    calligraphy weights (lambda_deriv 1, lambda_bbox 5), and the Adam step with
    its cosine decay and clamps, captured once in a HIP graph and replayed."""
    import torch
    from paper_2606_31764_amd import synth
    from paper_2606_31764_amd.render import Adam, Context, Params, Reg, Renderer, param_tensors
    b = synth.config4()
    p = Params().replace(**synth.CONFIG_PARAMS[4])
    ctx = Context(0)
    pert = synth.perturbed(b, seed=4999)
    tr = Renderer(pert, p, ctx=ctx)
    target = tr.run_forward(param_tensors(pert)).clone()
    del tr
    t0 = param_tensors(b)
    sizer = Renderer(b, p, ctx=ctx)
    sizer.run_forward(t0)
    cnt = sizer.read_counters()
    del sizer
    # the parameters move during the run: capacities with 2x slack
    caps = dict(gauss=2 * cnt[3] + 1024, pairs=2 * cnt[4] + 4096, boundary=2 * cnt[5] + 64)
    t = [x.clone() for x in t0]
    r = Renderer(b, p, caps=caps, ctx=ctx)
    # Adam moves each parameter by about its learning rate per step, so the
    # rates follow this workload's scales: the calligraphy rates of the
    # supplement (intervals 0.1, widths 0.2) are for a few dozen normalised
    # intervals, while these curves have 1997 intervals of ~5e-4 each, and
    # would leave the value domain (tau < 0 is clamped, widths <= 0 are
    # invalid) within a few steps
    med_tau = float(np.median(b.tau))
    lrs = (0.5, 0.01, 0.02, 0.02 * med_tau, 0.01, 0.01)
    opt = Adam(t, lr=lrs, total_steps=150, ctx=ctx)
    dL = torch.empty_like(target)
    grads = [torch.empty_like(x) for x in t]
    losses = torch.zeros(3, device="cuda")
    reg = Reg(bbox_weight=5.0, bbox_kind=0, deriv_weight=1.0, deriv_order=3, loss=losses[1:])

    def step():
        img = r.run_forward(t, sync=False)
        ctx.check(ctx.lib.nsplat_l2_grad(ctx.h, ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                         ctypes.c_void_p(dL.data_ptr()), ctypes.c_void_p(losses.data_ptr()),
                                         img.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        r.backward(t, dL, reg=reg, grads=grads)
        opt.step(grads)

    s_cap = torch.cuda.Stream()
    s_cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_cap):
        for _ in range(2):
            step()
    torch.cuda.current_stream().wait_stream(s_cap)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    K = args.optim_steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    losses.zero_()
    e0.record()
    for _ in range(K):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    cnt = r.read_counters()
    lv = (losses / K).cpu().numpy().tolist()
    # per-phase times of one eager step (outside the timed region)
    timing_on(ctx, True)
    step()
    torch.cuda.synchronize()
    ph = timing_read(ctx)
    timing_on(ctx, False)
    del g
    res = dict(workload="16 open cubics x 2000 key points, 1024x1024 grayscale, delta_c 10; L2 + derivative "
                        "loss (r = 3) + bounding-box loss, Adam", gaussians=int(cnt[0]), pairs=int(cnt[1]),
               status=int(cnt[2]), ms_per_step=ms, gaussians_per_s=cnt[0] / (ms * 1e-3),
               loss_l2_bbox_deriv=lv, phases_ms={k: v[0] for k, v in ph.items()})
    res["learning_rates"] = list(lrs)
    log("optim step: %d Gaussians, %.3f ms/step (reg %.3f ms), status %d" % (cnt[0], ms, ph["reg"][0], cnt[2]))
    # a step whose curves left the value domain renders nothing and times no work
    if cnt[2] != 0 or cnt[0] == 0:
        raise RuntimeError("optimisation step degenerated: status %d, %d Gaussians" % (cnt[2], cnt[0]))
    return res


def cpu_baseline(b, p, target):
    """The FP64 oracle as it stands, on a bounded sample of the same workload."""
    import oracle
    op = {k: float(np.float32(getattr(p, k))) for k in ("delta_c", "delta_b", "rho", "eta", "gamma", "nl_factor",
                                                        "fill_pad", "h", "alpha_max", "eps_T", "delta_a")}
    op["kappa"] = int(p.kappa)
    op["cutoff"] = float(p.k_sigma)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    g = oracle.gaussians(b, op)
    t_sample = time.perf_counter() - t0
    G = len(g["sigma"])
    H, W = 512, 512
    rows = 256  # the middle half of the image: about 15 s of oracle work on 16 host cores
    y0 = (H - rows) // 2
    pix = np.array([[0, y, x] for y in range(y0, y0 + rows) for x in range(W)], np.int32)
    t0 = time.perf_counter()
    img, T = oracle.composite(b, g, op, pixels=pix)
    t_fwd = time.perf_counter() - t0
    up = 2.0 * (img - target.reshape(3, H, W)[:, y0:y0 + rows, :].transpose(1, 2, 0).reshape(-1, 3))
    t0 = time.perf_counter()
    _, _, adj = oracle.composite(b, g, op, pixels=pix, upstream=up)
    t_bwd_px = time.perf_counter() - t0
    # parameter gradients for a sample of curves
    nc = 128
    seeds = []
    for c in range(nc):
        k0, k1 = b.key_off[c], b.key_off[c + 1]
        t0_, t1_ = b.tau_off[c], b.tau_off[c + 1]
        for k in range(k1 - k0):
            for kind in (1, 2, 3):
                seeds.append((c, kind, k))
        for t in range(t1_ - t0_):
            seeds.append((c, 5, t))
        seeds.append((c, 6, 0))
    t0 = time.perf_counter()
    oracle.param_grad_seeds(b, g, adj, np.array(seeds, np.int32), op)
    t_grad = time.perf_counter() - t0
    est = t_sample + (t_fwd + t_bwd_px) * (H / rows) + t_grad * (b.n_curves / nc)
    log("cpu oracle: sample %.2fs, %d-row composite %.2fs + adjoint %.2fs, %d-curve grads %.2fs -> est %.1fs"
        % (t_sample, rows, t_fwd, t_bwd_px, nc, t_grad, est))
    return dict(value=G / est, unit="Gaussians/s", cores=threads, kind="oracle",
                sample="all %d Gaussians sampled; composite + compositing adjoint on %d of 512 rows (x%d); "
                       "parameter gradients of %d of 256 curves (x%d); measured %.1f s, extrapolated to %.1f s "
                       "per step" % (G, rows, H // rows, nc, b.n_curves // nc,
                                     t_sample + t_fwd + t_bwd_px + t_grad, est))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the render path of this repository runs on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.only == "batched":
        out = bench_batched(args)
    elif args.only == "optim":
        out = bench_optim(args)
    elif args.only == "aniso":
        out = bench_aniso(args)
    else:
        out = bench_main(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
