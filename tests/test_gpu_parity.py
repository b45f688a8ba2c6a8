"""GPU path vs the FP64 oracle on the same seeded inputs (staged and end to end).

Sizes are small enough for the brute-force oracle to finish in seconds but
span several tiles with ragged edges (canvases that are not tile multiples).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from helpers import IMG_TOL, grad_close, gpu_run, gpu_vs_oracle, oracle_params, plans_equal
from paper_2606_31764_amd import synth
from paper_2606_31764_amd.render import Params

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "c1": (synth.config1(), Params().replace(delta_c=1.5)),
        "c2s": (synth.config2(seed=2100, n_curves=8, size=120), Params().replace(delta_c=3.0)),
        # the calligraphy configuration at its full size: 32 strokes, 256^2
        "c2_full": (synth.config2(), Params().replace(delta_c=3.0)),
        "c3s_h2": (synth.config3(seed=3100, n_paths=10, size=100), Params().replace(h=2.0)),
        "c3s_h1": (synth.config3(seed=3200, n_paths=6, size=72), Params().replace(h=1.0)),
        "c4s": (synth.config4(seed=4100, n_curves=2, n_cp=60, size=200), Params().replace(delta_c=10.0)),
        # dense cases whose tile lists span several 512-position chunks of the adjoint
        "c3s_dense": (synth.config3(seed=3300, n_paths=10, size=64), Params().replace(h=0.5)),
        "c4s_dense": (synth.config4(seed=4200, n_curves=6, n_cp=120, size=96), Params().replace(delta_c=10.0)),
    }


CASES = _cases()


def _target(name):
    b, p = CASES[name]
    if name == "c1":
        tb = synth.config1(1001)
    else:
        tb = synth.perturbed(b, seed=99)
    return oracle.render(tb, oracle_params(p))[0]


@pytest.mark.parametrize("name", list(CASES))
def test_plan_and_gaussians(name):
    b, p = CASES[name]
    op = oracle_params(p)
    ref = oracle.gaussians(b, op)
    out = gpu_run(b, p, backward=False)
    print(name, "G =", out["counters"][0], "pairs =", out["counters"][1], flush=True)
    assert out["counters"][2] == 0, "status bits %d" % out["counters"][2]
    # counts, sample numbers, fill windows, offsets: bit-exact
    plans_equal(out["plan"], ref["plan"])
    g = out["gauss"]
    assert len(g["sigma"]) == len(ref["sigma"])
    np.testing.assert_array_equal(g["curve"], ref["curve"])
    np.testing.assert_array_equal(g["local"], ref["local"])
    assert np.abs(g["mu"] - ref["mu"]).max() < 1e-9
    np.testing.assert_allclose(g["sigma"], ref["sigma"].astype(np.float32), rtol=2e-7, atol=0)
    assert np.abs(g["opacity"] - ref["opacity"]).max() < 2e-7


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_bin_bitexact(name, tile):
    b, p = CASES[name]
    p = p.replace(tile=tile)
    ref_g = oracle.gaussians(b, oracle_params(p))
    ranges_ref, idx_ref = oracle.bin_gaussians(b, ref_g, tile=tile, k_sigma=p.k_sigma)
    out = gpu_run(b, p, backward=False)
    np.testing.assert_array_equal(out["ranges"], ranges_ref)
    np.testing.assert_array_equal(out["idx"], idx_ref)


@pytest.mark.parametrize("name", list(CASES))
def test_forward_end_to_end(name):
    b, p = CASES[name]
    img_ref, T_ref, _ = oracle.render(b, oracle_params(p))
    out = gpu_run(b, p, backward=False)
    err = np.abs(out["image"] - img_ref).max()
    print(name, "image max abs err", err, flush=True)
    assert err <= IMG_TOL
    assert np.abs(out["T"] - T_ref).max() <= IMG_TOL


@pytest.mark.parametrize("name", list(CASES))
def test_backward_end_to_end(name):
    b, p = CASES[name]
    out, worst, rep = gpu_vs_oracle(b, p, _target(name))
    print(name, "grad worst ratio", worst, rep, flush=True)


@pytest.mark.parametrize("name", ["c2s", "c3s_h2"])
def test_persistent_matches_plain(name):
    b, p = CASES[name]
    target = _target(name)
    a = gpu_run(b, p, target=target, persistent=False)
    c = gpu_run(b, p, target=target, persistent=True)
    np.testing.assert_array_equal(a["image"], c["image"])
    np.testing.assert_array_equal(a["n_last"], c["n_last"])
    assert grad_close(c["grads"], a["grads"], rtol=1e-5, atol=1e-7) <= 1.0


@pytest.mark.parametrize("name", ["c3s_dense", "c4s_dense"])
@pytest.mark.parametrize("tile", [16, 32])
def test_backward_across_chunks(name, tile):
    """Tile lists longer than two 512-position chunks: the adjoint starts the
    later chunks from the forward's stored state, and the gradients still
    match the oracle."""
    b, p = CASES[name]
    p = p.replace(tile=tile)
    out, worst, rep = gpu_vs_oracle(b, p, _target(name))
    lens = out["ranges"][:, 1] - out["ranges"][:, 0]
    print(name, tile, "longest list", int(lens.max()), "grad worst ratio", worst, flush=True)
    assert lens.max() > 2 * 512


def _tile32_case(name):
    if name == "behind_fills_h1":  # strokes behind opaque fills, fill runs walked at h = 1
        from test_gpu_grad_components import behind_fills
        b, p = behind_fills(7102), Params().replace(delta_c=2.0, h=1.0)
    elif name == "c3s_dense_h1":
        b, p = synth.config3(seed=3300, n_paths=10, size=64), Params().replace(h=1.0)
    else:
        b, p = CASES[name]
        return b, p, _target(name)
    return b, p, oracle.render(synth.perturbed(b, seed=97), oracle_params(p))[0]


@pytest.mark.parametrize("name", ["c3s_h1", "c3s_h2", "c3s_dense_h1", "behind_fills_h1"])
def test_backward_tile32_fill_blocks(name):
    """At 32 x 32 tiles a batch with fills takes its adjoint in sixteen 8 x 8
    pixel blocks per tile (fill runs pixel by pixel at h = 1, entry by entry
    otherwise and for strokes), starting from the forward's stored state laid
    out by its 16 x 16 quadrants: image and every gradient component against
    the oracle, lists spanning several chunks in the dense case."""
    b, p, target = _tile32_case(name)
    p = p.replace(tile=32)
    out, worst, rep = gpu_vs_oracle(b, p, target)
    lens = out["ranges"][:, 1] - out["ranges"][:, 0]
    print(name, "longest list", int(lens.max()), "grad worst ratio", worst, rep, flush=True)
    if name == "c3s_dense_h1":
        assert lens.max() > 2 * 512
