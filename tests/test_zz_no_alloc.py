"""nsplat_udf_loss_noalloc (scratch in the library's static device array)
against nsplat_udf_loss (scratch in the workspace), through the C ABI, on two
calls in a row, the second with a smaller input."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import oracle_params
from paper_2606_31764_amd import synth
from paper_2606_31764_amd.render import Params

pytestmark = pytest.mark.gpu


def _case(batch, p, seed, selected):
    import torch
    from paper_2606_31764_amd.render import Renderer, param_tensors
    r = Renderer(batch, p)
    t = param_tensors(batch)
    img = r.run_forward(t).clone()
    rng = np.random.default_rng(seed)
    tgt = torch.as_tensor(rng.uniform(0, 1, img.numel()).astype(np.float32), device="cuda")
    sel = None
    if selected:
        sel = torch.as_tensor((rng.uniform(size=batch.n_curves) < 0.6).astype(np.int32), device="cuda")
    return r, t, img, tgt, sel


def _both(r, t, img, tgt, sel, tau):
    import torch
    loss_a = torch.zeros(1, device="cuda")
    loss_b = torch.zeros(1, device="cuda")
    da = r.udf_loss(t, img, tgt, tau=tau, sel=sel, loss=loss_a)
    db = r.udf_loss(t, img, tgt, tau=tau, sel=sel, loss=loss_b, noalloc=True)
    torch.cuda.synchronize()
    return da.cpu().numpy(), db.cpu().numpy(), float(loss_a.item()), float(loss_b.item())


def _close(da, db, la, lb):
    # the per-scene sums are FP64 atomics in either form, so the weights agree
    # to rounding; dL/dImage is stored in FP32
    assert np.abs(db - da).max() <= 1e-6 * np.abs(da).max() + 1e-12
    assert abs(lb - la) <= 1e-6 * abs(la) + 1e-12
    assert np.abs(da).max() > 0 and la > 0


def test_noalloc_udf_loss_matches_workspace_form_twice():
    p = Params().replace(delta_c=2.0, h=2.0)
    big = synth.concat([synth.config3(seed=6100, n_paths=6, size=80), synth.config2(seed=6101, n_curves=2, size=40),
                        synth.config3(seed=6102, n_paths=4, size=56)])
    small = synth.config3(seed=6103, n_paths=3, size=40)
    r1, t1, img1, tgt1, sel1 = _case(big, p, 6104, selected=True)
    _close(*_both(r1, t1, img1, tgt1, sel1, tau=8.0))
    # second call, smaller input: one scene where the first had three, so
    # the array still holds the first call's sums beyond the first slots
    r2, t2, img2, tgt2, sel2 = _case(small, p, 6105, selected=False)
    _close(*_both(r2, t2, img2, tgt2, sel2, tau=6.0))
    # and the larger one again after the smaller
    _close(*_both(r1, t1, img1, tgt1, sel1, tau=8.0))


def test_noalloc_rejects_too_many_scenes():
    """More scenes than the static array holds is an argument error (checked on
    the host before any device work)."""
    from paper_2606_31764_amd import _lib as L
    from paper_2606_31764_amd.render import Renderer, param_tensors
    import torch
    b = synth._assemble([], [[8, 8]] * 4096, [[1.0, 1.0, 1.0]] * 4096, 3)
    r = Renderer(b, Params())
    t = param_tensors(b)
    img = r.run_forward(t).clone()
    with pytest.raises(L.NSplatError, match="at most 4095 scenes"):
        r.udf_loss(t, img, torch.zeros_like(img), tau=4.0, noalloc=True)
    # the workspace form takes them
    r.udf_loss(t, img, torch.zeros_like(img), tau=4.0)
    torch.cuda.synchronize()
