"""The torch.autograd path (render() -> loss.backward()) against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from helpers import IMG_TOL, grad_check, oracle_params, oracle_reference
from paper_2606_31764_amd import synth

pytestmark = pytest.mark.gpu


def _setup(batch, prm):
    import torch
    from paper_2606_31764_amd.render import Params, Renderer, param_tensors
    p = Params().replace(**prm)
    op = oracle_params(p)
    target = oracle.render(synth.perturbed(batch, 9), op)[0]
    r = Renderer(batch, p)
    return r, p, op, target, torch.as_tensor(np.asarray(target, np.float32), device="cuda")


@pytest.mark.parametrize("name", ["strokes", "fills"])
def test_loss_backward_matches_oracle(name):
    import torch
    from paper_2606_31764_amd.render import param_tensors, render
    if name == "strokes":
        b, prm = synth.config2(seed=2701, n_curves=6, size=64), dict(delta_c=3.0)
    else:
        b = synth._assemble(synth.fills(2702, n_paths=8, size=72, radius=(4.0, 20.0)), [[72, 72]],
                            [[1.0, 1.0, 1.0]], 3)
        prm = dict(h=1.5)
    r, p, op, target, tgt = _setup(b, prm)
    ref_img, up, gref, scale = oracle_reference(b, target, op)
    ts = param_tensors(b, requires_grad=True)
    img = render(r, *ts)
    # a loss whose dL/dImage is the oracle's L2 gradient, so that both sides
    # differentiate the same function
    loss = (img * torch.as_tensor(up.astype(np.float32), device="cuda")).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert np.abs(img.detach().cpu().numpy() - ref_img).max() <= IMG_TOL
    got = dict(zip(("key_xy", "key_w", "key_s", "tau", "color", "opacity"), [t.grad.cpu().numpy() for t in ts]))
    worst, rep = grad_check(got, gref, scale)
    assert worst <= 1.0, rep


def test_frozen_groups_get_no_gradient():
    """Weights and knot intervals held fixed (requires_grad False, the ablations
    of Table 1): their .grad stays None and the other groups are unchanged."""
    import torch
    from paper_2606_31764_amd.render import param_tensors, render
    b = synth.config2(seed=2703, n_curves=5, size=64)
    r, p, op, target, tgt = _setup(b, dict(delta_c=3.0))
    full = param_tensors(b, requires_grad=True)
    ((render(r, *full) - tgt) ** 2).sum().backward()
    part = list(param_tensors(b, requires_grad=True))
    part[1].requires_grad_(False)
    part[3].requires_grad_(False)
    ((render(r, *part) - tgt) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert part[1].grad is None and part[3].grad is None
    for i in (0, 2, 4, 5):
        np.testing.assert_allclose(part[i].grad.cpu().numpy(), full[i].grad.cpu().numpy(), rtol=1e-5, atol=1e-6)


def test_backward_after_another_forward_raises():
    from paper_2606_31764_amd.render import param_tensors, render
    b = synth.config2(seed=2704, n_curves=4, size=48)
    r, p, op, target, tgt = _setup(b, dict(delta_c=3.0))
    ts = param_tensors(b, requires_grad=True)
    loss1 = ((render(r, *ts) - tgt) ** 2).sum()
    loss2 = ((render(r, *ts) - tgt) ** 2).sum()
    with pytest.raises(RuntimeError, match="another forward"):
        loss1.backward()
    loss2.backward()  # the latest forward's node still works
    assert ts[0].grad is not None and np.all(np.isfinite(ts[0].grad.cpu().numpy()))
