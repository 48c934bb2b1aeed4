"""Restoration network on the GPU (bfloat16 MFMA kernels) against the float64
oracle, and the trained network's gain over the plain decode.

Tolerances: the GPU rounds its input, weights and the activations and
backward signals between layers to bfloat16 exactly where the oracle does
(``round_acts``); what remains is fp32 against fp64 accumulation, which can
flip a bfloat16 rounding (one unit in the last place, 2^-8 relative) of a
value next to a rounding boundary.  Forward outputs must agree to 1e-4 for
99.9 % of the values and to 2e-3 (scaled by the output range) everywhere;
gradients to 2e-4 in relative L2 norm per tensor (measured: at most 1.1e-5,
where a few bfloat16 roundings flip; about 1e-7 otherwise) and the loss to
1e-5 relative.
"""
import numpy as np
import pytest
import torch

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def _mods():
    from paper_2208_10859_amd import cnn, restore
    return cnn, restore


def _case(seed, shape):
    """Input, target and parameters, all bfloat16-representable where the GPU
    stores bfloat16 (inputs and weights; biases stay fp32)."""
    rng = np.random.default_rng(seed)
    x = ocnn.bf16(rng.uniform(0, 1, shape + (3,)))
    t = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1)
    params = ocnn.init_params(seed)
    for i in range(0, 8, 2):
        params[i] = ocnn.bf16(params[i] * (10.0 if i == 6 else 1.0))
    for i in range(1, 8, 2):
        params[i] = rng.normal(0, 0.05, params[i].shape)
    return x, t, params


def _dev_x(x):
    n, h, w, _ = x.shape
    x4 = np.zeros((n, h, w, 4), np.float32)
    x4[..., :3] = x
    return torch.from_numpy(x4).to(torch.bfloat16).cuda()


def _dev_t(t):
    n, h, w, _ = t.shape
    t4 = np.zeros((n, h, w, 4), np.float32)
    t4[..., :3] = t
    return torch.from_numpy(t4).cuda()


@pytest.mark.parametrize("shape", [(2, 19, 45), (1, 8, 32), (1, 33, 7)])
def test_forward_matches_oracle(shape):
    cnn, _ = _mods()
    x, t, params = _case(21 + shape[1], shape)
    net = cnn.Net(int(np.prod(shape)))
    net.set_params(cnn.flatten(params))
    z = torch.zeros(shape + (4,), dtype=torch.float32, device="cuda")
    net.forward(_dev_x(x), z)
    torch.cuda.synchronize()
    got = z.cpu().numpy()
    _, want, _ = ocnn.forward(x, params, round_acts=True)
    assert np.all(got[..., 3] == 0)
    err = np.abs(got[..., :3] - want)
    scale = max(1.0, float(np.abs(want).max()))
    assert np.mean(err <= 1e-4 * scale) >= 0.999, float(np.quantile(err, 0.999))
    assert err.max() <= 2e-3 * scale, float(err.max())


@pytest.mark.parametrize("shape", [(2, 16, 40), (1, 21, 33)])
def test_infer_equals_forward(shape):
    # the inference pass runs the same products without keeping activations:
    # bit-identical output, and no backward pass may follow it
    cnn, _ = _mods()
    x, _, params = _case(41 + shape[2], shape)
    net = cnn.Net(int(np.prod(shape)))
    net.set_params(cnn.flatten(params))
    xd = _dev_x(x)
    z1 = torch.zeros(shape + (4,), dtype=torch.float32, device="cuda")
    z2 = torch.full(shape + (4,), 7.0, dtype=torch.float32, device="cuda")
    net.forward(xd, z1)
    net.infer(xd, z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    with pytest.raises(RuntimeError):
        net.loss_grad(torch.zeros(shape + (4,), dtype=torch.float32, device="cuda"))


@pytest.mark.parametrize("shape", [(2, 16, 40), (1, 21, 33), (2, 19, 45)])
def test_gradients_match_oracle(shape):
    cnn, _ = _mods()
    x, t, params = _case(5 + shape[2], shape)
    net = cnn.Net(int(np.prod(shape)))
    net.set_params(cnn.flatten(params))
    net.forward(_dev_x(x))
    loss = net.loss_grad(_dev_t(t))
    grads = torch.zeros(cnn.param_count(), dtype=torch.float32, device="cuda")
    net.backward(grads)
    torch.cuda.synchronize()
    want_loss, want = ocnn.loss_and_grads(x, t, params, round_acts=True)
    assert abs(loss.item() - want_loss) <= 1e-5 * want_loss
    got = cnn.unflatten(grads.cpu().numpy())
    for k, (g, w) in enumerate(zip(got, want)):
        rel = np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-12)
        assert rel <= 2e-4, (k, rel)


def test_guard_falls_back_to_the_plain_decode():
    cnn, restore = _mods()
    dec, _ = restore.make_pairs(1, 3, tiles=2, tile=64, levels=3)
    net = cnn.Net(128 * 128)
    p = cnn.unflatten(restore.init_params(1))
    p[7] = np.full(3, 0.5)                       # z = +0.5 everywhere: above any sane guard
    net.set_params(cnn.flatten(p))
    out, fell = net.restore(dec[0], 64, 2, 2, guard=0.05)
    assert fell == 4 and torch.equal(out, dec[0])
    p[7] = np.zeros(3)
    p[6] = np.zeros_like(p[6])                   # z = 0: identity, kept
    net.set_params(cnn.flatten(p))
    out, fell = net.restore(dec[0], 64, 2, 2, guard=0.05)
    assert fell == 0 and torch.equal(out, dec[0])
    p[7] = np.array([np.nan, 0.0, 0.0])          # non-finite output: falls back
    net.set_params(cnn.flatten(p))
    out, fell = net.restore(dec[0], 64, 2, 2, guard=0.05)
    assert fell == 4 and torch.equal(out, dec[0])


def test_training_gains_over_the_plain_decode():
    """A short training run on codec-made pairs (step 16) lowers the loss and
    raises the PSNR of held-out viewports above the plain decode's."""
    cnn, restore = _mods()
    dec_tr, ref_tr = restore.make_pairs(24, 7, tiles=2, tile=128, levels=4)
    dec_ev, ref_ev = restore.make_pairs(6, 8, tiles=2, tile=128, levels=4)
    net = cnn.Net(16 * 64 * 64 + 256 * 256)
    net.set_params(restore.init_params(7))
    first, last = restore.train(net, dec_tr, ref_tr, steps=1500, batch=16, crop=64, tiles=2,
                                tile=128, log_every=100)
    assert last < 0.85 * first, (first, last)      # one batch each: a noisy measure
    res = restore.evaluate(net, dec_ev, ref_ev, guard=0.05, tiles=2, tile=128)
    # the same PSNR computed by the oracle's definition on one viewport
    r0, _ = net.restore(dec_ev[0], 128, 2, 2, 0.05)
    assert abs(restore.psnr(r0, ref_ev[0]) - ocnn.psnr(r0.cpu().numpy(), ref_ev[0].cpu().numpy())) < 1e-6
    assert res["fallback_rate"] == 0.0
    assert res["psnr_gain_db"] > 0.15, res
