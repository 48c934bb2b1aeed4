"""Learned restoration of decoded viewports: training data from the codec,
training on the GPU, evaluation against the uncompressed frames.

The pairs are produced by the codec itself: seeded synthetic YUV420 frames
(wvinputs), encoded at a coarse quantisation step and decoded (the input),
and encoded at step 1 -- lossless for the integer 5/3 transform -- and decoded
(the target).  Both sides go through the same colour conversion, so the
network learns to undo quantisation only.  Every step (encode, decode,
crops, forward, backward, Adam, restore with its guard) runs in libwv.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import wvinputs
from . import cnn
from . import wv


def init_params(seed):
    """He-normal weights, zero biases; the last layer is scaled down so the
    network starts close to the identity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for li, (ci, co) in enumerate(cnn.LAYERS):
        w = rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), (co, 3, 3, ci))
        if li == len(cnn.LAYERS) - 1:
            w *= 0.1
        parts += [w, np.zeros(co)]
    return cnn.flatten(parts)


def make_pairs(n, seed, tiles=4, tile=512, levels=5, step=16):
    """n viewports of tiles x tiles tiles: (decoded at `step`, lossless) as
    device uint8 [n][tiles * tiles][3][tile][tile] (tile-planar RGB)."""
    W = H = tiles * tile
    dec = wv.Decoder(W, H, tile, levels, wv.W53, wv.YUV420)
    nt = tiles * tiles
    mask = np.ones(nt, np.uint8)
    out_dec = torch.empty((n, nt, 3, tile, tile), dtype=torch.uint8, device="cuda")
    out_ref = torch.empty_like(out_dec)
    coef = [torch.empty(dec.plane_shape(p), dtype=torch.int16, device="cuda") for p in range(3)]
    ref = wv.Reference(dec)                 # intra frames only: never read
    for i in range(n):
        spec = wvinputs.FrameSpec(W, H, tile, wvinputs.derive_seed(seed, "restore", i))
        src = [p.reshape(dec.plane_shape(k)) for k, p in
               enumerate(wvinputs.source_planes(spec, device="cuda"))]
        for q, dst in ((step, out_dec[i]), (1, out_ref[i])):
            dec.encode_intra(src, coef, q)
            dec.decode_viewport(coef, 0, True, q, mask, ref, dst)
    torch.cuda.synchronize()
    return out_dec, out_ref


def train(net, decoded, original, steps, batch=16, crop=128, lr=2e-3, seed=0, tiles=4, tile=512,
          log_every=0):
    """Adam on random crops of the pairs; lr follows a cosine decay.  Returns
    the loss of the first and the last logged steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = decoded.shape[0]
    side = tiles * tile
    first = last = None
    for s in range(1, steps + 1):
        crops = np.stack([rng.integers(0, n, batch), rng.integers(0, side - crop + 1, batch),
                          rng.integers(0, side - crop + 1, batch)], axis=1)
        x = net.gather(decoded, tile, tiles, tiles, crops, crop, False)
        t = net.gather(original, tile, tiles, tiles, crops, crop, True)
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * (s - 1) / steps))
        loss = net.train_step(x, t, lr_s, s)
        if s == 1 or s == steps or (log_every and s % log_every == 0):
            v = float(loss.item())
            first = v if first is None else first
            last = v
    return first, last


def psnr(a, b):
    """PSNR in dB of two uint8 tensors."""
    mse = torch.mean((a.float() - b.float()) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


def evaluate(net, decoded, original, guard, tiles=4, tile=512):
    """Mean PSNR of the plain decode and of the restored viewports against the
    uncompressed ones, and the fraction of tiles that fell back."""
    p_dec, p_res, fell = [], [], 0
    for i in range(decoded.shape[0]):
        restored, f = net.restore(decoded[i], tile, tiles, tiles, guard)
        fell += f
        p_dec.append(psnr(decoded[i], original[i]))
        p_res.append(psnr(restored, original[i]))
    n_tiles = decoded.shape[0] * tiles * tiles
    return {"psnr_decoded_db": float(np.mean(p_dec)), "psnr_restored_db": float(np.mean(p_res)),
            "psnr_gain_db": float(np.mean(p_res) - np.mean(p_dec)), "fallback_rate": fell / n_tiles}


def run(n_train=2000, n_eval=16, steps=1500, batch=16, crop=128, seed=10859, guard=0.05,
        tiles=4, tile=512, log=None):
    """The whole experiment: pairs, training, evaluation, timings."""
    t0 = time.perf_counter()
    dec_tr, ref_tr = make_pairs(n_train, seed, tiles, tile)
    dec_ev, ref_ev = make_pairs(n_eval, seed + 1, tiles, tile)
    t1 = time.perf_counter()
    net = cnn.Net(max(batch * crop * crop, tiles * tile * tiles * tile))
    net.set_params(init_params(seed))
    first, last = train(net, dec_tr, ref_tr, steps, batch, crop, seed=seed, tiles=tiles, tile=tile)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res = evaluate(net, dec_ev, ref_ev, guard, tiles, tile)
    t3 = time.perf_counter()
    px = steps * batch * crop * crop
    res.update({"pairs": n_train, "eval_pairs": n_eval, "viewport": f"{tiles * tile}x{tiles * tile}x3",
                "step": 16, "train_steps": steps, "batch": f"{batch}x{crop}x{crop}",
                "loss_first": first, "loss_last": last, "pairs_s": t1 - t0, "train_s": t2 - t1,
                "train_mpix_s": px / (t2 - t1) / 1e6, "eval_s": t3 - t2, "guard": guard})
    net.close()
    return res
