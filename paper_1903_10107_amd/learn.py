"""Learned offsets for the check node: train per-iteration, per-base-edge
offsets of the differentiable FP32 offset min-sum (the library's forward and
backward kernels) on synthetic frames, quantize them to the integer decoder's
LLR step, and evaluate the integer decoder with them by frame error rate,
efficiency and iterations.

Training inputs are the quantized channel LLRs the integer decoder sees,
scaled back by the quantization step (llr_int * DELTA), so the FP32 model
learns on the integer decoder's input grid; the integer offset table is then
round(beta / DELTA), clamped to [0, msg_max].
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import binding as B
from . import inputs as I
from . import metrics as M


@dataclass
class TrainResult:
    beta: np.ndarray            # [T, n_blocks] FP32 offsets (LLR units)
    offsets: np.ndarray         # [T, n_blocks] int8 offsets (integer LLR steps)
    losses: list                # mean loss per step
    steps: int
    frames_per_step: int
    seconds: float
    ms_per_step: float          # forward + backward + update, GPU time per step


def int_offsets(beta: np.ndarray, msg_max: int = 63, delta: float = I.DELTA) -> np.ndarray:
    """Offsets in integer LLR steps: round(beta / delta) clamped to [0, msg_max]."""
    return np.clip(np.rint(np.asarray(beta, dtype=np.float64) / delta), 0, msg_max).astype(np.int8)


def training_llr(fr: I.Frames, delta: float = I.DELTA) -> np.ndarray:
    """The integer decoder's view of the channel, in LLR units."""
    return fr.llr.astype(np.float32) * np.float32(delta)


def train(code: I.Code, qber: float, n_short: int, *, n_iter: int = 20, frames: int = 512, steps: int = 200,
          lr: float = 0.02, init: float = 0.0, weights=None, seed: int = 4242, log=None) -> TrainResult:
    """Adam on the mean per-frame loss; offsets projected onto beta >= 0 after
    every step; fresh seeded frames every step."""
    import torch
    dec = B.OmsDecoder(code.base, code.z, n_iter, weights)
    beta = torch.full((n_iter, code.n_blocks), float(init), dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([beta], lr=lr)
    losses = []
    gpu_ms = 0.0
    t0 = time.time()
    for step in range(steps):
        fr = I.make_frames(code, frames, qber, seed, n_short=n_short, frame_offset=step * frames)
        syn = torch.from_numpy(fr.syn).cuda()
        llr = torch.from_numpy(training_llr(fr)).cuda()
        xb = torch.from_numpy(I.pack_bits(fr.x)).cuda()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        opt.zero_grad(set_to_none=True)
        loss = dec.loss(syn, llr, xb, beta).mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            beta.clamp_(min=0.0)
        b.record()
        torch.cuda.synchronize()
        gpu_ms += a.elapsed_time(b)
        losses.append(float(loss.detach()))
        if log and (step % 20 == 0 or step == steps - 1):
            log(f"step {step:4d} loss {losses[-1]:.5f} mean beta {float(beta.mean()):.4f}")
    bt = beta.detach().cpu().numpy()
    return TrainResult(beta=bt, offsets=int_offsets(bt), losses=losses, steps=steps, frames_per_step=frames,
                       seconds=time.time() - t0, ms_per_step=gpu_ms / max(steps, 1))


def evaluate(code: I.Code, qber: float, n_short: int, *, max_iter: int, frames: int = 4096, seed: int = 777,
             cn_rule: int = B.LDPC_RULE_RCBP_FB, offsets=None) -> dict:
    """Frame error rate, efficiency and iterations of the integer decoder."""
    fr = I.make_frames(code, frames, qber, seed, n_short=n_short)
    gc = B.Code(code.base, code.z, cn_rule=cn_rule, offsets=offsets)
    out = B.decode(gc, fr.syn, fr.llr, max_iter)
    ok, und = M.frame_outcomes(fr.x, I.unpack_bits(out["bits"], code.n), out["conv"])
    fails = int(frames - ok.sum())
    return {"frames": frames, "fer": fails / frames, "fer_ci95": [round(v, 5) for v in M.wilson_interval(fails, frames)],
            "undetected": int(und.sum()), "mean_iters": float(out["iters"].mean()),
            "efficiency_f": float(np.mean(M.efficiency(code.n, code.m, fr.n_punct, fr.n_short, fr.qber))),
            "kernel": gc.plan()["kernel"]}


def evaluate_fp32(code: I.Code, qber: float, n_short: int, beta, *, n_iter: int, frames: int = 4096,
                  seed: int = 777, batch: int = 512) -> dict:
    """Frame error rate of the FP32 offset min-sum itself (hard decisions of the
    soft values after n_iter iterations, no early stop) on the training grid."""
    import torch
    dec = B.OmsDecoder(code.base, code.z, n_iter)
    bt = torch.as_tensor(np.asarray(beta), dtype=torch.float32).cuda()
    fails = 0
    for f0 in range(0, frames, batch):
        nb = min(batch, frames - f0)
        fr = I.make_frames(code, nb, qber, seed, n_short=n_short, frame_offset=f0)
        _, E = dec.loss(torch.from_numpy(fr.syn).cuda(), torch.from_numpy(training_llr(fr)).cuda(),
                        torch.from_numpy(I.pack_bits(fr.x)).cuda(), bt, want_E=True)
        bits = (E < 0).to(torch.uint8).cpu().numpy()
        fails += int((bits != fr.x).any(axis=1).sum())
    return {"frames": frames, "fer": fails / frames,
            "fer_ci95": [round(v, 5) for v in M.wilson_interval(fails, frames)]}
