"""Interactive reveal-and-retry (Sec. 4.1: puncturing and shortening of one
mother code adapt its rate; a failed decode is followed by Alice revealing the
values of further punctured positions, which then count as shortened, and Bob
decoding again).

Frames keep the canonical layout of the rate-adaptation candidate order
(punctured = its first p positions, shortened = the next s): a round reveals
the last punctured positions first, so after k reveals a frame's LLRs are those
of (p - k, s + k). Each round decodes only the frames that have not converged
(a persistent launch whose decode order lists them, padded with skipped
entries), reveals on the GPU with ldpc_reveal_batch, and stops when every frame
has converged, a round limit is hit, or the failed frames have nothing left to
reveal. Bob only sees convergence (H x^ = s); a converged frame whose word is
not Alice's counts as an undetected error.

Efficiency of a frame with p punctured and s shortened positions at the end:
f = (1 - R_eff) / h(q) with R_eff = (k - s) / (n - p - s), i.e.
(m - p) / ((n - p - s) h(q)): every revealed bit is leaked.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import binding as B
from . import inputs as I
from . import metrics as M


@dataclass
class RetryResult:
    rounds: np.ndarray        # [F] reveal rounds used by each frame
    converged: np.ndarray     # [F] bool
    correct: np.ndarray       # [F] bool: converged to Alice's word
    n_punct: np.ndarray       # [F] final
    n_short: np.ndarray       # [F] final
    efficiency: np.ndarray    # [F] final f
    bits: np.ndarray          # [F, ceil(n/8)] final decisions
    gpu_ms: float             # decode and reveal launches
    wall_s: float
    decoded_frames: int       # frame decodes over all rounds

    def summary(self, code: I.Code, qber) -> dict:
        F = len(self.rounds)
        fails = int(F - self.correct.sum())
        key = (code.n - self.n_punct - self.n_short)[self.correct].sum()
        return {"frames": F, "fer": fails / F, "fer_ci95": [round(v, 5) for v in M.wilson_interval(fails, F)],
                "undetected": int((self.converged & ~self.correct).sum()),
                "mean_rounds": float(self.rounds.mean()), "max_rounds": int(self.rounds.max()),
                "mean_f_success": float(self.efficiency[self.correct].mean()) if self.correct.any() else None,
                "decoded_frames": self.decoded_frames, "gpu_ms": round(self.gpu_ms, 3),
                "mbit_s_gpu": round(float(key) / (self.gpu_ms / 1e3) / 1e6, 2) if self.gpu_ms > 0 else None}


def reveal_plan(order: np.ndarray, n_punct: np.ndarray, ids: np.ndarray, step: int):
    """Positions [k, r] (padded with -1) and counts to reveal for frames ids:
    the last min(step, p) punctured positions of each."""
    kf = np.minimum(step, n_punct[ids]).astype(np.int64)
    r = int(kf.max()) if len(kf) else 0
    pos = np.full((len(ids), max(r, 1)), -1, dtype=np.int32)
    for i, f in enumerate(ids):
        p = int(n_punct[f])
        if kf[i]:
            pos[i, :kf[i]] = order[p - kf[i]:p]
    return pos, kf


def reconcile(code: I.Code, fr: I.Frames, max_iter: int, *, reveal_step: int, max_rounds: int,
              workgroups: int = 512) -> RetryResult:
    """Decode, then reveal and decode the failed frames again, round by round."""
    import torch
    t_wall = time.time()
    gc = B.Code(code.base, code.z)
    persistent = gc.plan()["kernel"] in B.PERSISTENT_FAMILIES
    F, n = fr.n_frames, code.n
    order = I.position_order(code)
    d_syn = torch.from_numpy(fr.syn).cuda()
    d_llr = torch.from_numpy(fr.llr.copy()).cuda()
    d_bits = torch.zeros((F, (n + 7) // 8), dtype=torch.uint8, device="cuda")
    d_conv = torch.zeros(F, dtype=torch.uint8, device="cuda")
    d_iters = torch.zeros(F, dtype=torch.int32, device="cuda")
    wgs = workgroups if persistent else 0
    ws_need = B.ldpc_workspace_bytes_sched(gc, F, wgs)
    d_ws = torch.empty(ws_need, dtype=torch.uint8, device="cuda") if ws_need else None
    p = fr.n_punct.astype(np.int64).copy()
    s = fr.n_short.astype(np.int64).copy()
    rounds = np.zeros(F, dtype=np.int64)
    gpu_ms, decoded = 0.0, 0

    def decode(ids):
        """Decode frames ids (all when None). Without a persistent kernel family
        the whole batch is decoded again; converged frames, whose LLRs did not
        change, give the same result."""
        nonlocal gpu_ms, decoded
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        order_d = None
        if ids is not None and persistent:
            o = np.full(F, F, dtype=np.int32)          # out-of-range entries are skipped
            o[:len(ids)] = ids
            order_d = torch.from_numpy(o).cuda()
        a.record()
        B.ldpc_decode_batch_sched(gc, d_syn, d_llr, F, max_iter, d_bits, d_conv, d_iters,
                                  persistent_workgroups=wgs, order=order_d, workspace=d_ws)
        b.record()
        torch.cuda.synchronize()
        gpu_ms += a.elapsed_time(b)
        decoded += F if ids is None or not persistent else len(ids)

    decode(None)
    for _ in range(max_rounds):
        conv = d_conv.cpu().numpy().astype(bool)
        ids = np.nonzero(~conv & (p > 0))[0].astype(np.int32)
        if len(ids) == 0:
            break
        pos, kf = reveal_plan(order, p, ids, reveal_step)
        vals = np.zeros(pos.shape, dtype=np.uint8)
        ok = pos >= 0
        rows = np.repeat(ids[:, None], pos.shape[1], axis=1)
        vals[ok] = fr.x[rows[ok], pos[ok]]                   # Alice's bits at the revealed positions
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        B.ldpc_reveal_batch(gc, d_llr, F, torch.from_numpy(ids).cuda(), torch.from_numpy(pos).cuda(),
                            torch.from_numpy(vals).cuda())
        b.record()
        torch.cuda.synchronize()
        gpu_ms += a.elapsed_time(b)
        p[ids] -= kf
        s[ids] += kf
        rounds[ids] += 1
        decode(ids)
    conv = d_conv.cpu().numpy().astype(bool)
    bits = d_bits.cpu().numpy()
    correct = conv & (I.unpack_bits(bits, n) == fr.x).all(axis=1)
    eff = M.efficiency(n, code.m, p, s, fr.qber)
    return RetryResult(rounds=rounds, converged=conv, correct=correct, n_punct=p, n_short=s, efficiency=eff,
                       bits=bits, gpu_ms=gpu_ms, wall_s=time.time() - t_wall, decoded_frames=decoded)
