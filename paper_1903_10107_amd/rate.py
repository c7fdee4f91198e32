"""Rate adaptation of one mother code to a QBER (Sec. 4.1): choose how many
positions to puncture or shorten so that the frame error rate stays at or below
a target.

The split is one signed knob kappa: kappa > 0 punctures kappa positions (rate
up), kappa < 0 shortens -kappa positions (rate down); positions come from the
code's candidate order (ascending column weight, ties by a seeded permutation),
punctured first. The frame error rate grows with kappa, so a bisection over
kappa, decoding a fixed seeded batch on the GPU at every probe, finds the
largest kappa that meets the target to within a step. Efficiency and effective
rate follow the rate-adaptive convention f = (1 - R_eff) / h(q) with
R_eff = (k - s) / (n - p - s).
"""
from __future__ import annotations

from dataclasses import asdict, dataclass

import numpy as np

from . import binding as B
from . import inputs as I
from . import metrics as M


@dataclass
class OperatingPoint:
    qber: float
    n_punct: int
    n_short: int
    fer: float
    fer_ci95: tuple
    frames: int
    r_eff: float
    efficiency: float
    mean_iters: float

    def as_dict(self):
        return asdict(self)


def split(kappa: int) -> tuple[int, int]:
    """(n_punct, n_short) of knob value kappa."""
    return (int(kappa), 0) if kappa >= 0 else (0, int(-kappa))


def measure(code: I.Code, gcode: B.Code, base_frames: I.Frames, kappa: int, max_iter: int,
            order: np.ndarray) -> tuple[float, float, int]:
    """(FER, mean iterations, failures) of the batch at knob value kappa."""
    p, s = split(kappa)
    fr = I.adapt_rate(base_frames, p, s, order)
    out = B.decode(gcode, fr.syn, fr.llr, max_iter)
    ok, _ = M.frame_outcomes(fr.x, I.unpack_bits(out["bits"], code.n), out["conv"])
    fails = int(fr.n_frames - ok.sum())
    return fails / fr.n_frames, float(np.mean(out["iters"])), fails


def search(code: I.Code, qber: float, *, frames: int = 2048, max_iter: int = 60, fer_target: float = 1e-2,
           step: int = 256, seed: int = 1903_10107, acc_bits: int = 0, log=None, **code_kw) -> OperatingPoint:
    """Largest kappa (to within step) whose batch FER is at most fer_target.
    code_kw (cn_rule, offsets, ...) configures the integer decoder evaluated."""
    gcode = B.Code(code.base, code.z, acc_bits=acc_bits, **code_kw)
    order = I.position_order(code)
    base = I.make_frames(code, frames, qber, seed)
    k = code.n - code.m
    cache = {}

    def fer(kappa):
        if kappa not in cache:
            cache[kappa] = measure(code, gcode, base, kappa, max_iter, order)
            if log:
                log(f"  q={qber} kappa={kappa} {split(kappa)} fer={cache[kappa][0]:.4f} "
                    f"iters={cache[kappa][1]:.2f}")
        return cache[kappa][0]

    if fer(0) <= fer_target:
        lo, hi = 0, k - 1                    # puncture: FER(lo) ok, FER(hi) presumed not
        if fer(hi) <= fer_target:
            lo = hi
    else:
        lo, hi = -(k - 1), 0                 # shorten
        if fer(lo) > fer_target:
            raise RuntimeError(f"no operating point at QBER {qber}: FER {fer(lo)} with {k - 1} shortened")
    while hi - lo > step:
        mid = (lo + hi) // 2
        if fer(mid) <= fer_target:
            lo = mid
        else:
            hi = mid
    f_, iters, fails = cache[lo] if lo in cache else measure(code, gcode, base, lo, max_iter, order)
    p, s = split(lo)
    r_eff = M.effective_rate(code.n, code.m, p, s)
    return OperatingPoint(qber=qber, n_punct=p, n_short=s, fer=f_,
                          fer_ci95=tuple(round(v, 5) for v in M.wilson_interval(fails, frames)), frames=frames,
                          r_eff=float(r_eff), efficiency=float(M.efficiency(code.n, code.m, p, s, qber)),
                          mean_iters=iters)


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="operating points of a mother code by bisection on the GPU decoder")
    ap.add_argument("--base", default="24x48", help="MbxNb of the seeded QC base (column weight 3)")
    ap.add_argument("--z", type=int, default=2048)
    ap.add_argument("--qber", default="0.01,0.02,0.04,0.06,0.08")
    ap.add_argument("--frames", type=int, default=2048)
    ap.add_argument("--max-iter", type=int, default=60)
    ap.add_argument("--fer", type=float, default=1e-2)
    ap.add_argument("--step", type=int, default=128)
    args = ap.parse_args()
    mb, nb = (int(v) for v in args.base.split("x"))
    code = I.Code(I.make_base(mb, nb, args.z), args.z)
    out = []
    for q in (float(v) for v in args.qber.split(",")):
        op = search(code, q, frames=args.frames, max_iter=args.max_iter, fer_target=args.fer, step=args.step,
                    log=lambda m: print(m, flush=True))
        print(json.dumps(op.as_dict()), flush=True)
        out.append(op.as_dict())
    print(json.dumps({"code": f"{args.base} Z={args.z}", "points": out}), flush=True)


if __name__ == "__main__":
    main()
