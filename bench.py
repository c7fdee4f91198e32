#!/usr/bin/env python3
"""Throughput of the quantized layered LDPC syndrome decoder on one MI355X.

One step decodes one batch of synthetic frames resident in HBM with one call of
ldpc_decode_batch_ex (one kernel launch). Default workload: 5x32 QC base with
Z = 1024 (n = 32768, design rate 27/32), 256 frames, QBER 2%, a third of the
positions shortened so that the frame error rate is at most 1e-2, 50
iterations. The reported value is corrected-key Mbit/s: the key bits (n minus
shortened positions) of frames decoded to Alice's word, per second of decode
time.

Prints one JSON line with the measurement, the roofline of the decode kernel
(algorithmic bytes: 4 B per edge per iteration with int8 soft values, 6 B with
int16, plus the frame I/O) and the CPU oracle timed on a bounded sample of the
same frames on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "corrected-key Mbit/s at FER≤1e-2, QBER 2%, n=32768 (plain vs batched/learned)"
HBM_PEAK_GBS = 8000.0
# Integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s; the
# decode kernels run packed 16-bit ops (two 8/16-bit operations per lane-op).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# One unpacked 32-bit op per lane per cycle (the offset min-sum kernels: no FMA, no packed FP32).
FP32_ALU_PEAK_TOPS = round(256 * 4 * 16 * 2.4e9 / 1e12, 1)


def algorithmic_int_ops(code_dims, iters_sum):
    """Integer operations the method performs per decode, independent of the
    implementation: per edge and iteration Eq. 8 with saturation (3), sign parity
    (1), magnitude and clip (2), message sign (2), Eq. 9 with saturation (3) and the
    Alg. 2 test (3) = 14; per check row of degree d, 3(d - 2) evaluations of Alg. 1
    at 9 operations each (forward-backward fold)."""
    z, degs = code_dims
    n_edges = z * sum(degs)
    per_iter = 14 * n_edges + 27 * z * sum(d - 2 for d in degs)
    return float(per_iter) * float(iters_sum)
# Least shortening of the n = 32768 code at QBER 2% with FER <= 1e-2: the
# bisection of paper_1903_10107_amd.rate (2048 frames per probe, 256-position
# steps) ends at 9720 shortened positions (29.7%).
I_LEAST_SHORT = 9720
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1903_10107_amd", "csrc")


# Decode kernel of each family (the symbol rocprofv3 reports) and the sources it
# is compiled from.
KERNEL_SYMBOLS = {"split_reg": "k_decode_frame_reg", "split": "k_decode_frame_split",
                  "split_global_l": "k_decode_frame_split", "pairs": "k_decode_frame_x2", "lds": "k_decode_frame",
                  "global": "k_decode_frame", "layer_sync": "k_multi_layer"}
KERNEL_SOURCES = {"split_reg": ("decode_reg.hip", "split_common.hpp", "kernels.hpp", "rcbp.hpp", "decoder.hpp",
                                "qc_code.hpp"),
                  "split": ("decode_split.hip", "split_common.hpp", "kernels.hpp", "rcbp.hpp", "decoder.hpp",
                            "qc_code.hpp")}
HEADLINE_FAMILY = "split_reg"


def kernel_source_hash(family: str = HEADLINE_FAMILY) -> str:
    """Hash of the sources the headline decode kernel is built from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[family]:
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_summary(workload: str) -> dict:
    """The "key: value" lines of the committed rocprofv3 counter summary of a
    workload (empty when there is none)."""
    path = os.path.join(PROFILES, f"decode_{workload}_traffic.txt")
    kv = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    kv = traffic_summary(workload)
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline_large(seconds: float):
    """The oracle on the n = 2^20 workload (10x64 base, Z = 16384, 16-bit soft
    values, QBER 2% unshortened, 80 iterations: every frame runs all of them), a
    bounded sample of frames, one per thread: frame-iterations per second, the
    unit the GPU figure reports beside it."""
    import numpy as np
    import oracle as O
    from paper_1903_10107_amd import inputs as I

    wl = I.WORKLOADS["n1048576_q2"]
    code = wl.code()
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    threads = max(1, min(threads, O.max_threads()))
    fr = I.make_frames(code, threads, wl.qber, 10107)
    # a shorter iteration limit keeps the sample bounded (QBER 2% unshortened runs
    # every iteration, so the work per iteration is fixed): two iterations
    # calibrate the count that fills the requested time
    t = time.perf_counter()
    O.decode(code.base, code.z, fr.syn, fr.llr, 2, acc_bits=wl.acc_bits, n_threads=threads)
    it = max(2, min(wl.max_iter, int(2 * seconds / max(time.perf_counter() - t, 1e-3))))
    t = time.perf_counter()
    r = O.decode(code.base, code.z, fr.syn, fr.llr, it, acc_bits=wl.acc_bits, n_threads=threads)
    el = time.perf_counter() - t
    fi = float(np.sum(r["iters"]))
    return {"frame_iterations_per_s": round(fi / el, 2), "cores": threads, "kind": "oracle",
            "sample": f"{threads} frames of n = {code.n}, {it} iterations each ({fi:.0f} frame-iterations, "
                      f"{el:.1f} s, one frame per OpenMP thread)"}


def cpu_baseline(code, fr, wl, seconds: float):
    import numpy as np
    import oracle as O
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    threads = max(1, min(threads, O.max_threads() if threads <= 0 else threads))
    done, bits_ok, elapsed, passes = 0, 0, 0.0, 0
    # whole chunks of `threads` frames, cycling over the batch until `seconds` of decoding
    while elapsed < seconds:
        start = done % fr.n_frames
        sl = slice(start, min(start + threads, fr.n_frames))
        t = time.perf_counter()
        r = O.decode(code.base, code.z, fr.syn[sl], fr.llr[sl], wl.max_iter, acc_bits=wl.acc_bits,
                     n_threads=threads)
        elapsed += time.perf_counter() - t
        ok, _ = M.frame_outcomes(fr.x[sl], I.unpack_bits(r["bits"], code.n), r["conv"])
        bits_ok += int(fr.key_bits()[sl][ok].sum())
        done += sl.stop - sl.start
    # the same oracle on one thread, over a smaller sample (a few frames)
    t1, ok1, n1 = 0.0, 0, 0
    while t1 < min(3.0, seconds / 4):
        sl = slice(n1 % fr.n_frames, n1 % fr.n_frames + 1)
        t = time.perf_counter()
        r = O.decode(code.base, code.z, fr.syn[sl], fr.llr[sl], wl.max_iter, acc_bits=wl.acc_bits, n_threads=1)
        t1 += time.perf_counter() - t
        ok, _ = M.frame_outcomes(fr.x[sl], I.unpack_bits(r["bits"], code.n), r["conv"])
        ok1 += int(fr.key_bits()[sl][ok].sum())
        n1 += 1
    return {"value": round(bits_ok / elapsed / 1e6, 3), "unit": "Mbit/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "build": "gcc -O3, OpenMP over frames, no intrinsics",
            "sample": f"{done} frame decodes cycling over the {fr.n_frames} frames of the same workload "
                      f"(oracle, {threads} OpenMP threads over frames, {elapsed:.1f} s of decoding)",
            "single_thread": {"value": round(ok1 / t1 / 1e6, 3), "unit": "Mbit/s", "cores": 1,
                              "sample": f"{n1} frame decodes of the same batch on one thread, {t1:.1f} s"}}


def copy_calibration(nbytes: int, steps: int, warmup: int):
    """A plain device-to-device copy of a known size: its FETCH_SIZE and
    WRITE_SIZE counters give the factor that turns counter readings into bytes."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    print(json.dumps({"copy_bytes": nbytes, "ms_per_copy": round(ms, 4),
                      "read_plus_write_GBs": round(2 * nbytes / (ms / 1e3) / 1e9, 1)}), flush=True)


def fer_sweep(wl, code, fracs, n_frames: int, qbers=None):
    """Frame error rate, iterations and efficiency at several shortened
    fractions of the workload's code, at its QBER or at each of qbers,
    decoding n_frames per point."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    torch.cuda.set_device(0)
    gc = B.Code(code.base, code.z, acc_bits=wl.acc_bits)
    for q, frac in [(q, f) for q in (qbers or [wl.qber]) for f in fracs]:
        ns = int(round(frac * code.n))
        fr = I.make_frames(code, n_frames, q, 777, n_short=ns)
        got = B.decode(gc, fr.syn, fr.llr, wl.max_iter)
        ok, und = M.frame_outcomes(fr.x, I.unpack_bits(got["bits"], code.n), got["conv"])
        fails = int(n_frames - ok.sum())
        lo, hi = M.wilson_interval(fails, n_frames)
        f_eff = float(np.mean(M.efficiency(code.n, code.m, fr.n_punct, fr.n_short, fr.qber)))
        print(json.dumps({"workload": wl.name, "qber": q, "short_frac": frac, "shortened": ns, "frames": n_frames,
                          "fer": fails / n_frames, "fer_ci95": [round(lo, 5), round(hi, 5)],
                          "undetected": int(und.sum()), "mean_iters": round(float(got["iters"].mean()), 3),
                          "p99_iters": float(np.percentile(got["iters"], 99)),
                          "efficiency_f": round(f_eff, 4)}), flush=True)


def batched(wl, code, n_short, n_frames, steps, warmup):
    """The same workload with many batches decoded per launch, under the fastest
    of a few frame schedules (one workgroup per frame, or persistent workgroups
    pulling frames from a queue, as given or with the frames whose hard decision
    fails the most checks first, that order computed on the GPU inside every
    timed step); the schedule is picked by the autotuner."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M
    from paper_1903_10107_amd import tune

    fr = I.make_frames(code, n_frames, wl.qber, 10107, n_short=n_short)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cands = [tune.Schedule("auto", 0, "none", False)]
    for fam in ("split_reg", "split"):
        cands += [tune.Schedule(fam, n_cu, "none", False), tune.Schedule(fam, 2 * n_cu, "none", True),
                  tune.Schedule(fam, n_cu, "unsat_first", True), tune.Schedule(fam, 2 * n_cu, "unsat_first", True)]
    best = tune.tune(code.base, code.z, fr.syn, fr.llr, wl.max_iter, acc_bits=wl.acc_bits, cache_path=None,
                     cands=cands, reps=2)
    sched = tune.Schedule(**best["schedule"])
    run = tune.Runner(code.base, code.z, fr.syn, fr.llr, wl.max_iter, sched, acc_bits=wl.acc_bits)
    ms = tune.time_ms(run, max(3, steps // 5), max(1, warmup))
    bits, conv, iters = run.outputs()
    correct, undetected = M.frame_outcomes(fr.x, I.unpack_bits(bits, code.n), conv)
    value = float(fr.key_bits()[correct].sum()) / (ms / 1e3) / 1e6
    degs = [int((code.base[b] >= 0).sum()) for b in range(code.mb)]
    tops = algorithmic_int_ops((code.z, degs), iters.sum()) / (ms / 1e3) / 1e12
    return {"value": round(value, 2), "unit": "Mbit/s", "frames_per_launch": n_frames,
            "ms_per_launch": round(ms, 4), "schedule": best["schedule"],
            "schedules_tried": best["candidates"], "alu_frac": round(tops / ALU_PEAK_TOPS, 4),
            "fer": round(float(n_frames - correct.sum()) / n_frames, 5),
            "undetected_errors": int(undetected.sum()), "mean_iters": round(float(iters.mean()), 3)}


def small_frames(batches, steps, warmup):
    """Short frames: the n = 1024 workload (5x32 base, Z = 32, QBER 1%, 50
    iterations), 64 frames as configured and larger batches for throughput,
    under the autotuner with the frames-per-workgroup axis (a frame is 32 lanes:
    two frames per wave, 1 to 16 waves per workgroup, no workgroup barrier)
    against one frame per 64-thread workgroup."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M
    from paper_1903_10107_amd import tune

    wl = I.WORKLOADS["n1024_q1"]
    code = wl.code()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"workload": wl.name, "code": "5x32 QC base, Z=32, column weight 3 (n=1024)", "qber": wl.qber,
           "max_iter": wl.max_iter}
    for F in batches:
        fr = I.make_frames(code, F, wl.qber, 10107)
        cands = [tune.Schedule("split_reg", 0, "none", False), tune.Schedule("split_reg", 0, "none", True)]
        cands += [c for c in tune.candidates(n_cu, False, code.z) if c.frames_per_workgroup]
        cands += [tune.Schedule("split_reg", 0, "none", True, 0, 2 * w) for w in (4, 16)]
        best = tune.tune(code.base, code.z, fr.syn, fr.llr, wl.max_iter, cache_path=None, cands=cands, reps=3)
        run = tune.Runner(code.base, code.z, fr.syn, fr.llr, wl.max_iter, tune.Schedule(**best["schedule"]))
        ms = tune.time_ms(run, max(5, steps // 5), max(1, warmup))
        bits, conv, iters = run.outputs()
        ok, und = M.frame_outcomes(fr.x, I.unpack_bits(bits, code.n), conv)
        alg = 4 * float(code.n_edges) * float(iters.sum()) + F * (code.n + (code.m + 7) // 8 + (code.n + 7) // 8 + 5)
        fails = int(F - ok.sum())
        out[f"frames_{F}"] = {"frames": F, "ms_per_launch": round(ms, 4),
                              "mbit_s": round(float(fr.key_bits()[ok].sum()) / (ms / 1e3) / 1e6, 2),
                              "hbm_equivalent_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                              "fer": round(fails / F, 5),
                              "fer_ci95": [round(v, 5) for v in M.wilson_interval(fails, F)],
                              "undetected_errors": int(und.sum()), "mean_iters": round(float(iters.mean()), 3),
                              "max_iters": int(iters.max()), "schedule": best["schedule"],
                              "schedules_tried": best["candidates"]}
    return out


def batched_headline(n_frames, steps, warmup):
    """The batched figure on the headline workload (for profiling it alone)."""
    from paper_1903_10107_amd import inputs as I
    wl = I.WORKLOADS["n32768_q2"]
    code = wl.code()
    return batched(wl, code, int(round(wl.short_frac * code.n)), n_frames, steps, warmup)


def ragged(n_frames, steps, warmup):
    """Ragged batch of the rate-adaptive mother code (24x48 base, Z = 2048,
    n = 98304, R = 1/2): each frame's QBER is drawn from {1, 2, 4, 6, 8}% and
    the frame is punctured to its bucket's FER <= 1e-2 operating point; 60
    iterations. Schedule picked by the autotuner among one-workgroup-per-frame
    and persistent launches, direct or replayed from a HIP graph (hardest first
    = highest QBER first)."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M
    from paper_1903_10107_amd import tune

    max_iter = 60
    code = I.Code(I.make_base(24, 48, 2048), 2048)
    fr = I.make_ragged_frames(code, n_frames, 10107)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cands = [tune.Schedule("auto", 0, "none", False), tune.Schedule("auto", n_cu, "none", False),
             tune.Schedule("auto", 2 * n_cu, "none", False), tune.Schedule("auto", 2 * n_cu, "hardest_first", False),
             tune.Schedule("auto", 2 * n_cu, "hardest_first", True),
             tune.Schedule("auto", 2 * n_cu, "unsat_first", True)]
    best = tune.tune(code.base, code.z, fr.syn, fr.llr, max_iter, difficulty=fr.qber, cache_path=None, cands=cands,
                     reps=2)
    sched = tune.Schedule(**best["schedule"])
    run = tune.Runner(code.base, code.z, fr.syn, fr.llr, max_iter, sched, fr.qber)
    ms = tune.time_ms(run, max(3, steps // 5), max(1, warmup))
    bits, conv, iters = run.outputs()
    correct, undetected = M.frame_outcomes(fr.x, I.unpack_bits(bits, code.n), conv)
    value = float(fr.key_bits()[correct].sum()) / (ms / 1e3) / 1e6
    degs = [int((code.base[b] >= 0).sum()) for b in range(code.mb)]
    tops = algorithmic_int_ops((code.z, degs), iters.sum()) / (ms / 1e3) / 1e12
    edge_iters = float(code.n_edges) * float(iters.sum())
    gbs = (4 * edge_iters + n_frames * (code.n + code.m // 8 + code.n // 8 + 5)) / (ms / 1e3) / 1e9
    per = {}
    f_eff = M.efficiency(code.n, code.m, fr.n_punct, fr.n_short, fr.qber)
    for q in sorted(set(fr.qber.tolist())):
        sel = fr.qber == q
        nf, nfail = int(sel.sum()), int(sel.sum() - correct[sel].sum())
        per[f"{q:.2f}"] = {"frames": nf, "n_punct": int(fr.n_punct[sel][0]),
                           "n_short": int(fr.n_short[sel][0]),
                           "fer": round(nfail / nf, 5),
                           "fer_ci95": [round(v, 5) for v in M.wilson_interval(nfail, nf)],
                           "efficiency_f": round(float(f_eff[sel][0]), 3),
                           "mean_iters": round(float(iters[sel].mean()), 2)}
    return {"value": round(value, 2), "unit": "Mbit/s", "workload": "n98304_ragged",
            "code": "24x48 QC base, Z=2048, column weight 3 (n=98304, R=1/2)", "frames_per_launch": n_frames,
            "max_iter": max_iter, "ms_per_launch": round(ms, 4), "schedule": best["schedule"],
            "schedules_tried": best["candidates"], "kernel": run.code.plan()["kernel"],
            "alu_frac": round(tops / ALU_PEAK_TOPS, 4), "hbm_equivalent_frac": round(gbs / HBM_PEAK_GBS, 4),
            "fer": round(float(1 - correct.mean()), 5), "undetected_errors": int(undetected.sum()),
            "mean_iters": round(float(iters.mean()), 3), "buckets": per}


def learned(steps_train, steps, warmup):
    """Learned check-node offsets on the 5x32, Z = 256 code (n = 8192), QBER 2%,
    36% shortened, 20 iterations: train per-iteration, per-edge offsets of the
    FP32 offset min-sum with the library's forward and backward kernels (Adam,
    512 frames per step from a fixed pool of 2048), quantize them to the
    integer LLR step, and evaluate the integer decoder (min-sum + learned offsets)
    against plain RCBP and plain min-sum on 4096 fresh frames."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import learn as LN
    from paper_1903_10107_amd import metrics as M
    from paper_1903_10107_amd import rate
    from paper_1903_10107_amd import tune

    T, F, q = 20, 512, 0.02
    code = I.Code(I.make_base(5, 32, 256), 256)
    ns = int(0.36 * code.n)
    pool = I.make_frames(code, 4 * F, q, 4242, n_short=ns)
    syn = torch.from_numpy(pool.syn).cuda()
    llr = torch.from_numpy(LN.training_llr(pool)).cuda()
    xb = torch.from_numpy(I.pack_bits(pool.x)).cuda()
    w = torch.from_numpy((np.linspace(0.1, 1.0, T) ** 2).astype(np.float32)).cuda()
    dec = B.OmsDecoder(code.base, code.z, T, w.cpu().numpy())
    beta = torch.full((T, code.n_blocks), 0.3, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([beta], lr=0.02)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the first steps allocate the tape, the workspace and Adam's state: the timed
    # region starts after them (the training itself is the same either way)
    untimed = min(3, max(steps_train - 1, 0))
    for step in range(steps_train):
        if step == untimed:
            a.record()
        sl = slice((step % 4) * F, (step % 4 + 1) * F)
        opt.zero_grad(set_to_none=True)
        loss = dec.loss(syn[sl], llr[sl], xb[sl], beta).mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            beta.clamp_(min=0.0)
    b.record()
    torch.cuda.synchronize()
    train_ms = a.elapsed_time(b) / max(steps_train - untimed, 1)
    final_loss = float(loss.detach())

    # the two kernels alone, on one batch
    code_h = dec.code
    tape = torch.empty(B.ldpc_oms_tape_bytes(code_h, F, T), dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(B.ldpc_oms_workspace_bytes(code_h, F, T), 1), dtype=torch.uint8, device="cuda")
    lo = torch.empty(F, device="cuda")
    db = torch.empty((T, code.n_blocks), device="cuda")
    bt = beta.detach().contiguous()
    g = torch.full((F,), 1.0 / F, device="cuda")
    fwd = lambda: B.ldpc_oms_forward(code_h, syn[:F], llr[:F], xb[:F], F, T, bt, w, lo, None, tape, ws)
    bwd = lambda: B.ldpc_oms_backward(code_h, syn[:F], xb[:F], F, T, bt, w, g, tape, db, None, ws)
    fwd_ms = tune.time_ms(fwd, max(3, steps // 5), max(1, warmup))
    bwd_ms = tune.time_ms(bwd, max(3, steps // 5), max(1, warmup))
    edge_iters = float(code.n_edges) * T * F
    # FP32 operations per edge-iteration of the method: forward 14 (Eq. 8, |.|, sign
    # parity, two-minimum update, exclusion select, offset, clamp, sign, Eq. 9). None
    # is a fused multiply-add and packed FP32 is not used, so the ALU peak is one
    # 32-bit op per lane per cycle: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T/s.
    fwd_tops = 14 * edge_iters / (fwd_ms / 1e3) / 1e12
    # HBM bytes of the forward: the tape it writes (per frame and iteration a
    # four-word record per check row and E) and the inputs it reads once (LLRs,
    # packed syndromes and target bits); the decoder state stays in LDS
    fwd_bytes = float(B.ldpc_oms_tape_bytes(code_h, F, T)) + \
        F * (4.0 * code.n + (code.m + 7) // 8 + (code.n + 7) // 8)
    fwd_gbs = fwd_bytes / (fwd_ms / 1e3) / 1e9
    # backward: reads the tape once (and the syndromes and target bits), writes the
    # per-frame offset gradients [F][T][n_blocks]; 10 FP32 ops per edge-iteration
    # (adjoint of Eq. 9, of the sign, of the clamp, the routing to the minimum or
    # second minimum, the adjoint of Eq. 8 into E and L, the offset gradient)
    bwd_bytes = float(B.ldpc_oms_tape_bytes(code_h, F, T)) + \
        F * ((code.m + 7) // 8 + (code.n + 7) // 8 + 4.0 * T * code.n_blocks)
    bwd_gbs = bwd_bytes / (bwd_ms / 1e3) / 1e9
    bwd_tops = 10 * edge_iters / (bwd_ms / 1e3) / 1e12

    offsets = LN.int_offsets(bt.cpu().numpy())
    decoders = (("rcbp", B.LDPC_RULE_RCBP_FB, None), ("minsum", B.LDPC_RULE_MINSUM, None),
                ("minsum_learned", B.LDPC_RULE_MINSUM, offsets), ("rcbp_learned", B.LDPC_RULE_RCBP_FB, offsets))
    # at the training rate (36% shortened) ...
    evaluated = {name: LN.evaluate(code, q, ns, max_iter=T, frames=4096, cn_rule=rule, offsets=off)
                 for name, rule, off in decoders}
    # ... and at equal frame error rate: each decoder at its own least shortening
    # with FER <= 1e-2 (bisection on 2048 frames, 64-position steps), evaluated on
    # 4096 fresh frames, with its throughput on a 512-frame batch there
    equal_fer = {}
    for name, rule, off in decoders:
        op = rate.search(code, q, frames=2048, max_iter=T, fer_target=1e-2, step=64, seed=5151,
                         cn_rule=rule, offsets=off)
        # the bisection's frames are few for a 1e-2 target: confirm on 4096 fresh
        # frames and shorten further, 64 positions at a time, while they miss it
        n_s = op.n_short
        ev = LN.evaluate(code, q, n_s, max_iter=T, frames=4096, seed=6161, cn_rule=rule, offsets=off)
        while ev["fer"] > 1e-2 and n_s + 64 < code.n - code.m:
            n_s += 64
            ev = LN.evaluate(code, q, n_s, max_iter=T, frames=4096, seed=6161, cn_rule=rule, offsets=off)
        fr = I.make_frames(code, F, q, 99, n_short=n_s)
        run = tune.Runner(code.base, code.z, fr.syn, fr.llr, T, tune.Schedule(), None, 0, cn_rule=rule, offsets=off)
        ms = tune.time_ms(run, max(3, steps // 5), max(1, warmup))
        bits, conv, _ = run.outputs()
        ok, _ = M.frame_outcomes(fr.x, I.unpack_bits(bits, code.n), conv)
        equal_fer[name] = {"shortened": n_s, "short_frac": round(n_s / code.n, 4),
                           "bisection_shortened": op.n_short, "bisection_fer": round(op.fer, 5),
                           "fer": round(ev["fer"], 5),
                           "fer_ci95": ev["fer_ci95"], "frames": ev["frames"], "undetected": ev["undetected"],
                           "efficiency_f": round(ev["efficiency_f"], 4), "mean_iters": round(ev["mean_iters"], 3),
                           "mbit_s": round(float(fr.key_bits()[ok].sum()) / (ms / 1e3) / 1e6, 2),
                           "ms_per_batch": round(ms, 4), "kernel": run.code.plan()["kernel"]}
        print(f"[learned] {name}: {n_s} shortened, FER {ev['fer']:.4f}, f {ev['efficiency_f']:.3f}",
              file=sys.stderr, flush=True)
    # throughput of the integer decoders on a 512-frame batch at the training rate
    fr = I.make_frames(code, F, q, 99, n_short=ns)
    for name, rule, off in decoders:
        run = tune.Runner(code.base, code.z, fr.syn, fr.llr, T, tune.Schedule(), None, 0, cn_rule=rule, offsets=off)
        ms = tune.time_ms(run, max(3, steps // 5), max(1, warmup))
        bits, conv, _ = run.outputs()
        ok, _ = M.frame_outcomes(fr.x, I.unpack_bits(bits, code.n), conv)
        evaluated[name]["mbit_s"] = round(float(fr.key_bits()[ok].sum()) / (ms / 1e3) / 1e6, 2)
        evaluated[name]["ms_per_batch"] = round(ms, 4)
        evaluated[name]["kernel"] = run.code.plan()["kernel"]
    return {"workload": "n8192_q2_learned", "code": "5x32 QC base, Z=256, column weight 3 (n=8192)",
            "qber": q, "short_frac": 0.36, "iterations": T, "train_steps": steps_train, "frames_per_step": F,
            "train_ms_per_step": round(train_ms, 3), "train_frames_per_s": round(F / (train_ms / 1e3), 1),
            "final_loss": round(final_loss, 5), "forward_ms": round(fwd_ms, 4), "backward_ms": round(bwd_ms, 4),
            "forward_roofline": {"bound": "alu", "achieved": round(fwd_tops, 3), "peak": FP32_ALU_PEAK_TOPS,
                                 "unit": "TOP/s", "frac": round(fwd_tops / FP32_ALU_PEAK_TOPS, 4),
                                 "unit_ops": f"14 FP32 ops per edge-iteration x {edge_iters:.0f} edge-iterations",
                                 "fp32_vector_peak_tflops": 157.3,
                                 "frac_of_fp32_vector_peak": round(fwd_tops / 157.3, 4),
                                 "hbm": {"achieved": round(fwd_gbs, 1), "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": round(fwd_gbs / HBM_PEAK_GBS, 4),
                                         "bytes_per_launch": fwd_bytes,
                                         "unit_bytes": "the tape written ((4m + n) FP32 words per frame-iteration) "
                                                       "+ LLRs, syndromes and target bits read"}},
            "backward_roofline": {"bound": "hbm", "achieved": round(bwd_gbs, 1), "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": round(bwd_gbs / HBM_PEAK_GBS, 4),
                                  "bytes_per_launch": bwd_bytes,
                                  "unit_bytes": "the tape read once + syndromes and target bits read + per-frame "
                                                "offset gradients written",
                                  "alu": {"achieved": round(bwd_tops, 3), "peak": FP32_ALU_PEAK_TOPS,
                                          "unit": "TOP/s", "frac": round(bwd_tops / FP32_ALU_PEAK_TOPS, 4),
                                          "frac_of_fp32_vector_peak": round(bwd_tops / 157.3, 4),
                                          "unit_ops": f"10 FP32 ops per edge-iteration x {edge_iters:.0f} "
                                                      "edge-iterations"}},
            "offsets_int_hist": np.bincount(offsets.ravel()).tolist(), "evaluated_at_training_rate": evaluated,
            "equal_fer": equal_fer,
            "note": "offsets learned on the FP32 offset min-sum relaxation; rcbp_learned applies the same "
                    "integer table to the RCBP check node (the paper's decoder has no trainable relaxation)"}


def retry_figure(n_frames, extra=2048, step=512, max_rounds=12):
    """Interactive reveal-and-retry on the ragged rate-adaptive batch: every frame
    starts `extra` punctured positions above its bucket's operating point (a
    higher rate), and each round Alice reveals `step` more punctured positions of
    the frames that have not converged, until all converge."""
    import numpy as np
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M
    from paper_1903_10107_amd import retry

    code = I.Code(I.make_base(24, 48, 2048), 2048)
    pts = I.RAGGED_POINTS
    base = I.make_ragged_frames(code, n_frames, 10107)
    fr0 = I.make_frames(code, n_frames, base.qber, 10107)
    p0 = np.array([pts[float(q)][0] + extra for q in base.qber], dtype=np.int64)
    fr = I.adapt_rate(fr0, np.minimum(p0, code.n - code.m - 1), np.zeros(n_frames, dtype=np.int64))
    res = retry.reconcile(code, fr, 60, reveal_step=step, max_rounds=max_rounds)
    out = res.summary(code, fr.qber)
    out.update({"workload": "n98304_ragged retry", "start": f"operating point + {extra} punctured",
                "reveal_step": step, "max_rounds": max_rounds, "buckets": {}})
    for q in sorted(pts):
        sel = fr.qber == q
        out["buckets"][f"{q:.2f}"] = {
            "frames": int(sel.sum()), "mean_rounds": round(float(res.rounds[sel].mean()), 2),
            "fer": round(float(1 - res.correct[sel].mean()), 5),
            "f_retry": round(float(res.efficiency[sel & res.correct].mean()), 4) if (sel & res.correct).any() else None,
            "f_fixed_point": round(float(M.efficiency(code.n, code.m, pts[q][0], pts[q][1], q)), 4)}
    return out


def syndrome_figure(n_frames, steps, warmup):
    """Alice's side (s = H x, ldpc_syndrome_batch) on n_frames random frames of
    the headline code (n = 32768) and on the 32 frames of the n = 2^20 code:
    encoded key bits per second and the HBM-equivalent fraction (packed bits in,
    packed syndrome out). The first frames are checked against the CPU
    generator's syndromes."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I

    out = {}
    for name, (mb, nb, z, F) in (("n32768", (5, 32, 1024, n_frames)), ("n1048576", (10, 64, 16384, 32))):
        code = I.Code(I.make_base(mb, nb, z), z)
        gc = B.Code(code.base, code.z)
        rng = np.random.default_rng(1903)
        x = rng.integers(0, 2, size=(F, code.n), dtype=np.uint8)
        xb = torch.from_numpy(I.pack_bits(x)).cuda()
        syn = torch.zeros((F, (code.m + 7) // 8), dtype=torch.uint8, device="cuda")
        for _ in range(max(1, warmup)):
            B.ldpc_syndrome_batch(gc, xb, F, syn)
        torch.cuda.synchronize()
        # a launch takes a few microseconds, less than a call from Python: the
        # launches are captured in a graph and replayed back to back
        reps = max(5, steps)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                for _ in range(reps):
                    B.ldpc_syndrome_batch(gc, xb, F, syn)
        torch.cuda.current_stream().wait_stream(side)
        syn.zero_()
        graph.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        graph.replay()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        ref = I.pack_bits(I.syndrome_bits(code, x[:2]))
        assert np.array_equal(syn[:2].cpu().numpy(), ref), "syndrome encoder disagrees with the generator"
        io = F * ((code.n + 7) // 8 + (code.m + 7) // 8)
        out[name] = {"frames": F, "ms_per_launch": round(ms, 4),
                     "gbit_s_encoded": round(F * code.n / (ms / 1e3) / 1e9, 1),
                     "hbm_equivalent_frac": round(io / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def end_to_end(gc, code, fr, max_iter, key_bits_ok, steps, warmup):
    """The headline step with the host link included: the batch's LLRs and
    syndromes copied from pinned host memory, the decode, and the packed bits,
    flags and counts copied back, all on one stream, timed with HIP events
    around each step (the PCIe-inclusive rate; `value` excludes the copies)."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B

    F = fr.n_frames
    h_syn = torch.from_numpy(fr.syn).pin_memory()
    h_llr = torch.from_numpy(fr.llr).pin_memory()
    h_bits = torch.empty((F, (code.n + 7) // 8), dtype=torch.uint8).pin_memory()
    h_conv = torch.empty(F, dtype=torch.uint8).pin_memory()
    h_iters = torch.empty(F, dtype=torch.int32).pin_memory()
    d_syn, d_llr = torch.empty_like(h_syn, device="cuda"), torch.empty_like(h_llr, device="cuda")
    d_bits, d_conv, d_iters = (torch.empty_like(h_bits, device="cuda"), torch.empty_like(h_conv, device="cuda"),
                               torch.empty_like(h_iters, device="cuda"))

    def step():
        d_syn.copy_(h_syn, non_blocking=True)
        d_llr.copy_(h_llr, non_blocking=True)
        B.ldpc_decode_batch_ex(gc, d_syn, d_llr, F, max_iter, d_bits, d_conv, d_iters)
        h_bits.copy_(d_bits, non_blocking=True)
        h_conv.copy_(d_conv, non_blocking=True)
        h_iters.copy_(d_iters, non_blocking=True)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    h2d = h_syn.numel() + h_llr.numel()
    d2h = h_bits.numel() + h_conv.numel() + 4 * h_iters.numel()
    return {"ms_per_step": round(ms, 4), "value": round(key_bits_ok / (ms / 1e3) / 1e6, 2), "unit": "Mbit/s",
            "h2d_bytes": int(h2d), "d2h_bytes": int(d2h), "timing": "median over steps of HIP events around "
            "copy in, decode, copy out on one stream (pinned host buffers)"}


def lds_peaks(reps: int = 256, n_wg: int = 2048) -> dict:
    """Measured LDS read bandwidth of the whole chip (GB/s) for 16-byte and for
    byte reads (ldpc_probe_lds_bandwidth: conflict-free reads, 1024-thread
    workgroups of 64 KB each, two per CU), median of five launches."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B

    out = torch.zeros(n_wg * 1024, dtype=torch.int32, device="cuda")
    res = {}
    for mode, width in ((0, 16), (1, 1)):
        B.ldpc_probe_lds_bandwidth(mode, n_wg, reps, out)
        times = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            B.ldpc_probe_lds_bandwidth(mode, n_wg, reps, out)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        res["read_b128" if mode == 0 else "read_u8"] = round(n_wg * 1024.0 * reps * 8 * width / (ms / 1e3) / 1e9, 1)
    return res


def pipelined(gc, code, fr, d_syn, d_llr, max_iter, ref, steps, warmup, n_streams=2):
    """The headline workload (256-frame batches, one launch each) with
    consecutive batches issued on alternating streams, so that the CUs freed by
    the early-finishing frames of one launch start the next launch's frames
    instead of idling until the launch's slowest frame ends. Every launch still
    decodes its whole batch; the figure is wall-clock throughput over K
    launches between two device synchronizations."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    F = fr.n_frames
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    outs = [(torch.zeros((F, (code.n + 7) // 8), dtype=torch.uint8, device="cuda"),
             torch.zeros(F, dtype=torch.uint8, device="cuda"),
             torch.zeros(F, dtype=torch.int32, device="cuda")) for _ in range(n_streams)]

    def launch(i):
        s = streams[i % n_streams]
        bits, conv, iters = outs[i % n_streams]
        B.ldpc_decode_batch_ex(gc, d_syn, d_llr, F, max_iter, bits, conv, iters, stream=s)

    torch.cuda.synchronize()
    for i in range(warmup):
        launch(i)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(steps):
        launch(i)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / steps
    for bits, conv, iters in outs:
        assert np.array_equal(bits.cpu().numpy(), ref[0]) and np.array_equal(iters.cpu().numpy(), ref[2])
    bits = I.unpack_bits(ref[0], code.n)
    ok, _ = M.frame_outcomes(fr.x, bits, ref[1])
    alg_bytes = 4 * float(code.n_edges) * float(ref[2].sum()) + F * (code.n + (code.m + 7) // 8 + (code.n + 7) // 8 + 5)
    return {"streams": n_streams, "frames_per_launch": F, "launches": steps, "ms_per_launch": round(ms, 4),
            "value": round(float(fr.key_bits()[ok].sum()) / (ms / 1e3) / 1e6, 2), "unit": "Mbit/s",
            "hbm_equivalent_frac": round(alg_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "timing": "wall clock over the launches between two device synchronizations"}


def large_frames(steps, warmup):
    """Frames of n = 1048576 (10x64 QC base, Z = 16384, 16-bit soft values), 32
    frames, 80 iterations: the literal configuration at QBER 2% (every frame
    runs all 80 iterations: a fixed amount of work) and the same code shortened
    by a third (corrected-key throughput), on the layer-synchronous family.
    Its launches are replayed as HIP graphs: the whole decode as one graph for
    the literal case; for the shortened case one graph per iteration, with the
    host reading the number of frames not yet retired after each and stopping
    at 0 (check_every = 1)."""
    import numpy as np
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M
    from paper_1903_10107_amd import tune

    wl = I.WORKLOADS["n1048576_q2"]
    code = wl.code()
    degs = [int((code.base[b] >= 0).sum()) for b in range(code.mb)]
    out = {"workload": wl.name, "code": "10x64 QC base, Z=16384, column weight 3 (n=1048576)", "frames": wl.frames,
           "max_iter": wl.max_iter, "soft_values": "int16"}
    for name, frac, check in (("literal", 0.0, 0), ("shortened_0.33", 0.33, 1)):
        fr = I.make_frames(code, wl.frames, wl.qber, 10107, n_short=int(frac * code.n))
        sched = tune.Schedule(graph=True, check_every=check)
        run = tune.Runner(code.base, code.z, fr.syn, fr.llr, wl.max_iter, sched, None, wl.acc_bits)
        ms = tune.time_ms(run, max(2, steps // 10), max(1, warmup // 2))
        bits, conv, iters = run.outputs()
        ok, und = M.frame_outcomes(fr.x, I.unpack_bits(bits, code.n), conv)
        tops = algorithmic_int_ops((code.z, degs), iters.sum()) / (ms / 1e3) / 1e12
        # 16-bit soft values: 6 B per edge-iteration (L read and written as 8 bits,
        # E read and written as 16 bits), plus the frame I/O
        alg_bytes = 6 * float(code.n_edges) * float(iters.sum()) + \
            wl.frames * (code.n + (code.m + 7) // 8 + (code.n + 7) // 8 + 5)
        out[name] = {"short_frac": frac, "ms_per_launch": round(ms, 3), "kernel": run.code.plan()["kernel"],
                     "check_every": check,
                     "mean_iters": round(float(iters.mean()), 2), "fer": round(float(1 - ok.mean()), 4),
                     "mbit_s": round(float(fr.key_bits()[ok].sum()) / (ms / 1e3) / 1e6, 2),
                     "frame_iterations_per_s": round(float(iters.sum()) / (ms / 1e3), 1),
                     "alu_frac": round(tops / ALU_PEAK_TOPS, 4),
                     "hbm_equivalent_frac": round(alg_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out



def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_launches(gc, d_syn, d_llr, F, max_iter, steps, warmup):
    """K single-launch decode steps of resident buffers on torch's current stream
    (the stream the library launches on), with HIP events around every launch
    and around the whole run. Returns (ms per step, mean launch ms, outputs)."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B

    n_bytes = (gc.n + 7) // 8
    d_bits = torch.zeros((F, n_bytes), dtype=torch.uint8, device="cuda")
    d_conv = torch.zeros(F, dtype=torch.uint8, device="cuda")
    d_iters = torch.zeros(F, dtype=torch.int32, device="cuda")
    ws_bytes = B.ldpc_workspace_bytes(gc, F)
    d_ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda") if ws_bytes else None

    def step():
        B.ldpc_decode_batch_ex(gc, d_syn, d_llr, F, max_iter, d_bits, d_conv, d_iters, None, None, d_ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for i in range(steps):
        ev[i][0].record()
        step()
        ev[i][1].record()
    t1.record()
    torch.cuda.synchronize()
    ms_per_step = t0.elapsed_time(t1) / steps
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    return ms_per_step, kernel_ms, (d_bits.cpu().numpy(), d_conv.cpu().numpy(), d_iters.cpu().numpy())


def operating_point(gc, wl, code, n_short, steps, warmup, fer_frames, with_lds=False):
    """One shortening of the headline workload: the timed 256-frame launches
    (corrected-key throughput, the roofline of the decode kernel) and the frame
    error rate on fer_frames fresh frames of the same shortening."""
    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    fr = I.make_frames(code, wl.frames, wl.qber, 10107, n_short=n_short)
    F = fr.n_frames
    d_syn = torch.from_numpy(fr.syn).cuda()
    d_llr = torch.from_numpy(fr.llr).cuda()
    ms_per_step, kernel_ms, ref = timed_launches(gc, d_syn, d_llr, F, wl.max_iter, steps, warmup)
    bits_p, conv, iters = ref
    correct, undetected = M.frame_outcomes(fr.x, I.unpack_bits(bits_p, code.n), conv)
    key_ok = float(fr.key_bits()[correct].sum())
    value = key_ok / (ms_per_step / 1e3) / 1e6
    fails = int(F - correct.sum())
    f_eff = float(np.mean(M.efficiency(code.n, code.m, fr.n_punct, fr.n_short, fr.qber)))

    # frame error rate on fresh frames (the timed batch is too small to show 1e-2)
    big = I.make_frames(code, fer_frames, wl.qber, 20190325, n_short=n_short)
    got = B.decode(gc, big.syn, big.llr, wl.max_iter)
    ok_b, und_b = M.frame_outcomes(big.x, I.unpack_bits(got["bits"], code.n), got["conv"])
    fails_b = int(fer_frames - ok_b.sum())

    family = gc.plan()["kernel"]
    bytes_per_edge_iter = 6 if wl.acc_bits == 16 else 4
    edge_iters = float(code.n_edges) * float(iters.sum())
    io_bytes = F * (code.n + (code.m + 7) // 8 + (code.n + 7) // 8 + 5)
    alg_bytes = bytes_per_edge_iter * edge_iters + io_bytes
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    degs = [int((code.base[b] >= 0).sum()) for b in range(code.mb)]
    int_ops = algorithmic_int_ops((code.z, degs), iters.sum())
    alu_tops = int_ops / (kernel_ms / 1e3) / 1e12
    traffic = measured_traffic(wl.name) if family == HEADLINE_FAMILY and n_short == int(
        round(I.WORKLOADS[wl.name].short_frac * code.n)) else None
    rl = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
          "kernel": KERNEL_SYMBOLS.get(family, family), "family": family, "kernel_ms": round(kernel_ms, 4),
          "algorithmic_bytes_per_launch": alg_bytes,
          "unit_bytes": f"{bytes_per_edge_iter} B per edge-iteration (L and E each read and written once) x "
                        f"{edge_iters:.0f} edge-iterations + {io_bytes} B frame I/O",
          "note": "HBM-equivalent: the decoder state stays in LDS and registers, so the measured HBM traffic "
                  "(traffic) is the frame I/O; the kernel is bound by integer VALU issue (alu)" + (
                      "; below 0.40 of the HBM roofline because a single launch lasts as long as its slowest "
                      "frame (tail.cu_busy_frac); launches that do not wait for it (pipelined, batched) go higher"
                      if achieved / HBM_PEAK_GBS < 0.40 else ""),
          "alu": {"achieved": round(alu_tops, 2), "peak": round(ALU_PEAK_TOPS, 1), "unit": "TOP/s",
                  "frac": round(alu_tops / ALU_PEAK_TOPS, 4), "algorithmic_ops_per_launch": int_ops,
                  "unit_ops": "14 int ops per edge-iteration + 27 per (row degree - 2) per check row-iteration; "
                              f"{int(iters.sum())} frame-iterations of {code.n_edges} edges",
                  "peak_source": "256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (packed 16-bit)"},
          # one frame per CU: the launch lasts as long as its slowest frame, so
          # the CUs of the other frames idle for the rest of it
          "tail": {"frames": F, "cus": torch.cuda.get_device_properties(0).multi_processor_count,
                   "mean_iters": round(float(iters.mean()), 3), "max_iters": int(iters.max()),
                   "cu_busy_frac": round(float(iters.mean()) / max(int(iters.max()), 1), 4)}}
    if with_lds and family in ("split_reg", "split", "pairs", "lds"):
        # the decoder state lives on chip: its state traffic against the measured
        # LDS read peaks (byte reads are the width of the decoder's E accesses)
        peaks = lds_peaks()
        lds_bytes = bytes_per_edge_iter * edge_iters
        lds_achieved = lds_bytes / (kernel_ms / 1e3) / 1e9
        rl["lds"] = {"achieved": round(lds_achieved, 1), "unit": "GB/s",
                     "peak_read_u8": peaks["read_u8"], "peak_read_b128": peaks["read_b128"],
                     "frac_of_u8_peak": round(lds_achieved / peaks["read_u8"], 4),
                     "frac_of_b128_peak": round(lds_achieved / peaks["read_b128"], 4),
                     "algorithmic_bytes_per_launch": lds_bytes,
                     "unit_bytes": f"{bytes_per_edge_iter} B per edge-iteration x {edge_iters:.0f} edge-iterations",
                     "peak_source": "ldpc_probe_lds_bandwidth, measured in this run"}
    return {"short_frac": round(n_short / code.n, 4), "shortened": n_short, "mbit_s": round(value, 2),
            "ms_per_step": round(ms_per_step, 4), "frames_per_launch": F,
            "fer": round(fails_b / fer_frames, 5),
            "fer_ci95": [round(v, 5) for v in M.wilson_interval(fails_b, fer_frames)],
            "fer_frames": fer_frames, "undetected_fer_frames": int(und_b.sum()),
            "fer_batch": round(fails / F, 5), "fer_batch_ci95": [round(v, 5) for v in M.wilson_interval(fails, F)],
            "undetected_errors": int(undetected.sum()), "efficiency_f": round(f_eff, 4),
            "mean_iters": round(float(iters.mean()), 3), "max_iters": int(iters.max()),
            "key_bits_ok": key_ok, "roofline": rl,
            "_frames": fr, "_syn": d_syn, "_llr": d_llr, "_ref": ref}


def float_bp_comparison(gc, wl, code, shorts, n_frames):
    """FP64 layered BP (the oracle, on the host's cores) beside the integer
    decoder (the library, on the GPU) on the same frames at each shortening:
    frame error rates with Wilson intervals, efficiency, mean iterations and the
    integer-minus-float FER gap. The floating-point decoder reads the unquantized
    channel LLRs (ln((1-q)/q), shortened positions at a large fixed value)."""
    import numpy as np
    import oracle as O
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    rows = []
    for ns in shorts:
        fr = I.make_frames(code, n_frames, wl.qber, 31415, n_short=ns)
        t = time.perf_counter()
        fl = O.bp_fp64_decode(code.base, code.z, fr.syn, fr.llr_f, wl.max_iter, n_threads=threads)
        el = time.perf_counter() - t
        it = B.decode(gc, fr.syn, fr.llr, wl.max_iter)
        ok_f, _ = M.frame_outcomes(fr.x, I.unpack_bits(fl["bits"], code.n), fl["conv"])
        ok_i, _ = M.frame_outcomes(fr.x, I.unpack_bits(it["bits"], code.n), it["conv"])
        ff, fi = int(n_frames - ok_f.sum()), int(n_frames - ok_i.sum())
        rows.append({"short_frac": round(ns / code.n, 4), "shortened": ns, "frames": n_frames,
                     "efficiency_f": round(float(np.mean(M.efficiency(code.n, code.m, fr.n_punct, fr.n_short,
                                                                      fr.qber))), 4),
                     "fer_fp64_bp": round(ff / n_frames, 5),
                     "fer_fp64_bp_ci95": [round(v, 5) for v in M.wilson_interval(ff, n_frames)],
                     "fer_int8": round(fi / n_frames, 5),
                     "fer_int8_ci95": [round(v, 5) for v in M.wilson_interval(fi, n_frames)],
                     "fer_gap_int8_minus_fp64": round((fi - ff) / n_frames, 5),
                     "mean_iters_fp64_bp": round(float(fl["iters"].mean()), 3),
                     "mean_iters_int8": round(float(it["iters"].mean()), 3),
                     "fp64_seconds": round(el, 2)})
        print(f"[float-bp] {wl.name} shortened {ns}: fp64 FER {ff}/{n_frames}, int8 FER {fi}/{n_frames}, "
              f"{el:.1f} s", file=sys.stderr, flush=True)
    return {"kind": "oracle", "decoder": "FP64 layered BP, exact box-plus (Eq. 6), same schedule and stopping rule",
            "cores": threads, "points": rows}


def float_compare(args):
    """The FP64-BP-versus-integer table of the profiles: the headline code at its
    two operating points and each bucket of the ragged rate-adaptive batch."""
    import numpy as np
    import oracle as O
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    torch.cuda.set_device(0)
    wl = I.WORKLOADS["n32768_q2"]
    code = wl.code()
    gc = B.Code(code.base, code.z)
    shorts = [int(round(wl.short_frac * code.n))] + ([args.least_short] if args.least_short is not None else [])
    res = {"headline": float_bp_comparison(gc, wl, code, shorts, args.float_frames)}
    print(json.dumps(res), flush=True)
    rcode = I.Code(I.make_base(24, 48, 2048), 2048)
    rgc = B.Code(rcode.base, rcode.z)
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    buckets = []
    for q in I.RAGGED_QBERS:
        p, sh = I.RAGGED_POINTS[q]
        fr = I.make_frames(rcode, args.ragged_float_frames, q, 27182, n_punct=p, n_short=sh)
        t = time.perf_counter()
        fl = O.bp_fp64_decode(rcode.base, rcode.z, fr.syn, fr.llr_f, 60, n_threads=threads)
        el = time.perf_counter() - t
        it = B.decode(rgc, fr.syn, fr.llr, 60)
        ok_f, _ = M.frame_outcomes(fr.x, I.unpack_bits(fl["bits"], rcode.n), fl["conv"])
        ok_i, _ = M.frame_outcomes(fr.x, I.unpack_bits(it["bits"], rcode.n), it["conv"])
        n = fr.n_frames
        ff, fi = int(n - ok_f.sum()), int(n - ok_i.sum())
        row = {"qber": q, "punctured": p, "shortened": sh, "frames": n,
               "efficiency_f": round(float(M.efficiency(rcode.n, rcode.m, p, sh, q)), 4),
               "fer_fp64_bp": round(ff / n, 5), "fer_fp64_bp_ci95": [round(v, 5) for v in M.wilson_interval(ff, n)],
               "fer_int8": round(fi / n, 5), "fer_int8_ci95": [round(v, 5) for v in M.wilson_interval(fi, n)],
               "fer_gap_int8_minus_fp64": round((fi - ff) / n, 5),
               "mean_iters_fp64_bp": round(float(fl["iters"].mean()), 3),
               "mean_iters_int8": round(float(it["iters"].mean()), 3), "fp64_seconds": round(el, 1)}
        buckets.append(row)
        print(json.dumps({"ragged_bucket": row}), flush=True)
    res["ragged"] = {"code": "24x48 QC base, Z=2048 (n=98304, R=1/2), 60 iterations", "buckets": buckets}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="n32768_q2")
    ap.add_argument("--short-frac", type=float, default=None,
                    help="override the workload's shortened fraction (operating-point studies)")
    ap.add_argument("--frames", type=int, default=None, help="override the workload's batch size")
    ap.add_argument("--least-short", type=int, default=I_LEAST_SHORT,
                    help="shortened positions of the least-shortening FER <= 1e-2 point, measured beside "
                         "the value point (negative: skip)")
    ap.add_argument("--fer-frames", type=int, default=4096,
                    help="fresh frames decoded at each operating point for its frame error rate")
    ap.add_argument("--float-frames", type=int, default=512,
                    help="frames per operating point decoded by the FP64 BP oracle beside the integer "
                         "decoder in the CPU-baseline leg (0: skip)")
    ap.add_argument("--ragged-float-frames", type=int, default=1024,
                    help="frames per ragged bucket in --float-compare")
    ap.add_argument("--float-compare", action="store_true",
                    help="print the FP64-BP-versus-integer table (headline operating points and the "
                         "ragged buckets) and exit")
    ap.add_argument("--batched-frames", type=int, default=4096,
                    help="frames of the same workload decoded per launch for the batched figure (0: skip)")
    ap.add_argument("--ragged-frames", type=int, default=2048,
                    help="frames of the ragged rate-adaptive batch (n = 98304) for its figure (0: skip)")
    ap.add_argument("--learned-steps", type=int, default=150,
                    help="training steps of the learned-offset figure (0: skip)")
    ap.add_argument("--retry-frames", type=int, default=2048,
                    help="frames of the reveal-and-retry figure on the ragged batch (0: skip)")
    ap.add_argument("--no-large", action="store_true", help="skip the n = 1048576 figure")
    ap.add_argument("--small-frames", default="64,65536",
                    help="batch sizes of the n = 1024 short-frame figure (0: skip)")
    ap.add_argument("--syndrome-frames", type=int, default=4096,
                    help="frames of the syndrome-encoder figure (Alice's side; 0: skip)")
    ap.add_argument("--pipelined-streams", type=int, default=3,
                    help="streams for the pipelined figure (consecutive batches overlapped; < 2: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fer-sweep", default="",
                    help="comma-separated shortened fractions: print FER, iterations and f at each")
    ap.add_argument("--qber-sweep", default="",
                    help="comma-separated QBERs for --fer-sweep (default: the workload's)")
    ap.add_argument("--sweep-frames", type=int, default=4096)
    ap.add_argument("--only", choices=("learned", "syndrome", "retry", "large", "batched", "ragged", "small"),
                    default=None,
                    help="run one figure alone and print it as one JSON line (for profiling its kernels)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="instead of decoding, run a plain device copy of BYTES bytes per step "
                         "(reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.least_short is not None and args.least_short < 0:
        args.least_short = None
    if args.gpus != 1:
        print(f"bench.py measures one GPU: frames are independent, so N GPUs would each decode their own "
              f"batch with no exchange; --gpus {args.gpus} is not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1903_10107_amd import binding as B
    from paper_1903_10107_amd import inputs as I
    from paper_1903_10107_amd import metrics as M

    if args.copy_calibration:
        copy_calibration(args.copy_calibration, args.steps, args.warmup)
        return
    if args.float_compare:
        float_compare(args)
        return
    if args.only:
        torch.cuda.set_device(0)
        fig = {"learned": lambda: learned(args.learned_steps, args.steps, args.warmup),
               "syndrome": lambda: syndrome_figure(args.syndrome_frames, args.steps, args.warmup),
               "retry": lambda: retry_figure(args.retry_frames),
               "large": lambda: large_frames(args.steps, args.warmup),
               "batched": lambda: batched_headline(args.batched_frames, args.steps, args.warmup),
               "ragged": lambda: ragged(args.ragged_frames, args.steps, args.warmup),
               "small": lambda: small_frames([int(v) for v in args.small_frames.split(",") if v],
                                             args.steps, args.warmup)}[args.only]()
        print(json.dumps({"figure": args.only, args.only: fig}), flush=True)
        return
    if args.workload == "n98304_ragged":
        # the ragged rate-adaptive batch alone (for profiling its kernel)
        torch.cuda.set_device(0)
        r = ragged(args.ragged_frames or 2048, args.steps, args.warmup)
        print(json.dumps({"metric": "corrected-key Mbit/s, ragged rate-adaptive batch, n=98304", "value": r["value"],
                          "unit": "Mbit/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": r["ms_per_launch"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "int8", "data": "synthetic",
                          "config": {"workload": "n98304_ragged"}, "ragged": r}), flush=True)
        return
    wl = I.WORKLOADS[args.workload]
    if args.short_frac is not None or args.frames is not None:
        import dataclasses
        wl = dataclasses.replace(wl, short_frac=wl.short_frac if args.short_frac is None else args.short_frac,
                                 frames=wl.frames if args.frames is None else args.frames)
    code = wl.code()
    if args.fer_sweep:
        fer_sweep(wl, code, [float(v) for v in args.fer_sweep.split(",")], args.sweep_frames,
                  [float(v) for v in args.qber_sweep.split(",")] if args.qber_sweep else None)
        return
    n_short = int(round(wl.short_frac * code.n))
    torch.cuda.set_device(0)
    gc = B.Code(code.base, code.z, acc_bits=wl.acc_bits)
    fer_frames = max(args.fer_frames, wl.frames)
    point = operating_point(gc, wl, code, n_short, args.steps, args.warmup, fer_frames, with_lds=True)
    fr, d_syn, d_llr, ref = point.pop("_frames"), point.pop("_syn"), point.pop("_llr"), point.pop("_ref")
    rl = point["roofline"]
    out = {
        "metric": METRIC,
        "value": point["mbit_s"],
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": point["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16" if wl.acc_bits == 16 else "int8",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": code.n, "frames": wl.frames, "qber": wl.qber, "shortened": n_short,
                   "short_frac": wl.short_frac,
                   "max_iter": wl.max_iter, "code": f"{wl.mb}x{wl.nb} QC base, Z={wl.z}, column weight 3",
                   "decoder": "plain (RCBP forward-backward check node, saturating VN)",
                   "operating_point": "the value point of the single-launch form (design notes, measurement); "
                                      "the least-shortening point with FER <= 1e-2 is in operating_points"},
        "roofline": rl,
        "fer": point["fer_batch"],
        "fer_ci95": point["fer_batch_ci95"],
        "undetected_errors": point["undetected_errors"],
        "efficiency_f": point["efficiency_f"],
        "mean_iters": point["mean_iters"],
        "max_iters_in_batch": point["max_iters"],
        "paper_context": "57.6 Mbit/s at f=1.108 on a 4-core i7-6700HQ with its own irregular codes (context only)",
    }
    pts = {"value_point": {k: v for k, v in point.items() if k != "roofline"}}
    pts["value_point"]["hbm_equivalent_frac"] = rl["frac"]
    pts["value_point"]["alu_frac"] = rl["alu"]["frac"]
    if args.least_short is not None and args.least_short != n_short:
        lp = operating_point(gc, wl, code, args.least_short, args.steps, args.warmup, fer_frames, with_lds=False)
        lfr, l_syn, l_llr, lref = lp.pop("_frames"), lp.pop("_syn"), lp.pop("_llr"), lp.pop("_ref")
        lrl = lp.pop("roofline")
        lp["hbm_equivalent_frac"] = lrl["frac"]
        lp["alu_frac"] = lrl["alu"]["frac"]
        lp["tail"] = lrl["tail"]
        lp["kernel_ms"] = lrl["kernel_ms"]
        if args.pipelined_streams > 1:
            lp["pipelined"] = pipelined(gc, code, lfr, l_syn, l_llr, wl.max_iter, lref, args.steps, args.warmup,
                                        args.pipelined_streams)
        lp["origin"] = ("least shortening with FER <= 1e-2 at QBER 2%: bisection over the shortened "
                        "positions (paper_1903_10107_amd.rate, 2048 frames per probe, 256-position steps)")
        pts["least_shortening"] = lp
        del lfr, l_syn, l_llr
    out["operating_points"] = pts
    out["end_to_end"] = end_to_end(gc, code, fr, wl.max_iter, point["key_bits_ok"],
                                   max(10, args.steps // 5), max(1, args.warmup))
    if args.pipelined_streams > 1:
        out["pipelined"] = pipelined(gc, code, fr, d_syn, d_llr, wl.max_iter, ref, args.steps, args.warmup,
                                     args.pipelined_streams)
    if args.batched_frames:
        out["batched"] = batched(wl, code, n_short, args.batched_frames, args.steps, args.warmup)
        if "least_shortening" in pts:
            # the batched form at the least shortening with FER <= 1e-2: it does not
            # wait for one batch's slowest frame, so this is where it pays most
            pts["least_shortening"]["batched"] = batched(wl, code, args.least_short, args.batched_frames,
                                                         args.steps, args.warmup)
    if args.ragged_frames:
        out["ragged"] = ragged(args.ragged_frames, args.steps, args.warmup)
    if args.learned_steps:
        out["learned"] = learned(args.learned_steps, args.steps, args.warmup)
    if args.retry_frames:
        out["retry"] = retry_figure(args.retry_frames)
    if args.syndrome_frames:
        out["syndrome"] = syndrome_figure(args.syndrome_frames, args.steps, args.warmup)
    if not args.no_large:
        out["large"] = large_frames(args.steps, args.warmup)
    small_batches = [int(v) for v in args.small_frames.split(",") if v.strip() and int(v) > 0]
    if small_batches:
        out["small"] = small_frames(small_batches, args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(code, fr, wl, args.cpu_seconds)
        if not args.no_large:
            out["cpu_baseline"]["large"] = cpu_baseline_large(args.cpu_seconds / 3)
        if args.float_frames:
            shorts = [n_short] + ([args.least_short] if args.least_short is not None else [])
            out["cpu_baseline"]["float_bp"] = float_bp_comparison(gc, wl, code, shorts, args.float_frames)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
