"""Autotuner for batch schedules of the decoder.

For a code, a batch size and an iteration limit it times candidate schedules on
a representative batch held on the GPU and keeps the fastest:

* kernel family (ldpc_params.kernel_hint): every family that applies to the code;
* persistent workgroups: 0 (one workgroup per frame, hardware dispatch) or a
  multiple of the CU count pulling frames from a device queue;
* decode order (persistent schedules only): as given; hardest first by a
  per-frame difficulty the caller supplies (for instance the frame's QBER or
  its expected iteration count); or by the number of check rows the channel
  hard decision fails, computed on the GPU before every decode
  (ldpc_order_by_unsat). The last two move long frames away from the end of
  the launch;
* graph: the decode captured once as a HIP graph and replayed, or launched
  directly;
* early stop (layer-synchronous family only): the host reads the number of
  frames not yet retired after every iteration and stops launching at 0;
* frames per workgroup (register-resident family, lifts Z <= 64): one frame
  per workgroup, or 64 / Z frames per wave and 1 to 16 waves per workgroup.

The row tile is the family's: one row per lane (lds, global), a row pair per
lane (pairs), a row pair per two lanes with the messages in LDS (split), in a
global slice (split_global_l) or in registers (split_reg), or a layer's row
pairs spread over several workgroups (layer_sync); `row_tile()` names it for
each candidate.

Every candidate must produce identical outputs (the schedule never changes the
results); a mismatch raises. Results are cached in a JSON file keyed by the
code, batch size, iteration limit, soft-value width, device name and library
version.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import asdict, dataclass

import numpy as np

from . import binding as B

DEFAULT_CACHE = os.environ.get("QKDLDPC_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "qkdldpc", "tune.json"))


@dataclass(frozen=True)
class Schedule:
    kernel: str = "auto"
    persistent_workgroups: int = 0
    order: str = "none"          # "none", "hardest_first" (caller's difficulty) or "unsat_first"
    graph: bool = False
    check_every: int = 0         # layer-synchronous family: iterations between host checks (0: none)
    frames_per_workgroup: int = 0  # split_reg with Z <= 64: frames per workgroup (0: one, with barriers)


ROW_TILES = {"global": "1 row per lane, state in global memory",
             "lds": "1 row per lane, state in LDS",
             "pairs": "2 rows (r, r + Z/2) per lane, all edges, state in LDS",
             "split": "2 rows per 2 lanes (half the edges each), E and L in LDS",
             "split_global_l": "2 rows per 2 lanes, E in LDS, L streamed from a global slice",
             "split_reg": "2 rows per 2 lanes, E in LDS, L in registers",
             "layer_sync": "2 rows per 2 lanes, a layer spread over Z/1024 workgroups per frame"}


def row_tile(family: str) -> str:
    return ROW_TILES.get(family, family)


def _key(base, z, n_frames, max_iter, acc_bits, has_difficulty) -> str:
    import torch
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(base, dtype=np.int32).tobytes())
    h.update(repr((int(z), int(n_frames), int(max_iter), int(acc_bits), bool(has_difficulty),
                   torch.cuda.get_device_name(0), B.ldpc_version())).encode())
    return h.hexdigest()[:24]


def candidates(n_cu: int, has_difficulty: bool, z: int = 0) -> list[Schedule]:
    out = []
    if 0 < z <= 64:
        fw = 64 // z
        for waves in (1, 2, 4, 8, 16):
            out.append(Schedule("split_reg", 0, "none", False, 0, fw * waves))
    for kernel in ("split_reg", "split", "split_global_l", "layer_sync", "pairs", "lds", "global"):
        out.append(Schedule(kernel, 0, "none", False))
        out.append(Schedule(kernel, 0, "none", True))
    for graph in (False, True):
        out.append(Schedule("layer_sync", 0, "none", graph, 1))
    for kernel in B.PERSISTENT_FAMILIES:
        for wgs in (n_cu, 2 * n_cu):
            for order in (("none", "hardest_first", "unsat_first") if has_difficulty else ("none", "unsat_first")):
                for graph in (False, True):
                    out.append(Schedule(kernel, wgs, order, graph))
    return out


class Runner:
    """Device buffers and a callable that decodes the batch with one schedule."""

    def __init__(self, base, z, syn, llr, max_iter, sched: Schedule, difficulty=None, acc_bits=0, **code_kw):
        import torch
        self.code = B.Code(base, z, acc_bits=acc_bits, kernel=sched.kernel, **code_kw)
        if sched.persistent_workgroups and self.code.plan()["kernel"] not in B.PERSISTENT_FAMILIES:
            raise B.LdpcError(B.LDPC_EUNSUPPORTED, "persistent schedule needs the split family")
        if sched.frames_per_workgroup and (self.code.plan()["kernel"] != "split_reg" or z > 64):
            raise B.LdpcError(B.LDPC_EUNSUPPORTED, "frames per workgroup need split_reg with Z <= 64")
        F = llr.shape[0]
        self.F = F
        self.syn = torch.from_numpy(np.ascontiguousarray(syn)).cuda()
        self.llr = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
        self.bits = torch.zeros((F, (self.code.n + 7) // 8), dtype=torch.uint8, device="cuda")
        self.conv = torch.zeros(F, dtype=torch.uint8, device="cuda")
        self.iters = torch.zeros(F, dtype=torch.int32, device="cuda")
        self.order = None
        self.unsat = None
        if sched.order == "hardest_first" and difficulty is not None:
            perm = np.argsort(-np.asarray(difficulty, dtype=np.float64), kind="stable").astype(np.int32)
            self.order = torch.from_numpy(perm).cuda()
        elif sched.order == "unsat_first" and sched.persistent_workgroups:
            # filled on the device before every decode (part of the timed step)
            self.unsat = torch.empty(F, dtype=torch.int32, device="cuda")
            self.order = torch.arange(F, dtype=torch.int32, device="cuda")
        need = B.ldpc_workspace_bytes_sched(self.code, F, sched.persistent_workgroups)
        self.ws = torch.empty(need, dtype=torch.uint8, device="cuda") if need else None
        self.sched = sched
        self.max_iter = max_iter
        self.batch = None
        if sched.graph:
            self.batch = B.Batch(self.code, self.syn, self.llr, F, max_iter, self.bits, self.conv, self.iters,
                                 sched.persistent_workgroups, self.order, self.ws, check_every=sched.check_every,
                                 frames_per_workgroup=sched.frames_per_workgroup)

    def __call__(self):
        if self.unsat is not None:
            B.ldpc_order_by_unsat(self.code, self.syn, self.llr, self.F, self.unsat, self.order)
        if self.batch is not None:
            self.batch.launch()
        else:
            B.ldpc_decode_batch_sched(self.code, self.syn, self.llr, self.F, self.max_iter, self.bits, self.conv,
                                      self.iters, self.sched.persistent_workgroups, self.order, self.ws,
                                      check_every=self.sched.check_every,
                                      frames_per_workgroup=self.sched.frames_per_workgroup)

    def outputs(self):
        return self.bits.cpu().numpy(), self.conv.cpu().numpy(), self.iters.cpu().numpy()


def time_ms(fn, reps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def tune(base, z, syn, llr, max_iter, *, difficulty=None, acc_bits=0, cache_path=DEFAULT_CACHE, reps=3, warmup=1,
         cands=None, use_cache=True) -> dict:
    """Fastest schedule for decoding batches shaped like (syn, llr)."""
    import torch
    key = _key(base, z, llr.shape[0], max_iter, acc_bits, difficulty is not None)
    cache = {}
    if use_cache and cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cands = cands if cands is not None else candidates(n_cu, difficulty is not None, int(z))
    results, ref = [], None
    for sched in cands:
        try:
            run = Runner(base, z, syn, llr, max_iter, sched, difficulty, acc_bits)
        except B.LdpcError as e:
            if e.code == B.LDPC_EUNSUPPORTED:
                continue
            raise
        ms = time_ms(run, reps, warmup)
        out = run.outputs()
        if ref is None:
            ref = out
        elif not all(np.array_equal(a, b) for a, b in zip(ref, out)):
            raise RuntimeError(f"schedule {sched} changed the decoded results")
        results.append({"schedule": asdict(sched), "row_tile": row_tile(run.code.plan()["kernel"]),
                        "ms": round(ms, 4)})
        del run
    if not results:
        raise RuntimeError("no schedule applies")
    best = min(results, key=lambda r: r["ms"])
    entry = {"schedule": best["schedule"], "ms": best["ms"], "candidates": results}
    if cache_path:
        cache[key] = entry
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return entry
