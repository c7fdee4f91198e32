"""Thin Python binding of libqkdldpc.so (include/qkdldpc.h).

Argument marshalling only: every step of decoding runs in the library's HIP
kernels. Tensors are torch tensors on the GPU (device pointers); the binding
checks their dtype, device, contiguity and shape on the host before any call,
so that a kernel never runs on buffers smaller than it assumes. The library is
required: when it is not built, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqkdldpc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qkdldpc.h")

LDPC_OK = 0
LDPC_EINVAL = -1
LDPC_ENOMEM = -2
LDPC_EDEVICE = -3
LDPC_EUNSUPPORTED = -4

LDPC_RULE_RCBP_FB = 0
LDPC_RULE_RCBP_EQ7 = 1
LDPC_RULE_MINSUM = 2

KERNEL_NAMES = {0: "global", 1: "lds", 2: "pairs", 3: "split", 4: "split_global_l", 5: "layer_sync",
                6: "split_reg"}
KERNEL_HINTS = {"auto": 0, "global": 1, "lds": 2, "pairs": 3, "split": 4, "split_global_l": 5, "layer_sync": 6,
                "split_reg": 7}
PERSISTENT_FAMILIES = ("split_reg", "split", "split_global_l")


class LdpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class ldpc_params(C.Structure):
    _fields_ = [("msg_max", C.c_int32), ("e_max", C.c_int32), ("acc_bits", C.c_int32),
                ("cn_rule", C.c_int32), ("offsets", C.c_void_p), ("offset_iters", C.c_int32),
                ("kernel_hint", C.c_int32)]


class ldpc_schedule(C.Structure):
    _fields_ = [("persistent_workgroups", C.c_int32), ("order", C.c_void_p), ("check_every", C.c_int32),
                ("frames_per_workgroup", C.c_int32)]


_lib = None


def lib():
    """Load the library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1903_10107_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname. Loading torch
        # first makes the library bind to that runtime, so device pointers and
        # streams from torch are valid in it; loading the library first would
        # bring in a second HIP runtime, and torch's device init then fails.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ldpc_code_create.restype = C.c_int
        L.ldpc_code_create.argtypes = [vp, i32, i32, i32, C.POINTER(ldpc_params), C.POINTER(vp)]
        L.ldpc_code_destroy.restype = None
        L.ldpc_code_destroy.argtypes = [vp]
        L.ldpc_code_dims.restype = C.c_int
        L.ldpc_code_dims.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64), C.POINTER(i32),
                                     C.POINTER(i32)]
        L.ldpc_decode_batch.restype = C.c_int
        L.ldpc_decode_batch.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
        L.ldpc_decode_batch_ex.restype = C.c_int
        L.ldpc_decode_batch_ex.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.ldpc_code_plan.restype = C.c_int
        L.ldpc_code_plan.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.ldpc_workspace_bytes.restype = C.c_size_t
        L.ldpc_workspace_bytes.argtypes = [vp, i32]
        L.ldpc_decode_batch_sched.restype = C.c_int
        L.ldpc_decode_batch_sched.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, C.POINTER(ldpc_schedule), vp,
                                              C.c_size_t, vp]
        L.ldpc_decode_batch_static.restype = C.c_int
        L.ldpc_decode_batch_static.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, C.POINTER(ldpc_schedule), vp]
        L.ldpc_workspace_bytes_sched.restype = C.c_size_t
        L.ldpc_workspace_bytes_sched.argtypes = [vp, i32, C.POINTER(ldpc_schedule)]
        L.ldpc_batch_create.restype = C.c_int
        L.ldpc_batch_create.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, C.POINTER(ldpc_schedule), vp, C.c_size_t,
                                        C.POINTER(vp)]
        L.ldpc_batch_launch.restype = C.c_int
        L.ldpc_batch_launch.argtypes = [vp, vp]
        L.ldpc_batch_destroy.restype = None
        L.ldpc_batch_destroy.argtypes = [vp]
        L.ldpc_syndrome_batch.restype = C.c_int
        L.ldpc_syndrome_batch.argtypes = [vp, vp, i32, vp, vp]
        L.ldpc_order_by_unsat.restype = C.c_int
        L.ldpc_order_by_unsat.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.ldpc_probe_lds_bandwidth.restype = C.c_int
        L.ldpc_probe_lds_bandwidth.argtypes = [i32, i32, i32, vp, vp]
        L.ldpc_last_error.restype = C.c_char_p
        L.ldpc_last_error.argtypes = []
        L.ldpc_version.restype = C.c_int
        L.ldpc_version.argtypes = []
        L.ldpc_host_tau_table.restype = C.c_int
        L.ldpc_host_tau_table.argtypes = [vp]
        L.ldpc_host_fold_pair.restype = C.c_int
        L.ldpc_host_fold_pair.argtypes = [i32, vp, vp, i32, vp, vp]
        L.ldpc_reveal_batch.restype = C.c_int
        L.ldpc_reveal_batch.argtypes = [vp, vp, i32, vp, i32, vp, vp, i32, vp]
        L.ldpc_oms_tape_bytes.restype = C.c_size_t
        L.ldpc_oms_tape_bytes.argtypes = [vp, i32, i32]
        L.ldpc_oms_workspace_bytes.restype = C.c_size_t
        L.ldpc_oms_workspace_bytes.argtypes = [vp, i32, i32]
        L.ldpc_oms_forward.restype = C.c_int
        L.ldpc_oms_forward.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, C.c_size_t, vp, C.c_size_t, vp]
        L.ldpc_oms_backward.restype = C.c_int
        L.ldpc_oms_backward.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp, C.c_size_t, vp, vp, vp, C.c_size_t,
                                        vp]
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/qkdldpc.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpc_[a-z0-9_]+)\s*\(", txt)))


def _check(rc: int):
    if rc != LDPC_OK:
        raise LdpcError(rc, lib().ldpc_last_error().decode())


def ldpc_probe_lds_bandwidth(mode: int, n_workgroups: int, reps: int, out, stream=None):
    """LDS read-bandwidth probe (mode 0: 16-byte reads, 1: byte reads) into the
    device uint32 tensor out[n_workgroups * 1024]."""
    import torch
    p_out = _dev_ptr(out, torch.int32, (int(n_workgroups) * 1024,), "out")
    _check(lib().ldpc_probe_lds_bandwidth(int(mode), int(n_workgroups), int(reps), p_out, _stream_ptr(stream)))


def ldpc_last_error() -> str:
    return lib().ldpc_last_error().decode()


def ldpc_version() -> int:
    return lib().ldpc_version()


def ldpc_host_tau_table() -> np.ndarray:
    out = np.zeros((64, 64), dtype=np.int32)
    _check(lib().ldpc_host_tau_table(out.ctypes.data))
    return out


class Code:
    """A QC-LDPC code handle (ldpc_code_create / ldpc_code_destroy)."""

    def __init__(self, base, z: int, *, msg_max: int = 0, e_max: int = 0, acc_bits: int = 0,
                 cn_rule: int = LDPC_RULE_RCBP_FB, offsets=None, kernel: str = "auto"):
        self._h = None
        base = np.ascontiguousarray(base, dtype=np.int32)
        if base.ndim != 2:
            raise ValueError("base must be a 2-D array")
        self.base = base
        self.z = int(z)
        self._offsets = None
        prm = ldpc_params(msg_max, e_max, acc_bits, cn_rule, None, 0, KERNEL_HINTS[kernel])
        if offsets is not None:
            self._offsets = np.ascontiguousarray(offsets, dtype=np.int8)
            if self._offsets.ndim != 2 or self._offsets.shape[1] != int((base >= 0).sum()):
                raise ValueError("offsets must be [offset_iters, n_blocks]")
            prm.offsets = self._offsets.ctypes.data
            prm.offset_iters = self._offsets.shape[0]
        h = C.c_void_p()
        _check(lib().ldpc_code_create(base.ctypes.data, base.shape[0], base.shape[1], self.z, C.byref(prm),
                                      C.byref(h)))
        self._h = h
        self.acc_bits = acc_bits or 8
        n, m, nb = C.c_int32(), C.c_int32(), C.c_int32()
        ne, h4 = C.c_int64(), C.c_int32()
        _check(lib().ldpc_code_dims(h, C.byref(n), C.byref(m), C.byref(ne), C.byref(nb), C.byref(h4)))
        self.n, self.m, self.n_edges, self.n_blocks = n.value, m.value, ne.value, nb.value
        self.has_4cycles = bool(h4.value)

    @property
    def handle(self):
        return self._h

    def plan(self) -> dict:
        """Kernel family, workgroup size and dynamic LDS of this code's decodes."""
        k, t, l = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().ldpc_code_plan(self._h, C.byref(k), C.byref(t), C.byref(l)))
        return {"kernel": KERNEL_NAMES[k.value], "threads": t.value, "lds_bytes": l.value}

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ldpc_code_destroy(self._h)
            self._h = None


def _dev_ptr(t, dtype, shape, name):
    """Host-side check of a device tensor before its pointer goes to a kernel."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < int(np.prod(shape)):
        raise ValueError(f"{name} has {t.numel()} elements; needs {int(np.prod(shape))} ({shape})")
    return t.data_ptr()


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def ldpc_workspace_bytes(code: Code, n_frames: int) -> int:
    return int(lib().ldpc_workspace_bytes(code.handle, int(n_frames)))


def ldpc_decode_batch_ex(code: Code, syndromes, llr_in, n_frames: int, max_iter: int, out_bits, out_converged,
                         out_iters=None, out_L=None, out_E=None, workspace=None, stream=None):
    import torch
    F = int(n_frames)
    sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
    if F < 0:
        raise ValueError("n_frames < 0")
    if F == 0:
        return
    p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
    p_llr = _dev_ptr(llr_in, torch.int8, (F, code.n), "llr_in")
    p_bits = _dev_ptr(out_bits, torch.uint8, (F, bb), "out_bits")
    p_conv = _dev_ptr(out_converged, torch.uint8, (F,), "out_converged")
    p_it = _dev_ptr(out_iters, torch.int32, (F,), "out_iters")
    p_L = _dev_ptr(out_L, torch.int8, (F, code.n_blocks, code.z), "out_L")
    p_E = _dev_ptr(out_E, torch.int16, (F, code.n), "out_E")
    need = ldpc_workspace_bytes(code, F)
    p_ws, ws_bytes = None, 0
    if workspace is not None:
        p_ws = _dev_ptr(workspace, torch.uint8, (need,), "workspace")
        ws_bytes = workspace.numel()
    _check(lib().ldpc_decode_batch_ex(code.handle, p_syn, p_llr, F, int(max_iter), p_bits, p_conv, p_it, p_L, p_E,
                                      p_ws, ws_bytes, _stream_ptr(stream)))


def ldpc_decode_batch(code: Code, syndromes, llr_in, n_frames: int, max_iter: int, out_bits, out_converged,
                      stream=None):
    import torch
    F = int(n_frames)
    if F < 0:
        raise ValueError("n_frames < 0")
    if F == 0:
        return
    sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
    p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
    p_llr = _dev_ptr(llr_in, torch.int8, (F, code.n), "llr_in")
    p_bits = _dev_ptr(out_bits, torch.uint8, (F, bb), "out_bits")
    p_conv = _dev_ptr(out_converged, torch.uint8, (F,), "out_converged")
    _check(lib().ldpc_decode_batch(code.handle, p_syn, p_llr, F, int(max_iter), p_bits, p_conv, _stream_ptr(stream)))


def _schedule(n_frames: int, persistent_workgroups: int, order, check_every: int = 0,
              frames_per_workgroup: int = 0):
    import torch
    p_order = _dev_ptr(order, torch.int32, (n_frames,), "order")
    return ldpc_schedule(int(persistent_workgroups), p_order, int(check_every), int(frames_per_workgroup))


def ldpc_workspace_bytes_sched(code: Code, n_frames: int, persistent_workgroups: int = 0) -> int:
    sch = ldpc_schedule(int(persistent_workgroups), None)
    return int(lib().ldpc_workspace_bytes_sched(code.handle, int(n_frames), C.byref(sch)))


def ldpc_decode_batch_sched(code: Code, syndromes, llr_in, n_frames: int, max_iter: int, out_bits, out_converged,
                            out_iters=None, persistent_workgroups: int = 0, order=None, workspace=None, stream=None,
                            check_every: int = 0, frames_per_workgroup: int = 0):
    import torch
    F = int(n_frames)
    if F < 0:
        raise ValueError("n_frames < 0")
    if F == 0:
        return
    sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
    p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
    p_llr = _dev_ptr(llr_in, torch.int8, (F, code.n), "llr_in")
    p_bits = _dev_ptr(out_bits, torch.uint8, (F, bb), "out_bits")
    p_conv = _dev_ptr(out_converged, torch.uint8, (F,), "out_converged")
    p_it = _dev_ptr(out_iters, torch.int32, (F,), "out_iters")
    sch = _schedule(F, persistent_workgroups, order, check_every, frames_per_workgroup)
    need = int(lib().ldpc_workspace_bytes_sched(code.handle, F, C.byref(sch)))
    p_ws, ws_bytes = None, 0
    if workspace is not None:
        p_ws = _dev_ptr(workspace, torch.uint8, (need,), "workspace")
        ws_bytes = workspace.numel()
    _check(lib().ldpc_decode_batch_sched(code.handle, p_syn, p_llr, F, int(max_iter), p_bits, p_conv, p_it,
                                         C.byref(sch), p_ws, ws_bytes, _stream_ptr(stream)))


STATIC_WORKSPACE_BYTES = 64 << 20   # LDPC_STATIC_WORKSPACE_BYTES


def ldpc_decode_batch_static(code: Code, syndromes, llr_in, n_frames: int, max_iter: int, out_bits, out_converged,
                             out_iters=None, persistent_workgroups: int = 0, order=None, stream=None,
                             check_every: int = 0, frames_per_workgroup: int = 0):
    """ldpc_decode_batch_sched with the library's static workspace (no device
    allocation by the library or here)."""
    import torch
    F = int(n_frames)
    if F < 0:
        raise ValueError("n_frames < 0")
    if F == 0:
        return
    sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
    p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
    p_llr = _dev_ptr(llr_in, torch.int8, (F, code.n), "llr_in")
    p_bits = _dev_ptr(out_bits, torch.uint8, (F, bb), "out_bits")
    p_conv = _dev_ptr(out_converged, torch.uint8, (F,), "out_converged")
    p_it = _dev_ptr(out_iters, torch.int32, (F,), "out_iters")
    sch = _schedule(F, persistent_workgroups, order, check_every, frames_per_workgroup)
    _check(lib().ldpc_decode_batch_static(code.handle, p_syn, p_llr, F, int(max_iter), p_bits, p_conv, p_it,
                                          C.byref(sch), _stream_ptr(stream)))


class Batch:
    """A decode of fixed device buffers captured as a HIP graph (ldpc_batch_*)."""

    def __init__(self, code: Code, syndromes, llr_in, n_frames: int, max_iter: int, out_bits, out_converged,
                 out_iters=None, persistent_workgroups: int = 0, order=None, workspace=None, check_every: int = 0,
                 frames_per_workgroup: int = 0):
        import torch
        self._h = None
        F = int(n_frames)
        sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
        self._keep = (code, syndromes, llr_in, out_bits, out_converged, out_iters, order, workspace)
        p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
        p_llr = _dev_ptr(llr_in, torch.int8, (F, code.n), "llr_in")
        p_bits = _dev_ptr(out_bits, torch.uint8, (F, bb), "out_bits")
        p_conv = _dev_ptr(out_converged, torch.uint8, (F,), "out_converged")
        p_it = _dev_ptr(out_iters, torch.int32, (F,), "out_iters")
        sch = _schedule(F, persistent_workgroups, order, check_every, frames_per_workgroup)
        need = int(lib().ldpc_workspace_bytes_sched(code.handle, F, C.byref(sch)))
        p_ws, ws_bytes = None, 0
        if workspace is not None:
            p_ws = _dev_ptr(workspace, torch.uint8, (need,), "workspace")
            ws_bytes = workspace.numel()
        h = C.c_void_p()
        _check(lib().ldpc_batch_create(code.handle, p_syn, p_llr, F, int(max_iter), p_bits, p_conv, p_it,
                                       C.byref(sch), p_ws, ws_bytes, C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().ldpc_batch_launch(self._h, _stream_ptr(stream)))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ldpc_batch_destroy(self._h)
            self._h = None


def ldpc_syndrome_batch(code: Code, bits, n_frames: int, out_syn, stream=None):
    import torch
    F = int(n_frames)
    if F <= 0:
        if F < 0:
            raise ValueError("n_frames < 0")
        return
    p_b = _dev_ptr(bits, torch.uint8, (F, (code.n + 7) // 8), "bits")
    p_s = _dev_ptr(out_syn, torch.uint8, (F, (code.m + 7) // 8), "out_syn")
    _check(lib().ldpc_syndrome_batch(code.handle, p_b, F, p_s, _stream_ptr(stream)))


def ldpc_order_by_unsat(code: Code, syndromes, llr_in, n_frames: int, out_unsat, out_order=None, stream=None):
    import torch
    F = int(n_frames)
    if F <= 0:
        if F < 0:
            raise ValueError("n_frames < 0")
        return
    p_s = _dev_ptr(syndromes, torch.uint8, (F, (code.m + 7) // 8), "syndromes")
    p_l = _dev_ptr(llr_in, torch.int8, (F, code.n), "llr_in")
    p_w = _dev_ptr(out_unsat, torch.int32, (F,), "out_unsat")
    p_o = _dev_ptr(out_order, torch.int32, (F,), "out_order") if out_order is not None else None
    _check(lib().ldpc_order_by_unsat(code.handle, p_s, p_l, F, p_w, p_o, _stream_ptr(stream)))


def decode(code: Code, syn, llr, max_iter: int, *, want_state: bool = False, device: str = "cuda"):
    """numpy in, numpy out: uploads, decodes on the GPU, downloads."""
    import torch
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    llr = np.ascontiguousarray(llr, dtype=np.int8)
    F = llr.shape[0]
    d_syn = torch.from_numpy(syn).to(device)
    d_llr = torch.from_numpy(llr).to(device)
    bits = torch.zeros((F, (code.n + 7) // 8), dtype=torch.uint8, device=device)
    conv = torch.zeros(F, dtype=torch.uint8, device=device)
    iters = torch.zeros(F, dtype=torch.int32, device=device)
    L = torch.zeros((F, code.n_blocks, code.z), dtype=torch.int8, device=device) if want_state else None
    E = torch.zeros((F, code.n), dtype=torch.int16, device=device) if want_state else None
    ldpc_decode_batch_ex(code, d_syn, d_llr, F, max_iter, bits, conv, iters, L, E)
    torch.cuda.synchronize()
    out = {"bits": bits.cpu().numpy(), "conv": conv.cpu().numpy(), "iters": iters.cpu().numpy()}
    if want_state:
        out["L"], out["E"] = L.cpu().numpy(), E.cpu().numpy()
    return out


def ldpc_reveal_batch(code: Code, llr, n_frames: int, frame_ids, positions, values, stream=None):
    """Set the LLRs of revealed positions to +-127 (see include/qkdldpc.h).
    frame_ids int32 [k], positions int32 [k, r], values uint8 [k, r], all on the GPU."""
    import torch
    F = int(n_frames)
    k = int(frame_ids.numel()) if frame_ids is not None else 0
    r = int(positions.shape[1]) if positions is not None and positions.dim() == 2 else 0
    if k == 0 or r == 0:
        return
    p_llr = _dev_ptr(llr, torch.int8, (F, code.n), "llr")
    p_id = _dev_ptr(frame_ids, torch.int32, (k,), "frame_ids")
    p_pos = _dev_ptr(positions, torch.int32, (k, r), "positions")
    p_val = _dev_ptr(values, torch.uint8, (k, r), "values")
    _check(lib().ldpc_reveal_batch(code.handle, p_llr, F, p_id, k, p_pos, p_val, r, _stream_ptr(stream)))


# --- differentiable offset min-sum ---------------------------------------------

def ldpc_oms_tape_bytes(code: Code, n_frames: int, n_iter: int) -> int:
    return int(lib().ldpc_oms_tape_bytes(code.handle, int(n_frames), int(n_iter)))


def ldpc_oms_workspace_bytes(code: Code, n_frames: int, n_iter: int) -> int:
    return int(lib().ldpc_oms_workspace_bytes(code.handle, int(n_frames), int(n_iter)))


def ldpc_oms_forward(code: Code, syndromes, llr, target_bits, n_frames: int, n_iter: int, beta, loss_weights,
                     out_loss, out_E, tape, workspace=None, stream=None):
    import torch
    F, T = int(n_frames), int(n_iter)
    sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
    p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
    p_llr = _dev_ptr(llr, torch.float32, (F, code.n), "llr")
    p_x = _dev_ptr(target_bits, torch.uint8, (F, bb), "target_bits")
    p_b = _dev_ptr(beta, torch.float32, (T, code.n_blocks), "beta")
    p_w = _dev_ptr(loss_weights, torch.float32, (T,), "loss_weights")
    p_l = _dev_ptr(out_loss, torch.float32, (F,), "out_loss")
    p_e = _dev_ptr(out_E, torch.float32, (F, code.n), "out_E")
    p_t = _dev_ptr(tape, torch.uint8, (ldpc_oms_tape_bytes(code, F, T),), "tape")
    need = ldpc_oms_workspace_bytes(code, F, T)
    p_ws = _dev_ptr(workspace, torch.uint8, (need,), "workspace") if workspace is not None else None
    _check(lib().ldpc_oms_forward(code.handle, p_syn, p_llr, p_x, F, T, p_b, p_w, p_l, p_e, p_t, tape.numel(),
                                  p_ws, workspace.numel() if workspace is not None else 0, _stream_ptr(stream)))


def ldpc_oms_backward(code: Code, syndromes, target_bits, n_frames: int, n_iter: int, beta, loss_weights, dloss,
                      tape, out_dbeta, out_dllr, workspace, stream=None):
    import torch
    F, T = int(n_frames), int(n_iter)
    sb, bb = (code.m + 7) // 8, (code.n + 7) // 8
    p_syn = _dev_ptr(syndromes, torch.uint8, (F, sb), "syndromes")
    p_x = _dev_ptr(target_bits, torch.uint8, (F, bb), "target_bits")
    p_b = _dev_ptr(beta, torch.float32, (T, code.n_blocks), "beta")
    p_w = _dev_ptr(loss_weights, torch.float32, (T,), "loss_weights")
    p_g = _dev_ptr(dloss, torch.float32, (F,), "dloss")
    p_t = _dev_ptr(tape, torch.uint8, (ldpc_oms_tape_bytes(code, F, T),), "tape")
    p_db = _dev_ptr(out_dbeta, torch.float32, (T, code.n_blocks), "out_dbeta")
    p_dl = _dev_ptr(out_dllr, torch.float32, (F, code.n), "out_dllr")
    need = ldpc_oms_workspace_bytes(code, F, T)
    p_ws = _dev_ptr(workspace, torch.uint8, (need,), "workspace") if workspace is not None else None
    _check(lib().ldpc_oms_backward(code.handle, p_syn, p_x, F, T, p_b, p_w, p_g, p_t, tape.numel(), p_db, p_dl,
                                   p_ws, workspace.numel() if workspace is not None else 0, _stream_ptr(stream)))


class OmsDecoder:
    """Differentiable FP32 offset min-sum of one code: per-frame training loss
    as a torch autograd function of the offsets beta [n_iter, n_blocks] and the
    channel LLRs, computed by the library's forward and backward kernels."""

    def __init__(self, base, z: int, n_iter: int, loss_weights=None):
        import torch
        self.code = Code(base, z)
        self.n_iter = int(n_iter)
        self.weights = None
        if loss_weights is not None:
            self.weights = torch.as_tensor(loss_weights, dtype=torch.float32).cuda().contiguous()

    def loss(self, syndromes, llr, target_bits, beta, want_E: bool = False):
        """Per-frame losses [F] (differentiable in beta and llr); with want_E also
        the soft values after the last iteration [F, n] (no gradient)."""
        out = _OmsFunction.apply(beta, llr, self, syndromes, target_bits)
        return out if want_E else out[0]


def _oms_function():
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, beta, llr, dec, syn, target):
            F, T, code = llr.shape[0], dec.n_iter, dec.code
            dev = llr.device
            tape = torch.empty(ldpc_oms_tape_bytes(code, F, T), dtype=torch.uint8, device=dev)
            need = ldpc_oms_workspace_bytes(code, F, T)
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
            loss = torch.empty(F, dtype=torch.float32, device=dev)
            E = torch.empty((F, code.n), dtype=torch.float32, device=dev)
            b = beta.detach().contiguous()
            ldpc_oms_forward(code, syn, llr.detach().contiguous(), target, F, T, b, dec.weights, loss, E, tape, ws)
            ctx.dec, ctx.syn, ctx.target, ctx.tape, ctx.ws, ctx.beta = dec, syn, target, tape, ws, b
            ctx.mark_non_differentiable(E)
            return loss, E

        @staticmethod
        def backward(ctx, dloss, _dE):
            dec, code = ctx.dec, ctx.dec.code
            F, T = ctx.syn.shape[0], dec.n_iter
            dbeta = torch.empty((T, code.n_blocks), dtype=torch.float32, device=dloss.device)
            dllr = torch.empty((F, code.n), dtype=torch.float32, device=dloss.device) if ctx.needs_input_grad[1] \
                else None
            ldpc_oms_backward(code, ctx.syn, ctx.target, F, T, ctx.beta, dec.weights, dloss.contiguous(), ctx.tape,
                              dbeta, dllr, ctx.ws)
            return dbeta, dllr, None, None, None

    return _Fn


class _LazyFn:
    _fn = None

    def apply(self, *args):
        if _LazyFn._fn is None:
            _LazyFn._fn = _oms_function()
        return _LazyFn._fn.apply(*args)


_OmsFunction = _LazyFn()
