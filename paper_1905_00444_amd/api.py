"""Python binding of the qFlex-style amplitude library (thin: marshalling only).

Every step of the computation runs in the HIP kernels behind include/qfmi.h; PyTorch only
provides device memory (the workspace, inputs and outputs) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import check, load
from .gates import gate_entries, is_two_qubit

PRECISIONS = {"fp32": _lib.QF_FP32, "bf16x3": _lib.QF_BF16X3, "fp16": _lib.QF_FP16}


def _torch():
    import torch
    return torch


class Context:
    """A device, a stream and a growable workspace (a torch uint8 buffer)."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(self.lib.qf_ctx_create(device, C.c_void_p(self.stream.cuda_stream), None, 0, C.byref(h)))
        self.h = h
        self.ws = None

    def ensure_workspace(self, nbytes: int) -> None:
        """Grow the workspace to at least nbytes.  The old buffer may still be in use by work
        queued on the context's stream: it is released only after that work (the stream is
        synchronised first), and the new one is allocated on the context's stream so that the
        caching allocator orders its reuse after the library's kernels."""
        torch = _torch()
        nbytes = max(int(nbytes), 4096)
        if self.ws is None or self.ws.numel() < nbytes:
            if self.ws is not None:
                self.stream.synchronize()
                self.ws = None
            with torch.cuda.stream(self.stream):
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            check(self.lib.qf_ctx_set_workspace(self.h, C.c_void_p(self.ws.data_ptr()), self.ws.numel()), self.h)

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if self.h:
            self.lib.qf_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def read_circuit_text(text: str):
    """(rows, cols, removed, n, ops) with ops = [(cycle, name, qubits)] from the text format:
    '# grid rows cols [r:c ...]', the qubit count, then '<cycle> <name> <q0> [<q1>]' lines."""
    rows = cols = None
    removed = []
    n = None
    ops = []
    for raw in text.splitlines():
        s = raw.strip()
        if not s:
            continue
        if s.startswith("#"):
            f = s[1:].split()
            if f and f[0] == "grid":
                rows, cols = int(f[1]), int(f[2])
                removed = [tuple(int(v) for v in x.split(":")) for x in f[3:]]
            continue
        if n is None:
            n = int(s)
            continue
        f = s.split()
        ops.append((int(f[0]), f[1], tuple(int(v) for v in f[2:])))
    if rows is None:
        rows, cols = 1, n
    return rows, cols, removed, n, ops


class Circuit:
    def __init__(self, ctx: Context, text: str):
        self.ctx = ctx
        self.text = text
        rows, cols, removed, n, ops = read_circuit_text(text)
        self.rows, self.cols, self.n = rows, cols, n
        present = np.ones(rows * cols, dtype=np.uint8)
        for r, c in removed:
            present[r * cols + c] = 0
        arr = (_lib.qf_op * len(ops))()
        self.values = np.zeros((len(ops), 4), dtype=np.complex64)
        for i, (cyc, name, qs) in enumerate(ops):
            ent = gate_entries(name)
            self.values[i] = ent
            arr[i].cycle = cyc
            if len(qs) == 1:
                arr[i].kind, arr[i].q0, arr[i].q1 = _lib.QF_OP_1Q, qs[0], -1
            else:
                if not is_two_qubit(name):
                    raise ValueError(f"{name} is not a diagonal two-qubit gate")
                arr[i].kind, arr[i].q0, arr[i].q1 = _lib.QF_OP_2Q_DIAG, qs[0], qs[1]
            for j in range(4):
                arr[i].values[2 * j] = float(ent[j].real)
                arr[i].values[2 * j + 1] = float(ent[j].imag)
        self.ops = ops
        self._present = present
        h = C.c_void_p()
        check(ctx.lib.qf_circuit_create(ctx.h, rows, cols, present.ctypes.data_as(C.c_void_p), len(ops), arr,
                                        C.byref(h)), ctx.h)
        self.h = h

    def set_values(self, values: np.ndarray) -> None:
        """values: (n_ops, 4) complex entries in op order."""
        v = np.ascontiguousarray(np.asarray(values, dtype=np.complex64).reshape(-1, 4))
        flat = v.view(np.float32).reshape(-1)
        check(self.ctx.lib.qf_circuit_set_values(self.h, flat.ctypes.data_as(C.POINTER(C.c_float))), self.ctx.h)
        self.values = v.copy()

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.qf_circuit_destroy(self.h)
                self.h = None
        except Exception:
            pass


class Plan:
    def __init__(self, ctx: Context, circuit: Circuit, plan: dict, precision: str = "fp32", hoist: bool = True,
                 backward: bool = False, batch: int = 1, graph: bool = False, renorm: bool = True):
        """renorm: keep a power-of-two exponent per stored tensor on the device (default); False
        stores every tensor at its true scale (backward plans always do)."""
        self.ctx = ctx
        self.circuit = circuit
        self.plan = plan
        self.precision = precision
        steps = np.ascontiguousarray(np.asarray(plan["steps"], dtype=np.int32).reshape(-1))
        cuts = plan.get("cuts", [])
        carr = (_lib.qf_cut * max(1, len(cuts)))()
        for i, (q0, q1, lo, nb) in enumerate(cuts):
            carr[i].q0, carr[i].q1, carr[i].bit_lo, carr[i].nbits = q0, q1, lo, nb
        opn = np.ascontiguousarray(np.asarray(plan.get("open", []), dtype=np.int32))
        self._keep = (steps, carr, opn)
        d = _lib.qf_plan_desc()
        d.n_steps = len(steps) // 2
        d.steps = steps.ctypes.data_as(C.POINTER(C.c_int32))
        d.n_cuts = len(cuts)
        d.cuts = carr
        d.n_open = len(opn)
        d.open = opn.ctypes.data_as(C.POINTER(C.c_int32)) if len(opn) else None
        d.precision = PRECISIONS[precision]
        d.flags = ((0 if hoist else _lib.QF_PLAN_NO_HOIST) | (_lib.QF_PLAN_BACKWARD if backward else 0)
                   | (_lib.QF_PLAN_GRAPH if graph else 0) | (0 if renorm else _lib.QF_PLAN_NO_RENORM))
        d.batch = int(batch)
        h = C.c_void_p()
        check(ctx.lib.qf_plan_create(ctx.h, circuit.h, C.byref(d), C.byref(h)), ctx.h)
        self.h = h
        self.n_open = len(opn)
        self._info = None

    def info(self) -> dict:
        """Sizes, flops and workspace of the plan (qf_plan_info_get; fixed at creation, read once)."""
        if self._info is None:
            inf = _lib.qf_plan_info()
            check(self.ctx.lib.qf_plan_info_get(self.h, C.byref(inf)), self.ctx.h)
            self._info = {k: getattr(inf, k) for k, _ in _lib.qf_plan_info._fields_}
        return dict(self._info)

    def steps(self) -> list:
        """Per-step layout the plan chose (TTGT roles, GEMM sizes, which operands are copied)."""
        out = []
        for i in range(self.info()["n_steps"]):
            si = _lib.qf_step_info()
            check(self.ctx.lib.qf_plan_step_info(self.h, i, C.byref(si)), self.ctx.h)
            out.append({k: getattr(si, k) for k, _ in _lib.qf_step_info._fields_})
        return out

    def graph_info(self) -> tuple:
        """(hipGraphLaunch calls so far, nodes of the captured graph) of a graph-captured plan."""
        launches, nodes = C.c_int64(), C.c_int64()
        check(self.ctx.lib.qf_plan_graph_info(self.h, C.byref(launches), C.byref(nodes)), self.ctx.h)
        return launches.value, nodes.value

    def flops(self, s_begin: int, s_end: int) -> float:
        """Executed algorithmic flops for one bitstring over slices [s_begin, s_end)."""
        f = C.c_double()
        check(self.ctx.lib.qf_plan_flops(self.h, int(s_begin), int(s_end), C.byref(f)), self.ctx.h)
        return f.value

    def amplitudes(self, bits, s_begin: int = 0, s_end: Optional[int] = None, out=None):
        """Amplitudes (n_batch, 2^n_open) complex128 on the device, summed over slices
        [s_begin, s_end) and added into `out` if given.  Everything is enqueued on the
        context's stream."""
        torch = _torch()
        info = self.info()
        if s_end is None:
            s_end = info["n_slices"]
        self.ctx.ensure_workspace(info["workspace_bytes"])
        with torch.cuda.stream(self.ctx.stream):
            if isinstance(bits, np.ndarray):
                bits_t = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint8)).to(self.ctx.device)
            else:
                bits_t = bits.to(device=self.ctx.device, dtype=torch.uint8).contiguous()
            nb = bits_t.shape[0]
            if out is None:
                out = torch.zeros((nb, 2 ** self.n_open), dtype=torch.complex128, device=self.ctx.device)
            st = self.ctx.lib.qf_amplitudes(self.h, nb, C.c_void_p(bits_t.data_ptr()), int(s_begin), int(s_end),
                                            C.c_void_p(out.data_ptr()))
        self._bits_keepalive = bits_t
        check(st, self.ctx.h)
        return out

    def amplitudes_static(self, bits, s_begin: int = 0, s_end: Optional[int] = None, out=None):
        """As amplitudes(), through qf_amplitudes_static: the plan runs in the library's own
        64 MiB device array instead of the context's workspace (no allocation by the library;
        `bits` and `out` must already be device tensors when the caller cannot allocate)."""
        torch = _torch()
        if s_end is None:
            s_end = self.info()["n_slices"]
        with torch.cuda.stream(self.ctx.stream):
            if isinstance(bits, np.ndarray):
                bits = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint8)).to(self.ctx.device)
            nb = bits.shape[0]
            if out is None:
                out = torch.zeros((nb, 2 ** self.n_open), dtype=torch.complex128, device=self.ctx.device)
            assert bits.dtype == torch.uint8 and bits.is_contiguous() and out.dtype == torch.complex128
            st = self.ctx.lib.qf_amplitudes_static(self.h, nb, C.c_void_p(bits.data_ptr()), int(s_begin), int(s_end),
                                                   C.c_void_p(out.data_ptr()))
        self._bits_keepalive = bits
        check(st, self.ctx.h)
        return out

    def backward(self, bits, cot, s_begin: int = 0, s_end: Optional[int] = None, grad=None):
        """Gradient (n_ops, 4) complex64 of the amplitudes contracted with the cotangent `cot`
        (n_batch, 2^n_open complex128): grad_G = sum_b cot_b conj(d a_b / d G), added into `grad`."""
        torch = _torch()
        info = self.info()
        if s_end is None:
            s_end = info["n_slices"]
        self.ctx.ensure_workspace(info["workspace_bytes"])
        with torch.cuda.stream(self.ctx.stream):
            if isinstance(bits, np.ndarray):
                bits_t = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint8)).to(self.ctx.device)
            else:
                bits_t = bits.to(device=self.ctx.device, dtype=torch.uint8).contiguous()
            cot_t = torch.as_tensor(cot).to(device=self.ctx.device, dtype=torch.complex128).contiguous()
            assert cot_t.shape == (bits_t.shape[0], 2 ** self.n_open)
            if grad is None:
                grad = torch.zeros((len(self.circuit.ops), 4), dtype=torch.complex64, device=self.ctx.device)
            st = self.ctx.lib.qf_backward(self.h, bits_t.shape[0], C.c_void_p(bits_t.data_ptr()),
                                          C.c_void_p(cot_t.data_ptr()), int(s_begin), int(s_end),
                                          C.c_void_p(grad.data_ptr()))
        self._bwd_keepalive = (bits_t, cot_t)
        check(st, self.ctx.h)
        return grad

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.qf_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass


# --- kernel-level calls --------------------------------------------------------------------

def permute(ctx: Context, src, dst, perm: Sequence[int], base: int = 0, scale: float = 1.0) -> None:
    p = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
    check(ctx.lib.qf_permute(ctx.h, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), len(p),
                             p.ctypes.data_as(C.POINTER(C.c_int32)), int(base), float(scale)), ctx.h)


def cgemm(ctx: Context, A, B, precision: str = "fp32", out=None, variant: str = "auto"):
    """C[m, n] = sum_k A[m, k] B[n, k] (complex64, no conjugation); `variant` names a kernel
    variant (one of _lib.GEMM_VARIANTS) instead of the shape's default."""
    torch = _torch()
    M, K = A.shape
    N, K2 = B.shape
    assert K == K2 and A.dtype == torch.complex64 and B.dtype == torch.complex64
    A = A.contiguous()
    B = B.contiguous()
    if out is None:
        out = torch.empty((M, N), dtype=torch.complex64, device=A.device)
    if precision == "fp16":
        ctx.ensure_workspace(4096)
    check(ctx.lib.qf_cgemm_variant(ctx.h, PRECISIONS[precision], _lib.GEMM_VARIANTS.index(variant), M, N, K,
                                   C.c_void_p(A.data_ptr()), C.c_void_p(B.data_ptr()), C.c_void_p(out.data_ptr()),
                                   1, 0, 0, 0), ctx.h)
    return out


def split_bf16(ctx: Context, x, out=None):
    """Split-BF16 form of a complex64 tensor of 2^b elements: hi plane then lo plane (uint32 words)."""
    torch = _torch()
    n = x.numel()
    b = n.bit_length() - 1
    assert n == 1 << b and x.dtype == torch.complex64
    if out is None:
        out = torch.empty(2 * n, dtype=torch.int32, device=x.device)
    check(ctx.lib.qf_split_bf16(ctx.h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), b), ctx.h)
    return out


def split_f16(ctx: Context, x, scale_exp: int = 0, out=None):
    """FP16 form of a complex64 tensor of 2^b elements: one plane of fp16 (re, im) pairs of
    x * 2^scale_exp (uint32 words)."""
    torch = _torch()
    n = x.numel()
    b = n.bit_length() - 1
    assert n == 1 << b and x.dtype == torch.complex64
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=x.device)
    check(ctx.lib.qf_split_f16(ctx.h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), b, int(scale_exp)),
          ctx.h)
    return out


def cgemm_presplit(ctx: Context, As, Bs, M: int, N: int, K: int, out=None, lda: int = 0, ldb: int = 0,
                   precision: str = "bf16x3"):
    """C = A B^T from converted operands (split_bf16 for "bf16x3", split_f16 for "fp16");
    lda / ldb: words between rows of a plane (0: dense, K)."""
    torch = _torch()
    if out is None:
        out = torch.empty((M, N), dtype=torch.complex64, device=As.device)
    check(ctx.lib.qf_cgemm_presplit(ctx.h, PRECISIONS[precision], M, N, K, C.c_void_p(As.data_ptr()),
                                    C.c_void_p(Bs.data_ptr()), C.c_void_p(out.data_ptr()), lda, ldb), ctx.h)
    return out


def time_cgemm_presplit(ctx: Context, As, Bs, C_out, M: int, N: int, K: int, reps: int = 5, lda: int = 0,
                        ldb: int = 0, precision: str = "bf16x3") -> float:
    ms = C.c_float()
    check(ctx.lib.qf_time_cgemm_presplit(ctx.h, PRECISIONS[precision], M, N, K, C.c_void_p(As.data_ptr()),
                                         C.c_void_p(Bs.data_ptr()), C.c_void_p(C_out.data_ptr()), lda, ldb, reps,
                                         C.byref(ms)), ctx.h)
    return ms.value


def time_cgemm(ctx: Context, A, B, C_out, precision: str, reps: int = 5) -> float:
    M, K = A.shape
    N = B.shape[0]
    ms = C.c_float()
    if precision == "fp16":
        ctx.ensure_workspace(4096)
    check(ctx.lib.qf_time_cgemm(ctx.h, PRECISIONS[precision], M, N, K, C.c_void_p(A.data_ptr()),
                                C.c_void_p(B.data_ptr()), C.c_void_p(C_out.data_ptr()), reps, C.byref(ms)), ctx.h)
    return ms.value


def time_permute(ctx: Context, src, dst, perm: Sequence[int], reps: int = 5) -> float:
    p = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
    ms = C.c_float()
    check(ctx.lib.qf_time_permute(ctx.h, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), len(p),
                                  p.ctypes.data_as(C.POINTER(C.c_int32)), reps, C.byref(ms)), ctx.h)
    return ms.value


def time_ceiling(ctx: Context, kind: str, precision: str = "bf16x3", size: int = 0, buf=None, reps: int = 3):
    """Measured ceiling of the card (qf_time_ceiling): kind "copy" streams size / 2 bytes of buf (a
    device tensor of size bytes, allocated here if None) into its other half; kind "mfma" runs
    `size` trips of the register-only MFMA loop of `precision`.  Returns (ms per launch, work of
    one launch: bytes moved or real flops)."""
    torch = _torch()
    kinds = {"copy": 0, "mfma": 1}
    if buf is None:
        n = size if kind == "copy" else 4
        with torch.cuda.stream(ctx.stream):
            buf = torch.empty(n, dtype=torch.uint8, device=ctx.device)
    ms = C.c_float()
    work = C.c_double()
    check(ctx.lib.qf_time_ceiling(ctx.h, kinds[kind], PRECISIONS[precision], C.c_void_p(buf.data_ptr()), int(size),
                                  int(reps), C.byref(ms), C.byref(work)), ctx.h)
    return ms.value, work.value


def profile_enable(ctx: Context, on: bool = True) -> None:
    check(ctx.lib.qf_profile_enable(ctx.h, 1 if on else 0), ctx.h)


def profile_read(ctx: Context, reset: bool = True):
    ms = C.c_double()
    n = C.c_int64()
    fl = C.c_double()
    check(ctx.lib.qf_profile_read(ctx.h, C.byref(ms), C.byref(n), C.byref(fl), 1 if reset else 0), ctx.h)
    return ms.value, n.value, fl.value


def autotune(plan: "Plan", cache_path: Optional[str] = None) -> None:
    """Time the GEMM kernel variants for every GEMM shape of `plan` and install the fastest in the
    plan's context (qf_autotune); cache_path: JSON file read first and rewritten."""
    ctx = plan.ctx
    ctx.ensure_workspace(plan.info()["workspace_bytes"])
    path = None if cache_path is None else os.fsencode(cache_path)
    with _torch().cuda.stream(ctx.stream):
        check(ctx.lib.qf_autotune(ctx.h, plan.h, path), ctx.h)


def tuned_variant(ctx: Context, precision: str, M: int, N: int, K: int, batch: int = 1) -> str:
    """Name of the GEMM variant installed for a shape on this context ("auto" if none)."""
    v = C.c_int()
    check(ctx.lib.qf_tuned_variant(ctx.h, PRECISIONS[precision], int(M), int(N), int(K), int(batch), C.byref(v)),
          ctx.h)
    return _lib.GEMM_VARIANTS[v.value]


def amplitudes(circuit_text: str, plan: dict, bits, precision: str = "bf16x3", ctx: Optional[Context] = None,
               s_begin: int = 0, s_end: Optional[int] = None):
    """One-call form: amplitudes (n_batch, 2^n_open) complex128 on the device for the bitstrings
    `bits` (n_batch x n, 0/1) of the circuit in text form, contracted with `plan` over slices
    [s_begin, s_end) (all slices by default: the whole amplitudes)."""
    ctx = ctx if ctx is not None else Context(0)
    p = Plan(ctx, Circuit(ctx, circuit_text), plan, precision)
    return p.amplitudes(bits, s_begin, s_end)
