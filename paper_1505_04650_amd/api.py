"""Python binding of the HIP compressed-NMF library.

Thin marshalling over the C ABI (include/cnmf.h): PyTorch provides device
memory and the stream; every step of the method runs in the library's HIP
kernels.  Functions allocate their outputs with torch on A's device and
enqueue on the current torch stream without synchronising.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

_DT = {torch.float64: L.CNMF_F64, torch.float32: L.CNMF_F32}
_PREC = {"f64": L.CNMF_F64, "f32": L.CNMF_F32, "bf16": L.CNMF_BF16, "fp8": L.CNMF_FP8_E4M3}
_SIDES = {"left": L.CNMF_LEFT, "right": L.CNMF_RIGHT, "both": L.CNMF_BOTH}
_METHODS = {"admm": L.CNMF_ADMM, "mu": L.CNMF_MU, "admm_full": L.CNMF_ADMM_FULL, "mu_full": L.CNMF_MU_FULL,
            "anls": L.CNMF_ANLS, "anls_full": L.CNMF_ANLS_FULL}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Handle:
    """A library handle bound to one device and one HIP stream."""

    def __init__(self, device=None, stream=None, workspace_limit: int = 0):
        lib = L.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = st
        h = C.c_void_p()
        L.check(lib.cnmf_create(dev.index, C.c_void_p(st.cuda_stream), workspace_limit, C.byref(h)))
        self._h = h
        self._lib = lib

    @property
    def raw(self):
        return self._h

    def close(self):
        if self._h:
            self._lib.cnmf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, enable: bool):
        L.check(self._lib.cnmf_set_timing(self._h, int(enable)), self._h)

    STAGES = ("convert", "pass_AX", "pass_ATZ", "orth", "iterations", "residual", "spa")

    def stages(self):
        """Per-stage (ms, flops, launches) of the last call (ms needs timing on)."""
        out = {}
        for i, name in enumerate(self.STAGES):
            out[name] = (self._lib.cnmf_stage_ms(self._h, i), self._lib.cnmf_stage_flops(self._h, i),
                         self._lib.cnmf_stage_launches(self._h, i))
        return out


_handles: dict = {}


def default_handle() -> Handle:
    dev = torch.cuda.current_device()
    st = torch.cuda.current_stream().cuda_stream
    key = (dev, st)
    h = _handles.get(key)
    if h is None:
        h = Handle(dev)
        _handles[key] = h
    return h


def _input(A: torch.Tensor, block_rows: int = 0) -> L.cnmf_input:
    """A as the library's input: a dense device tensor; a dense host tensor
    (streamed through the device in row blocks; pin it for overlapped
    copies); or a sparse CSR device tensor (torch.sparse_csr_tensor)."""
    if A.dtype not in _DT:
        raise TypeError("A must be float64 or float32")
    if A.layout == torch.sparse_csr:
        if A.device.type != "cuda":
            raise ValueError("a sparse A must be on the device")
        crow = A.crow_indices()
        col = A.col_indices().to(torch.int32).contiguous()
        vals = A.values().contiguous()
        if crow.dtype != torch.int64:
            crow = crow.to(torch.int64)
        inp = L.cnmf_input(_ptr(vals), _DT[A.dtype], A.shape[0], A.shape[1], A.shape[1], L.CNMF_CSR, 0,
                           _ptr(crow), _ptr(col), vals.numel(), 0)
        inp._keep = (crow, col, vals)       # alive until the call has enqueued its work
        return inp
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor (unit column stride)")
    fmt = L.CNMF_DENSE if A.device.type == "cuda" else L.CNMF_DENSE_HOST
    return L.cnmf_input(_ptr(A), _DT[A.dtype], A.shape[0], A.shape[1], A.stride(0), fmt, 0, None, None, 0,
                        int(block_rows))


def _out_device(A, h) -> torch.device:
    return A.device if A.device.type == "cuda" else h.device


def _after(A, h):
    """A host input is read by copies that run after the call returns: wait
    for them, so the caller may release or change A afterwards."""
    if A.device.type != "cuda":
        h.stream.synchronize()


_TEST = {"gaussian": L.CNMF_TEST_GAUSSIAN, "srht": L.CNMF_TEST_SRHT}


def _sketch_desc(r, k, q, sides, omega_left, omega_right, pass_dtype, final_dtype, seed=0, test_matrix="gaussian"):
    return L.cnmf_sketch_desc(int(r), int(k), int(q), _SIDES[sides] if isinstance(sides, str) else int(sides),
                              _PREC[pass_dtype], _PREC[final_dtype], int(seed) & (2 ** 64 - 1),
                              _ptr(omega_left), _ptr(omega_right), _TEST[test_matrix], 0)


def _acc_dtype(A, pass_dtype):
    return torch.float64 if pass_dtype == "f64" else torch.float32


def _default_prec(A, pass_dtype, final_dtype):
    if pass_dtype is None:
        pass_dtype = "f64" if A.dtype == torch.float64 else "f32"
    if final_dtype is None:
        final_dtype = "f64" if pass_dtype == "f64" else ("f32" if pass_dtype == "f32" else "bf16")
    return pass_dtype, final_dtype


@dataclass
class Sketch:
    L: torch.Tensor | None
    R: torch.Tensor | None
    B: torch.Tensor | None
    At: torch.Tensor | None
    Ac: torch.Tensor | None
    stats: torch.Tensor


def sketch(A, r, k, q, omega_left=None, omega_right=None, sides="both", pass_dtype=None, final_dtype=None,
           want_ac=False, seed=0, block_rows=0, test_matrix="gaussian", handle: Handle | None = None) -> Sketch:
    """Structured random compression (Alg. 1) of A on one or both sides, and
    the small sketches B = L^T A, At = L^T A R^T, Ac = A R^T.  A test matrix
    left as None is drawn on the device from `seed` (see gaussian())."""
    h = handle or default_handle()
    pass_dtype, final_dtype = _default_prec(A, pass_dtype, final_dtype)
    m, n = A.shape
    dev = _out_device(A, h)
    od = _acc_dtype(A, pass_dtype)
    sd = _SIDES[sides] if isinstance(sides, str) else sides
    left, right = bool(sd & 1), bool(sd & 2)
    Lt = torch.empty((m, k), dtype=od, device=dev) if left else None
    Rt = torch.empty((k, n), dtype=od, device=dev) if right else None
    Bt = torch.empty((k, n), dtype=od, device=dev) if left else None
    Att = torch.empty((k, k), dtype=od, device=dev) if (left and right) else None
    Act = torch.empty((m, k), dtype=od, device=dev) if (right and want_ac) else None
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    inp = _input(A, block_rows)
    d = _sketch_desc(r, k, q, sd, omega_left, omega_right, pass_dtype, final_dtype, seed, test_matrix)
    out = L.cnmf_sketch_out(_ptr(Lt), _ptr(Rt), _ptr(Bt), _ptr(Att), _ptr(Act), _ptr(stats))
    L.check(h._lib.cnmf_sketch(h.raw, C.byref(inp), C.byref(d), C.byref(out)), h.raw)
    _after(A, h)
    return Sketch(Lt, Rt, Bt, Att, Act, stats)


@dataclass
class Factorization:
    U: torch.Tensor
    V: torch.Tensor
    rel_residual: torch.Tensor
    sketch: Sketch | None


def factorize(A, r, k, q, U0, V0, omega_left=None, omega_right=None, method="admm", iters=100,
              lam=1.0, phi=None, xi=1.0, mu_eps=1e-16, pass_dtype=None, final_dtype=None,
              want_sketch=False, seed=0, block_rows=0, test_matrix="gaussian",
              handle: Handle | None = None) -> Factorization:
    """Compressed NMF: two-sided sketch, then ADMM (Alg. 3), MU (Alg. 2) or
    alternating NNLS (Section 3, Eq. alternateLS_nmf_compressed) on the
    compressed factors, then the FP64 relative residual.  The *_full methods
    run the same iterations uncompressed (L = I, R = I)."""
    h = handle or default_handle()
    pass_dtype, final_dtype = _default_prec(A, pass_dtype, final_dtype)
    m, n = A.shape
    dev = _out_device(A, h)
    od = _acc_dtype(A, pass_dtype)
    U = torch.empty((m, r), dtype=od, device=dev)
    V = torch.empty((r, n), dtype=od, device=dev)
    res = torch.zeros(1, dtype=torch.float64, device=dev)
    sk = None
    if want_sketch:
        sk = Sketch(torch.empty((m, k), dtype=od, device=dev), torch.empty((k, n), dtype=od, device=dev),
                    torch.empty((k, n), dtype=od, device=dev), torch.empty((k, k), dtype=od, device=dev),
                    torch.empty((m, k), dtype=od, device=dev) if method in ("mu", "anls") else None,
                    torch.zeros(4, dtype=torch.float64, device=dev))
        so = L.cnmf_sketch_out(_ptr(sk.L), _ptr(sk.R), _ptr(sk.B), _ptr(sk.At), _ptr(sk.Ac), _ptr(sk.stats))
    else:
        so = L.cnmf_sketch_out()
    U0 = U0.to(device=dev, dtype=torch.float64).contiguous()
    V0 = V0.to(device=dev, dtype=torch.float64).contiguous()
    inp = _input(A, block_rows)
    d = L.cnmf_factorize_desc(_sketch_desc(r, k, q, L.CNMF_BOTH, omega_left, omega_right, pass_dtype, final_dtype,
                                           seed, test_matrix),
                              _METHODS[method], int(iters), float(lam), float(lam if phi is None else phi),
                              float(xi), float(mu_eps), _ptr(U0), _ptr(V0))
    out = L.cnmf_factorize_out(_ptr(U), _ptr(V), _ptr(res), so)
    L.check(h._lib.cnmf_factorize(h.raw, C.byref(inp), C.byref(d), C.byref(out)), h.raw)
    _after(A, h)
    return Factorization(U, V, res, sk)


class FactorizeGraph:
    """One factorisation captured as a HIP graph (cnmf_factorize_capture) on
    a stream of its own, replayed by replay(): each replay recomputes the
    factorisation from the current contents of A, U0, V0 (and the test
    matrices) into U, V and rel_residual.  The arguments are those of
    factorize(); the tensors are kept alive by the object."""

    def __init__(self, A, r, k, q, U0, V0, omega_left=None, omega_right=None, method="admm", iters=100,
                 lam=1.0, phi=None, xi=1.0, mu_eps=1e-16, pass_dtype=None, final_dtype=None, seed=0,
                 test_matrix="gaussian"):
        if A.device.type != "cuda":
            raise ValueError("a captured factorisation takes a device A")
        self.stream = torch.cuda.Stream(device=A.device)
        self.handle = Handle(A.device.index, stream=self.stream)
        h = self.handle
        pass_dtype, final_dtype = _default_prec(A, pass_dtype, final_dtype)
        m, n = A.shape
        od = _acc_dtype(A, pass_dtype)
        dev = A.device
        self.U = torch.empty((m, r), dtype=od, device=dev)
        self.V = torch.empty((r, n), dtype=od, device=dev)
        self.rel_residual = torch.zeros(1, dtype=torch.float64, device=dev)
        self.U0 = U0.to(device=dev, dtype=torch.float64).contiguous()
        self.V0 = V0.to(device=dev, dtype=torch.float64).contiguous()
        self._keep = (A, omega_left, omega_right)
        torch.cuda.current_stream(dev).synchronize()   # inputs produced elsewhere are ready
        inp = _input(A)
        self._inp = inp
        d = L.cnmf_factorize_desc(_sketch_desc(r, k, q, L.CNMF_BOTH, omega_left, omega_right, pass_dtype,
                                               final_dtype, seed, test_matrix),
                                  _METHODS[method], int(iters), float(lam), float(lam if phi is None else phi),
                                  float(xi), float(mu_eps), _ptr(self.U0), _ptr(self.V0))
        out = L.cnmf_factorize_out(_ptr(self.U), _ptr(self.V), _ptr(self.rel_residual), L.cnmf_sketch_out())
        g = C.c_void_p()
        L.check(h._lib.cnmf_factorize_capture(h.raw, C.byref(inp), C.byref(d), C.byref(out), C.byref(g)), h.raw)
        self._g = g

    def replay(self):
        """Enqueue one factorisation on the graph's stream (returns at once)."""
        L.check(self.handle._lib.cnmf_graph_launch(self._g), self.handle.raw)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "_g", None):
            self.handle._lib.cnmf_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def select(A, r, k, q, omega_left=None, omega_right=None, sides="left", pass_dtype=None, final_dtype=None,
           want_scores=False, want_B=False, seed=0, block_rows=0, test_matrix="gaussian",
           handle: Handle | None = None):
    """Compressed separable NMF column selection (Alg. SNMF steps 1-2): the
    sketch, B = Q^T A, and SPA on B.  Returns int64 indices (device)."""
    h = handle or default_handle()
    pass_dtype, final_dtype = _default_prec(A, pass_dtype, final_dtype)
    dev = _out_device(A, h)
    K = torch.empty(r, dtype=torch.int64, device=dev)
    score = torch.empty(r, dtype=torch.float64, device=dev) if want_scores else None
    B = torch.empty((k, A.shape[1]), dtype=_acc_dtype(A, pass_dtype), device=dev) if want_B else None
    inp = _input(A, block_rows)
    d = _sketch_desc(r, k, q, sides, omega_left, omega_right, pass_dtype, final_dtype, seed, test_matrix)
    L.check(h._lib.snmf_select(h.raw, C.byref(inp), C.byref(d), _ptr(K), _ptr(score), _ptr(B)), h.raw)
    _after(A, h)
    return K, score, B


def snmf_nnls(B, K, want_info=False, handle: Handle | None = None):
    """Right factor of separable NMF on the compressed B (k x n device
    matrix) for the selected columns K (int64 device): H (r x n, FP64) with
    H[:, j] = argmin_{h >= 0} ||B[:, j] - B[:, K] h||."""
    h = handle or default_handle()
    if B.dtype not in _DT or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major float64/float32 2-D tensor")
    if K.dtype != torch.int64 or K.dim() != 1 or not K.is_contiguous():
        raise ValueError("K must be a contiguous int64 vector")
    r = K.shape[0]
    H = torch.empty((r, B.shape[1]), dtype=torch.float64, device=B.device)
    info = torch.zeros(3, dtype=torch.int32, device=B.device)
    L.check(h._lib.snmf_nnls(h.raw, _ptr(B), _DT[B.dtype], B.shape[0], B.shape[1], B.stride(0), int(r), _ptr(K),
                             _ptr(H), H.stride(0), _ptr(info)), h.raw)
    return (H, info) if want_info else H


def synchronize(handle: Handle | None = None):
    """Wait for the handle's stream; raises CnmfError(CNMF_EBREAKDOWN) when an
    orthonormalisation breakdown was left unresolved since the last call."""
    h = handle or default_handle()
    L.check(h._lib.cnmf_synchronize(h.raw), h.raw)


def gaussian(rows, cols, seed, matrix_id=0, device=None, handle: Handle | None = None):
    """The library's Gaussian test matrix `matrix_id` under `seed` (rows x
    cols FP64 on the device): id 0 is the sketch's Omega_L, id 1 Omega_R."""
    h = handle or default_handle()
    dev = h.device if device is None else torch.device(device)
    out = torch.empty((rows, cols), dtype=torch.float64, device=dev)
    L.check(h._lib.cnmf_gaussian(h.raw, int(seed) & (2 ** 64 - 1), int(matrix_id), int(rows), int(cols), _ptr(out),
                                 max(int(cols), 1)), h.raw)
    return out


def srht(rows, cols, seed, matrix_id=0, device=None, handle: Handle | None = None):
    """The library's SRHT test matrix `matrix_id` under `seed` (rows x cols
    FP64 on the device), as a sketch with test_matrix="srht" draws it."""
    h = handle or default_handle()
    dev = h.device if device is None else torch.device(device)
    out = torch.empty((rows, cols), dtype=torch.float64, device=dev)
    L.check(h._lib.cnmf_srht(h.raw, int(seed) & (2 ** 64 - 1), int(matrix_id), int(rows), int(cols), _ptr(out),
                             max(int(cols), 1)), h.raw)
    return out


def spa(B, r, want_scores=False, noalloc=False, K=None, score=None, handle: Handle | None = None):
    """SPA on the columns of a given k x n device matrix B (FP64 arithmetic).
    noalloc: use cnmf_spa_noalloc (working storage in the library's fixed
    device scratch); K / score may then be passed in preallocated."""
    h = handle or default_handle()
    if B.dtype not in _DT or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major float64/float32 2-D tensor")
    if K is None:
        K = torch.empty(r, dtype=torch.int64, device=B.device)
    if score is None and want_scores:
        score = torch.empty(r, dtype=torch.float64, device=B.device)
    fn = h._lib.cnmf_spa_noalloc if noalloc else h._lib.cnmf_spa
    L.check(fn(h.raw, _ptr(B), _DT[B.dtype], B.shape[0], B.shape[1], B.stride(0), int(r), _ptr(K), _ptr(score)),
            h.raw)
    return K, score


def range_product(A, X, trans=False, handle: Handle | None = None):
    """One streaming pass: A @ X (trans False) or A.T @ X (trans True)."""
    h = handle or default_handle()
    if X.dtype != A.dtype or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous 2-D tensor of A's dtype")
    rows_out = A.shape[1] if trans else A.shape[0]
    Y = torch.empty((rows_out, X.shape[1]), dtype=A.dtype, device=A.device)
    inp = _input(A)
    L.check(h._lib.cnmf_range_product(h.raw, C.byref(inp), int(bool(trans)), _ptr(X), X.shape[1], _ptr(Y)), h.raw)
    return Y


def range_product_lowp(A, X, trans=False, pass_dtype="bf16", handle: Handle | None = None):
    """One pass with BF16 / FP8 operands: A @ X or A.T @ X, FP32 result.

    A: FP32 device matrix; X: FP64, (n or m) x kx.  FP8 operand column scales
    are divided out of the result."""
    h = handle or default_handle()
    if A.dtype != torch.float32:
        raise ValueError("reduced-precision passes need an FP32 A")
    if X.dtype != torch.float64 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous 2-D FP64 tensor")
    rows_out = A.shape[1] if trans else A.shape[0]
    Y = torch.empty((rows_out, X.shape[1]), dtype=torch.float32, device=A.device)
    inp = _input(A)
    L.check(h._lib.cnmf_range_product_lowp(h.raw, C.byref(inp), int(bool(trans)), _PREC[pass_dtype], _ptr(X),
                                           X.shape[1], _ptr(Y)), h.raw)
    return Y


def workspace_bytes(m, n, r, k, q, method="admm", iters=100, pass_dtype="f32", final_dtype=None):
    """Device workspace a factorisation of an m x n input needs (host only)."""
    lib = L.load()
    if final_dtype is None:
        final_dtype = pass_dtype if pass_dtype in ("f64", "f32") else "bf16"
    d = L.cnmf_factorize_desc(_sketch_desc(r, k, q, L.CNMF_BOTH, None, None, pass_dtype, final_dtype),
                              _METHODS[method], int(iters), 1.0, 1.0, 1.0, 0.0, None, None)
    out = C.c_size_t()
    L.check(lib.cnmf_workspace_bytes(int(m), int(n), C.byref(d), C.byref(out)))
    return out.value


# --------------------------------------------------------------------------
# Serving (continuous batching; see cnmf_server_* in include/cnmf.h)
# --------------------------------------------------------------------------

@dataclass
class Ticket:
    id: int
    U: torch.Tensor
    V: torch.Tensor
    rel_residual: torch.Tensor
    keep: tuple  # inputs kept alive until the request is done


class Server:
    """A request server on one GPU.  submit() returns at once; poll() /
    wait() report completion; outputs are device tensors of the ticket."""

    STATES = ("queued", "prologue", "ready", "batch", "epilogue", "done")

    def __init__(self, hbm_budget_bytes: int, max_batch: int = 128, workers: int = 3, device: int = 0,
                 graphs: bool = False, one_step: bool = False):
        self._lib = L.load()
        flags = (L.CNMF_SERVER_GRAPHS if graphs else 0) | (L.CNMF_SERVER_ONE_STEP if one_step else 0)
        cfg = L.cnmf_server_config(int(device), int(max_batch), int(workers), flags, int(hbm_budget_bytes))
        raw = C.c_void_p()
        L.check_server(self._lib.cnmf_server_start(C.byref(cfg), C.byref(raw)))
        self.raw = raw
        self.device = torch.device("cuda", device)

    def submit(self, A, r, k, q, U0, V0, omega_left=None, omega_right=None, method="admm", iters=100, lam=1.0,
               phi=None, xi=1.0, mu_eps=1e-16, pass_dtype=None, final_dtype=None, stream=None, seed=0) -> Ticket:
        pass_dtype, final_dtype = _default_prec(A, pass_dtype, final_dtype)
        m, n = A.shape
        od = _acc_dtype(A, pass_dtype)
        U = torch.empty((m, r), dtype=od, device=A.device)
        V = torch.empty((r, n), dtype=od, device=A.device)
        res = torch.zeros(1, dtype=torch.float64, device=A.device)
        U0 = U0.to(device=A.device, dtype=torch.float64).contiguous()
        V0 = V0.to(device=A.device, dtype=torch.float64).contiguous()
        inp = _input(A)
        d = L.cnmf_factorize_desc(_sketch_desc(r, k, q, L.CNMF_BOTH, omega_left, omega_right, pass_dtype,
                                               final_dtype, seed),
                                  _METHODS[method], int(iters), float(lam), float(lam if phi is None else phi),
                                  float(xi), float(mu_eps), _ptr(U0), _ptr(V0))
        out = L.cnmf_factorize_out(_ptr(U), _ptr(V), _ptr(res), L.cnmf_sketch_out())
        st = stream if stream is not None else torch.cuda.current_stream(A.device)
        t = C.c_uint64()
        L.check_server(self._lib.cnmf_server_submit(self.raw, C.byref(inp), C.byref(d), C.byref(out),
                                                    C.c_void_p(st.cuda_stream), C.byref(t)))
        return Ticket(t.value, U, V, res, (A, U0, V0, omega_left, omega_right))

    def poll(self, ticket: Ticket) -> dict:
        info = L.cnmf_ticket_info()
        L.check_server(self._lib.cnmf_server_poll(self.raw, ticket.id, C.byref(info)))
        return {"state": self.STATES[info.state], "done": bool(info.done), "status": info.status,
                "queue_ms": info.queue_ms, "total_ms": info.total_ms, "message": info.message.decode()}

    def wait(self, ticket: Ticket, timeout_s: float = 120.0, sleep_s: float = 2e-4) -> dict:
        import time
        t0 = time.perf_counter()
        while True:
            info = self.poll(ticket)
            if info["done"]:
                if info["status"] != L.CNMF_OK:
                    raise L.CnmfError(info["status"], info["message"])
                return info
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket.id} not done after {timeout_s} s ({info['state']})")
            time.sleep(sleep_s)

    def release(self, ticket: Ticket):
        L.check_server(self._lib.cnmf_server_release(self.raw, ticket.id))

    def stats(self) -> dict:
        s = L.cnmf_server_stats()
        L.check_server(self._lib.cnmf_server_get_stats(self.raw, C.byref(s)))
        return {f: getattr(s, f) for f, _ in L.cnmf_server_stats._fields_}

    def stop(self):
        if self.raw:
            L.check_server(self._lib.cnmf_server_stop(self.raw))
            self.raw = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


def simulate_admission(arrival_ms, nbytes, service_ms, budget, max_inflight):
    """Host-only replay of the server's admission policy (no GPU)."""
    import numpy as np
    lib = L.load()
    a = np.ascontiguousarray(arrival_ms, dtype=np.float64)
    b = np.ascontiguousarray(nbytes, dtype=np.uint64)
    s = np.ascontiguousarray(service_ms, dtype=np.float64)
    n = len(a)
    adm = np.empty(n, dtype=np.float64)
    done = np.empty(n, dtype=np.float64)
    peak = C.c_uint64()
    dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))
    L.check_server(lib.cnmf_server_simulate(n, dp(a), b.ctypes.data_as(C.POINTER(C.c_uint64)), dp(s), int(budget),
                                            int(max_inflight), dp(adm), dp(done), C.byref(peak)))
    return adm, done, peak.value
