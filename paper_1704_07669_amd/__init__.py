"""MI355X single-pass PCA (Algorithm 4 of Yu et al., IJCAI 2017) behind a C ABI.

Thin ctypes binding of ``include/sketch.h``: the functions below carry the C names and only
marshal arguments; every step of the computation runs in the HIP library ``libsketch.so``.
PyTorch provides device memory (workspace and outputs) and the HIP stream.

The library must be built first (``python -m paper_1704_07669_amd.build``); loading fails loudly
when it is missing -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsketch.so")

# sketch_dtype
F64, F32, BF16, BF16X2, FP8_E4M3 = 0, 1, 2, 3, 4
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "bf16x2": BF16X2, "fp8": FP8_E4M3}
STATUS = {0: "SKETCH_OK", 1: "SKETCH_E_INVAL", 2: "SKETCH_E_STATE", 3: "SKETCH_E_NOMEM",
          4: "SKETCH_E_CAPACITY", 5: "SKETCH_E_NONFINITE", 6: "SKETCH_E_DEVICE"}
EXPORTED = [
    "sketch_workspace_size", "sketch_init", "sketch_reset", "sketch_set_omega",
    "sketch_ingest_block", "sketch_poll", "sketch_finalize", "sketch_finalize_paths",
    "sketch_debug_force_paths",
    "sketch_get_omega", "sketch_checkpoint_size", "sketch_checkpoint", "sketch_restore",
    "sketch_merge", "sketch_pca_static", "sketch_power_restart", "sketch_column_mean",
    "sketch_debug_state", "sketch_philox_words", "sketch_jacobi_schedule",
    "sketch_profile_enable", "sketch_profile_read",
    "sketch_destroy", "sketch_last_error",
    "sketch_server_workspace_size", "sketch_server_stream_bytes", "sketch_server_create",
    "sketch_server_open", "sketch_server_submit", "sketch_server_submit_ex", "sketch_server_clock",
    "sketch_server_step", "sketch_server_poll",
    "sketch_server_finalize", "sketch_server_get_stats", "sketch_server_destroy",
]


class SketchError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class sketch_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m_capacity", ctypes.c_int64), ("max_block_rows", ctypes.c_int64),
        ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("b", ctypes.c_int32),
        ("compute", ctypes.c_int32), ("host_slots", ctypes.c_int32), ("host_src", ctypes.c_int32),
        ("want_u", ctypes.c_int32), ("omega_from_seed", ctypes.c_int32),
        ("centre", ctypes.c_int32), ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64),
    ]


class sketch_server_config(ctypes.Structure):
    _fields_ = [
        ("compute", ctypes.c_int32), ("src", ctypes.c_int32), ("l", ctypes.c_int32),
        ("max_group", ctypes.c_int32), ("max_n", ctypes.c_int64), ("max_m", ctypes.c_int64),
        ("max_block_rows", ctypes.c_int64), ("state_bytes", ctypes.c_int64),
        ("worker", ctypes.c_int32), ("host_slots", ctypes.c_int32),
    ]


class sketch_server_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "active", "queued", "state_used", "state_peak", "groups", "blocks", "max_blocks_in_group",
        "finalized", "queued_peak")]


_lib = None


def load_library(path=None):
    """Load libsketch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    # PyTorch ships its own HIP runtime with the same soname as /opt/rocm's; loading torch first
    # makes this library bind to that one runtime instead of pulling in a second copy.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_1704_07669_amd.build)")
    lib = ctypes.CDLL(path)
    P, I32, I64, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                           ctypes.c_double)
    cfgp = ctypes.POINTER(sketch_config)
    scfgp = ctypes.POINTER(sketch_server_config)
    sig = {
        "sketch_workspace_size": (ctypes.c_size_t, [cfgp]),
        "sketch_init": (I32, [ctypes.POINTER(P), cfgp, P, ctypes.c_size_t, P]),
        "sketch_reset": (I32, [P, U64]),
        "sketch_set_omega": (I32, [P, P, I64]),
        "sketch_ingest_block": (I32, [P, P, I32, I64, I64, I32, ctypes.POINTER(U64)]),
        "sketch_poll": (I32, [P, U64, ctypes.POINTER(I32)]),
        "sketch_finalize": (I32, [P, P, P, I64, P, I64, ctypes.POINTER(I32)]),
        "sketch_finalize_paths": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "sketch_debug_force_paths": (I32, [P, I32, I32]),
        "sketch_get_omega": (I32, [P, P, I64]),
        "sketch_checkpoint_size": (ctypes.c_size_t, [P]),
        "sketch_checkpoint": (I32, [P, P, ctypes.c_size_t]),
        "sketch_restore": (I32, [P, P, ctypes.c_size_t]),
        "sketch_merge": (I32, [P, P, ctypes.c_size_t]),
        "sketch_power_restart": (I32, [P, I32, ctypes.POINTER(I32)]),
        "sketch_column_mean": (I32, [P, P]),
        "sketch_pca_static": (I32, [cfgp, P, I32, I64, I64, P, P, I64, P, I64,
                                    ctypes.POINTER(I32), P]),
        "sketch_debug_state": (I32, [P, P, P, ctypes.POINTER(I64)]),
        "sketch_philox_words": (I32, [U64, U64, I64, P, P]),
        "sketch_jacobi_schedule": (I32, [I32, P, I64, ctypes.POINTER(I32)]),
        "sketch_profile_enable": (I32, [P, I32]),
        "sketch_profile_read": (I32, [P, I32, ctypes.POINTER(I64), ctypes.POINTER(D)]),
        "sketch_destroy": (I32, [P]),
        "sketch_last_error": (ctypes.c_char_p, []),
        "sketch_server_workspace_size": (ctypes.c_size_t, [scfgp]),
        "sketch_server_stream_bytes": (ctypes.c_size_t, [scfgp, cfgp]),
        "sketch_server_create": (I32, [ctypes.POINTER(P), scfgp, P, ctypes.c_size_t, P]),
        "sketch_server_open": (I32, [P, cfgp, ctypes.POINTER(U64), ctypes.POINTER(I32)]),
        "sketch_server_submit": (I32, [P, U64, P, I64, I64, ctypes.POINTER(U64)]),
        "sketch_server_submit_ex": (I32, [P, U64, P, I32, I64, I64, D, ctypes.POINTER(U64)]),
        "sketch_server_clock": (D, []),
        "sketch_server_step": (I32, [P, ctypes.POINTER(I32)]),
        "sketch_server_poll": (I32, [P, ctypes.POINTER(U64), ctypes.POINTER(D), I32,
                                     ctypes.POINTER(I32)]),
        "sketch_server_finalize": (I32, [P, U64, P, P, I64, P, I64, ctypes.POINTER(I32)]),
        "sketch_server_get_stats": (I32, [P, ctypes.POINTER(sketch_server_stats)]),
        "sketch_server_destroy": (I32, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st):
    if st != 0:
        raise SketchError(st, _lib.sketch_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ C-named wrappers
def sketch_workspace_size(cfg):
    lib = load_library()
    n = lib.sketch_workspace_size(ctypes.byref(cfg))
    if n == 0:
        raise SketchError(1, lib.sketch_last_error().decode())
    return int(n)


def sketch_init(cfg, workspace, stream=None):
    lib = load_library()
    h = ctypes.c_void_p()
    _check(lib.sketch_init(ctypes.byref(h), ctypes.byref(cfg), _ptr(workspace),
                           workspace.numel() * workspace.element_size(), _stream_handle(stream)))
    return h


def sketch_reset(h, seed):
    _check(load_library().sketch_reset(h, seed))


def sketch_set_omega(h, omega_dev):
    _check(load_library().sketch_set_omega(h, _ptr(omega_dev), omega_dev.stride(0)))


def sketch_ingest_block(h, rows, src_dtype, src_is_device):
    tk = ctypes.c_uint64()
    _check(load_library().sketch_ingest_block(h, _ptr(rows), src_dtype, rows.shape[0],
                                              rows.stride(0), int(src_is_device),
                                              ctypes.byref(tk)))
    return tk.value


def sketch_poll(h, ticket):
    d = ctypes.c_int32()
    _check(load_library().sketch_poll(h, ticket, ctypes.byref(d)))
    return bool(d.value)


def sketch_finalize(h, S, U, V):
    r = ctypes.c_int32()
    _check(load_library().sketch_finalize(h, _ptr(S), _ptr(U), 0 if U is None else U.stride(0),
                                          _ptr(V), V.stride(0), ctypes.byref(r)))
    return r.value


def sketch_finalize_paths(h):
    """(loop_path, rb_path) of the last finalize: 0 Cholesky QR, 1 the Householder fallback."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().sketch_finalize_paths(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def sketch_debug_force_paths(h, loop_householder, rb_mode):
    _check(load_library().sketch_debug_force_paths(h, int(loop_householder), int(rb_mode)))


def sketch_checkpoint_size(h):
    n = load_library().sketch_checkpoint_size(h)
    if n == 0:
        raise SketchError(-1, _lib.sketch_last_error().decode())
    return n


def sketch_checkpoint(h, buf):
    """Writes the pass state into `buf` (a writable numpy uint8 array)."""
    _check(load_library().sketch_checkpoint(h, buf.ctypes.data, buf.nbytes))


def sketch_restore(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(load_library().sketch_restore(h, buf.ctypes.data, buf.nbytes))


def sketch_merge(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(load_library().sketch_merge(h, buf.ctypes.data, buf.nbytes))


def sketch_pca_static(cfg, A, S, U, V, stream=None):
    """One call of the whole method on a device matrix A (torch CUDA tensor, row-major), with the
    library's fixed device scratch as workspace; returns the rank."""
    import torch
    src = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[A.dtype]
    rank = ctypes.c_int32()
    _check(load_library().sketch_pca_static(
        ctypes.byref(cfg), _ptr(A), src, A.shape[0], A.stride(0), _ptr(S),
        _ptr(U) if U is not None else None, U.stride(0) if U is not None else 0, _ptr(V),
        V.stride(0), ctypes.byref(rank), _stream_handle(stream)))
    return rank.value


def sketch_power_restart(h, route=0):
    used = ctypes.c_int32(-1)
    _check(load_library().sketch_power_restart(h, int(route), ctypes.byref(used)))
    return used.value


def sketch_column_mean(h, out):
    _check(load_library().sketch_column_mean(h, _ptr(out)))


def sketch_get_omega(h, out):
    _check(load_library().sketch_get_omega(h, _ptr(out), out.stride(0)))


def sketch_debug_state(h, G, H):
    rows = ctypes.c_int64()
    _check(load_library().sketch_debug_state(h, _ptr(G), _ptr(H), ctypes.byref(rows)))
    return rows.value


def sketch_philox_words(seed, first, count, out, stream=None):
    _check(load_library().sketch_philox_words(seed, first, count, _ptr(out),
                                              _stream_handle(stream)))


def sketch_jacobi_schedule(n):
    """The pair table of one Jacobi sweep over n columns: a bytes object of rounds x 64 x 2
    (home, visitor; 255 for an idle group) and the number of rounds."""
    cap = 2 * 64 * 128
    buf = (ctypes.c_uint8 * cap)()
    rounds = ctypes.c_int32()
    _check(load_library().sketch_jacobi_schedule(n, buf, cap, ctypes.byref(rounds)))
    return bytes(buf[:rounds.value * 128]), rounds.value


def sketch_profile_enable(h, on=True):
    _check(load_library().sketch_profile_enable(h, int(on)))


def sketch_profile_read(h, kind):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(load_library().sketch_profile_read(h, kind, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def sketch_destroy(h):
    _check(load_library().sketch_destroy(h))


def sketch_last_error():
    return load_library().sketch_last_error().decode()


# ------------------------------------------------------------------ convenience object
class Sketch:
    """One single-pass PCA stream on the current CUDA (HIP) device.

    ``compute`` is one of 'f64', 'f32', 'bf16', 'bf16x2', 'fp8'.  Omega is drawn on the device
    from ``seed`` unless ``omega`` (an n x l float64 array/tensor) is given.
    """

    def __init__(self, n, m_capacity, max_block_rows, k, l, b=10, compute="f32", host_slots=0,
                 host_src="f32", want_u=False, seed=0, omega=None, stream=None, centre=False):
        import torch
        load_library()
        self.cfg = sketch_config(
            n=n, m_capacity=m_capacity, max_block_rows=max_block_rows, k=k, l=l, b=b,
            compute=DTYPES[compute], host_slots=host_slots, host_src=DTYPES[host_src],
            want_u=int(bool(want_u)), omega_from_seed=int(omega is None),
            centre=int(bool(centre)), seed=seed)
        self.n, self.k, self.l = n, k, l
        self.stream = stream
        ws = sketch_workspace_size(self.cfg)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device="cuda")
        self.h = sketch_init(self.cfg, self.workspace, stream)
        self.closed = False
        if omega is not None:
            om = torch.as_tensor(np.asarray(omega, dtype=np.float64)).to("cuda")
            sketch_set_omega(self.h, om.contiguous())
            torch.cuda.synchronize()

    _TORCH2DT = None

    @staticmethod
    def _src_code(t):
        import torch
        return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]

    def ingest(self, rows):
        """Ingest a 2-D block: a CUDA tensor, or a pinned CPU tensor (host_slots > 0)."""
        if rows.dim() != 2 or rows.shape[1] != self.n or rows.stride(1) != 1:
            raise ValueError("rows must be a row-major nrows x n tensor")
        return sketch_ingest_block(self.h, rows, self._src_code(rows), rows.is_cuda)

    def poll(self, ticket):
        return sketch_poll(self.h, ticket)

    def finalize(self, want_u=None):
        import torch
        want_u = bool(self.cfg.want_u) if want_u is None else want_u
        S = torch.empty(self.k, dtype=torch.float64, device="cuda")
        V = torch.empty(self.n, self.k, dtype=torch.float64, device="cuda")
        U = None
        if want_u:
            U = torch.empty(self.rows_capacity_used(), self.k, dtype=torch.float64, device="cuda")
        rank = sketch_finalize(self.h, S, U, V)
        return S, V, U, rank

    def finalize_paths(self):
        return sketch_finalize_paths(self.h)

    def force_paths(self, loop_householder, rb_mode):
        sketch_debug_force_paths(self.h, loop_householder, rb_mode)

    def rows_capacity_used(self):
        import torch
        rows = ctypes.c_int64()
        _check(load_library().sketch_debug_state(self.h, None, None, ctypes.byref(rows)))
        return rows.value

    def omega(self):
        import torch
        out = torch.empty(self.n, self.l, dtype=torch.float64, device="cuda")
        sketch_get_omega(self.h, out)
        return out

    def state(self):
        import torch
        rows = self.rows_capacity_used()
        G = torch.empty(rows, self.l, dtype=torch.float64, device="cuda")
        H = torch.empty(self.n, self.l, dtype=torch.float64, device="cuda")
        sketch_debug_state(self.h, G, H)
        return G, H

    def reset(self, seed=None):
        sketch_reset(self.h, self.cfg.seed if seed is None else seed)

    def checkpoint(self):
        """The pass state as a host byte image (numpy uint8)."""
        buf = np.empty(sketch_checkpoint_size(self.h), dtype=np.uint8)
        sketch_checkpoint(self.h, buf)
        return buf

    def restore(self, buf):
        sketch_restore(self.h, buf)

    def merge(self, buf):
        sketch_merge(self.h, buf)

    def column_mean(self):
        """Column means of the rows ingested (handles created with centre=True)."""
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        sketch_column_mean(self.h, out)
        return out

    def power_restart(self, route=0):
        """Power scheme P = 1: Omega <- sqrt(n) orth(H) and a new pass; re-ingest A, then
        finalize.  Returns the orthonormalisation route used."""
        return sketch_power_restart(self.h, route)

    def profile(self, on=True):
        sketch_profile_enable(self.h, on)

    def profile_read(self, kind):
        return sketch_profile_read(self.h, kind)

    def close(self):
        if not self.closed:
            sketch_destroy(self.h)
            self.closed = True

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
def sketch_server_workspace_size(scfg):
    lib = load_library()
    n = lib.sketch_server_workspace_size(ctypes.byref(scfg))
    if n == 0:
        raise SketchError(1, lib.sketch_last_error().decode())
    return int(n)


def sketch_server_stream_bytes(scfg, cfg):
    lib = load_library()
    n = lib.sketch_server_stream_bytes(ctypes.byref(scfg), ctypes.byref(cfg))
    if n == 0:
        raise SketchError(1, lib.sketch_last_error().decode())
    return int(n)


def sketch_server_create(scfg, workspace, stream=None):
    lib = load_library()
    h = ctypes.c_void_p()
    _check(lib.sketch_server_create(ctypes.byref(h), ctypes.byref(scfg), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(),
                                    _stream_handle(stream)))
    return h


def sketch_server_open(srv, cfg):
    sid, adm = ctypes.c_uint64(), ctypes.c_int32()
    _check(load_library().sketch_server_open(srv, ctypes.byref(cfg), ctypes.byref(sid),
                                             ctypes.byref(adm)))
    return sid.value, bool(adm.value)


def sketch_server_submit(srv, sid, rows):
    tk = ctypes.c_uint64()
    _check(load_library().sketch_server_submit(srv, sid, _ptr(rows), rows.shape[0],
                                               rows.stride(0), ctypes.byref(tk)))
    return tk.value


def sketch_server_submit_ex(srv, sid, rows, arrival_s=-1.0):
    """rows: a CUDA tensor or a pinned CPU tensor (row-major)."""
    tk = ctypes.c_uint64()
    _check(load_library().sketch_server_submit_ex(srv, sid, _ptr(rows), int(rows.is_cuda),
                                                  rows.shape[0], rows.stride(0), float(arrival_s),
                                                  ctypes.byref(tk)))
    return tk.value


def sketch_server_clock():
    return load_library().sketch_server_clock()


def sketch_server_step(srv):
    n = ctypes.c_int32()
    _check(load_library().sketch_server_step(srv, ctypes.byref(n)))
    return n.value


def sketch_server_poll(srv, cap=4096):
    tks = (ctypes.c_uint64 * cap)()
    lat = (ctypes.c_double * cap)()
    n = ctypes.c_int32()
    _check(load_library().sketch_server_poll(srv, tks, lat, cap, ctypes.byref(n)))
    return [(tks[i], lat[i]) for i in range(n.value)]


def sketch_server_finalize(srv, sid, S, U, V):
    r = ctypes.c_int32()
    _check(load_library().sketch_server_finalize(srv, sid, _ptr(S), _ptr(U),
                                                 0 if U is None else U.stride(0), _ptr(V),
                                                 V.stride(0), ctypes.byref(r)))
    return r.value


def sketch_server_get_stats(srv):
    st = sketch_server_stats()
    _check(load_library().sketch_server_get_stats(srv, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in sketch_server_stats._fields_}


def sketch_server_destroy(srv):
    _check(load_library().sketch_server_destroy(srv))


class Server:
    """Continuous-batching server of many single-pass PCA streams on the current device.

    ``state_bytes`` is the device-memory budget for resident stream states (admission control);
    the workspace (group scratch, finalize scratch and that budget) is one torch allocation."""

    def __init__(self, l, max_n, max_m, max_block_rows, state_bytes, compute="f32", src="f32",
                 max_group=16, worker=True, stream=None, host_slots=0):
        import torch
        load_library()
        self.cfg = sketch_server_config(
            compute=DTYPES[compute], src=DTYPES[src], l=l, max_group=max_group, max_n=max_n,
            max_m=max_m, max_block_rows=max_block_rows, state_bytes=state_bytes,
            worker=int(bool(worker)), host_slots=host_slots)
        self.l, self.compute, self.src = l, compute, src
        ws = sketch_server_workspace_size(self.cfg)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device="cuda")
        self.h = sketch_server_create(self.cfg, self.workspace, stream)
        self.meta = {}
        self._held = {}   # ticket -> (stream id, rows) until retired
        self.closed = False

    def stream_config(self, n, m, k, b, seed, max_block_rows=None, want_u=False):
        return sketch_config(n=n, m_capacity=m, max_block_rows=max_block_rows or
                             self.cfg.max_block_rows, k=k, l=self.l, b=b,
                             compute=self.cfg.compute, host_slots=0, host_src=self.cfg.src,
                             want_u=int(bool(want_u)), omega_from_seed=1, seed=seed)

    def stream_bytes(self, n, m, k, b, seed=0):
        return sketch_server_stream_bytes(self.cfg, self.stream_config(n, m, k, b, seed))

    def open(self, n, m, k, b, seed, want_u=False, max_block_rows=None):
        cfg = self.stream_config(n, m, k, b, seed, max_block_rows, want_u)
        sid, admitted = sketch_server_open(self.h, cfg)
        self.meta[sid] = cfg
        return sid, admitted

    def submit(self, sid, rows, arrival_s=-1.0):
        """rows: a row-major 2-D CUDA tensor, or a pinned CPU tensor when host_slots > 0, of the
        server's source type.  The server keeps a reference to it until its ticket is polled or
        its stream finalized (the library reads the rows asynchronously).  arrival_s, on the
        clock of ``clock()``, is when the block arrived; by default the submit time."""
        import torch
        if rows.dim() != 2 or rows.stride(1) != 1:
            raise ValueError("rows must be a row-major 2-D tensor")
        want = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[self.src]
        if rows.dtype != want:
            raise ValueError(f"rows must be {want}, got {rows.dtype}")
        if rows.is_cuda and arrival_s < 0:
            tk = sketch_server_submit(self.h, sid, rows)
        else:
            tk = sketch_server_submit_ex(self.h, sid, rows, arrival_s)
        self._held[tk] = (sid, rows)
        return tk

    @staticmethod
    def clock():
        """The host clock (seconds) that arrival times and latencies are measured on."""
        return sketch_server_clock()

    def step(self):
        return sketch_server_step(self.h)

    def poll(self, cap=4096):
        """(ticket, latency_s) of retired blocks: arrival to the GPU completion of the grouped
        launch that consumed the block."""
        out = sketch_server_poll(self.h, cap)
        for tk, _ in out:
            self._held.pop(tk, None)
        return out

    def finalize(self, sid, want_u=None):
        import torch
        cfg = self.meta[sid]
        want_u = bool(cfg.want_u) if want_u is None else want_u
        S = torch.empty(cfg.k, dtype=torch.float64, device="cuda")
        V = torch.empty(cfg.n, cfg.k, dtype=torch.float64, device="cuda")
        U = torch.empty(cfg.m_capacity, cfg.k, dtype=torch.float64, device="cuda") if want_u else None
        rank = sketch_server_finalize(self.h, sid, S, U, V)
        del self.meta[sid]
        for tk in [t for t, (s, _) in self._held.items() if s == sid]:
            del self._held[tk]
        return S, V, U, rank

    def stats(self):
        return sketch_server_get_stats(self.h)

    def close(self):
        if not self.closed:
            sketch_server_destroy(self.h)
            self.closed = True

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
