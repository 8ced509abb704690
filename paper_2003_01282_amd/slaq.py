"""Thin Python binding of libslaq.so (argument marshalling only).

Every computation runs in the HIP library; torch supplies device memory and
the current stream.  Names follow the C ABI in include/slaq.h.  The library
must be built (paper_2003_01282_amd.build); there is no fallback path.
"""
import ctypes
from pathlib import Path

import torch

LIB_PATH = Path(__file__).resolve().parent / "libslaq.so"

SLAQ_LAP_NORMALIZED = 0
SLAQ_LAP_COMBINATORIAL = 1
SLAQ_SIG_HEAT = 0
SLAQ_SIG_WAVE = 1
SLAQ_FLAG_CHECK = 1
SLAQ_FLAG_RELABEL = 2
SLAQ_FLAG_NO_RELABEL = 4
SLAQ_RELABEL_MIN_NNZ = 1 << 22
SLAQ_PREC_FP32 = 0
SLAQ_PREC_FP64 = 1
SLAQ_CV_NONE = 0
SLAQ_CV_TAYLOR = 1
SLAQ_CV_FITTED = 2
SLAQ_MAX_PROBES = 4096
SLAQ_MAX_STEPS = 64
SLAQ_ERR_INVALID_ARG = 1
SLAQ_ERR_NUMERIC = 3
SLAQ_ERR_WORKSPACE = 4
SLAQ_STATUS_NONFINITE = 1
SLAQ_STATUS_NO_CONVERGENCE = 2
SLAQ_STATUS_GRID = 4

STATUS = {
    0: "SLAQ_OK", 1: "SLAQ_ERR_INVALID_ARG", 2: "SLAQ_ERR_NOT_SYMMETRIC", 3: "SLAQ_ERR_NUMERIC",
    4: "SLAQ_ERR_WORKSPACE", 5: "SLAQ_ERR_HIP", 6: "SLAQ_ERR_UNSUPPORTED", 7: "SLAQ_ERR_BAD_CSR",
}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_sz = ctypes.c_size_t

# name -> argument types (all return slaq_status except slaq_last_error)
SIGNATURES = {
    "slaq_graph_scratch_bytes": [_i64, _i64, ctypes.POINTER(_sz)],
    "slaq_build_graph": [_i64, _i64, _vp, _vp, _vp, _int, ctypes.c_uint, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp)],
    "slaq_graph_info": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)],
    "slaq_graph_destroy": [_vp],
    "slaq_graph_internal": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_i64), _vp, _vp, _vp],
    "slaq_graph_traces": [_vp, _vp, _vp],
    "slaq_signature_cv": [_vp, _vp, _int, _int, _i64, _vp, _vp, _int, _int, _int, _vp, _vp],
    "slaq_vnge_cv": [_vp, _vp, _vp, _int, _int, _vp, _int, _vp, _vp],
    "slaq_graph_set_schedule": [_vp, _int, _int, _vp],
    "slaq_graph_set_tile": [_vp, _int],
    "slaq_graph_set_cache_rows": [_vp, _i64],
    "slaq_graph_set_fused": [_vp, _int],
    "slaq_graph_set_sign_step": [_vp, _int],
    "slaq_graph_autotune": [_vp, _int, _int, ctypes.c_uint64, _vp, _vp, _vp, _vp, _sz, _int, ctypes.c_char_p,
                            ctypes.POINTER(_int), _vp],
    "slaq_graph_autotune_workspace": [_vp, _int, _int, ctypes.POINTER(_sz)],
    "slaq_graph_settings": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_i64),
                            ctypes.POINTER(_int)],
    "slaq_graph_cache_rows": [_vp, ctypes.POINTER(_i64)],
    "slaq_graph_set_precision": [_vp, _int],
    "slaq_graph_precision": [_vp, ctypes.POINTER(_int)],
    "slaq_graph_schedule": [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_i64),
                            ctypes.POINTER(_i64)],
    "slaq_lanczos_workspace": [_vp, _int, _int, ctypes.POINTER(_sz)],
    "slaq_lanczos": [_vp, _int, _int, ctypes.c_uint64, _vp, _vp, _vp, _vp, _sz, _vp],
    "slaq_lanczos_noalloc": [_vp, _int, _int, ctypes.c_uint64, _vp, _vp, _vp, _vp],
    "slaq_ritz": [_vp, _vp, _vp, _int, _int, _vp, _vp, _vp],
    "slaq_signature": [_vp, _vp, _int, _int, _i64, _vp, _int, _int, _vp, _vp],
    "slaq_vnge": [_vp, _vp, _vp, _int, _int, _vp, _vp],
    "slaq_batch_plan": [_i64, _vp, _vp, _vp, _vp, _vp, _int, _int, _int, _vp, _int, ctypes.POINTER(_vp)],
    "slaq_batch_plan_grown": [_i64, _vp, _vp, _vp, _vp, _vp, _int, _int, _int, ctypes.c_double, _vp, _int,
                              ctypes.POINTER(_vp)],
    "slaq_batch_autotune_edges": [_i64, _vp, _vp, _vp, _vp, _vp, _int, _int, _int, _vp, _int,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float),
                                  ctypes.POINTER(_vp), _vp],
    "slaq_batch_buckets": [_vp, ctypes.POINTER(_int), _vp, _vp, _vp, _vp],
    "slaq_batch_run": [_vp, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint, _vp],
    "slaq_batch_set_seeds": [_vp, _vp],
    "slaq_batch_set_sign_step": [_vp, _int],
    "slaq_batch_workspace": [_vp, ctypes.POINTER(_sz)],
    "slaq_batch_set_workspace": [_vp, _vp, _sz],
    "slaq_batch_autotune": [_vp, _vp, _vp, _vp, _int, _vp, _vp, _vp],
    "slaq_batch_destroy": [_vp],
    "slaq_closure_create": [_int, _int, _int, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)],
    "slaq_closure_destroy": [_vp],
    "slaq_closure_info": [_vp, ctypes.POINTER(_i64), _vp, _vp],
    "slaq_closure_workspace": [_vp, _i64, ctypes.POINTER(_sz)],
    "slaq_closure_get": [_vp, _int, _vp, _vp],
    "slaq_closure_set": [_vp, _vp, _int, _vp],
    "slaq_closure_get_step": [_vp, _vp],
    "slaq_closure_set_optimizer": [_vp, _vp, _vp, _int, _vp],
    "slaq_closure_forward": [_vp, _vp, _i64, _vp, _vp, _sz, _vp],
    "slaq_closure_train_step": [_vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp, _sz, _vp],
    "slaq_closure_rules": [_vp, _vp, _vp, _i64, _int, _int, _vp, _vp, _vp, _vp, _vp],
    "slaq_closure_features": [_vp, _vp, _i64, _int, _vp, _vp],
    "slaq_closure_gauss_values": [_vp, _vp, _i64, _int, _int, _vp, _int, _vp, _vp],
    "slaq_closure_targets": [_vp, _vp, _i64, _vp, _vp],
    "slaq_closure_apply": [_vp, _vp, _vp, _int, _int, _int, _vp, ctypes.c_double, _vp, _vp, _vp],
    "slaq_lsd": [_vp, _vp, _vp, _int, _int, _i64, _vp, _int, _int, _vp, _vp],
    "slaq_vnge_slq": [_vp, _vp, _vp, _int, _int, _i64, ctypes.c_double, _vp, _vp],
    "slaq_device_status": [ctypes.POINTER(ctypes.c_uint), _int, _vp],
    "slaq_hutchinson_mean": [_vp, _int, _int, _int, _vp, _vp, _vp],
    "slaq_profile_enable": [_int],
    "slaq_profile_reset": [],
    "slaq_profile_read": [ctypes.c_char_p, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)],
}

_LIB = None


class SlaqError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def lib():
    """Loads libslaq.so once; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2003_01282_amd.build`")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.slaq_last_error.argtypes = []
        L.slaq_last_error.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def _check(status):
    if status != 0:
        raise SlaqError(status, lib().slaq_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _empty_aligned(nbytes, device):
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Graph:
    """Handle returned by build_graph; keeps its device buffers alive."""

    def __init__(self, handle, n, nnz, laplacian, keep):
        self.handle = handle
        self.n = n
        self.nnz = nnz
        self.laplacian = laplacian
        self._keep = keep

    @property
    def dinv(self):
        return self._keep["dinv"]

    def info(self):
        n, nnz, iso = _i64(), _i64(), _i64()
        tr, mx = ctypes.c_double(), ctypes.c_double()
        _check(lib().slaq_graph_info(self.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(tr),
                                     ctypes.byref(iso), ctypes.byref(mx)))
        return {"n": n.value, "nnz": nnz.value, "trace": tr.value, "n_isolated": iso.value,
                "max_degree": mx.value}

    def set_schedule(self, heavy_min, piece, stream=None):
        _check(lib().slaq_graph_set_schedule(self.handle, heavy_min, piece, _stream(stream)))

    def set_tile(self, tile_quads):
        _check(lib().slaq_graph_set_tile(self.handle, tile_quads))

    def set_cache_rows(self, rows):
        _check(lib().slaq_graph_set_cache_rows(self.handle, int(rows)))

    def cache_rows(self):
        r = _i64()
        _check(lib().slaq_graph_cache_rows(self.handle, ctypes.byref(r)))
        return r.value

    def set_fused(self, blocks):
        """slaq_graph_set_fused: -1 automatic, 0 never, 1..256 workgroups."""
        _check(lib().slaq_graph_set_fused(self.handle, int(blocks)))

    def set_sign_step(self, on):
        """slaq_graph_set_sign_step: first step's gathers from sign records
        (True, the default) or from the vector rows (False); same results."""
        _check(lib().slaq_graph_set_sign_step(self.handle, 1 if on else 0))

    def settings(self):
        """slaq_graph_settings -> {heavy_min, piece, cache_rows, fused}."""
        hm, pc, cr, fu = _int(), _int(), _i64(), _int()
        _check(lib().slaq_graph_settings(self.handle, ctypes.byref(hm), ctypes.byref(pc), ctypes.byref(cr),
                                         ctypes.byref(fu)))
        return {"heavy_min": hm.value, "piece": pc.value, "cache_rows": cr.value, "fused": fu.value}

    def autotune(self, nv, m, seed=0, reps=2, cache_path=None, stream=None):
        """slaq_graph_autotune with buffers of its own; returns (settings,
        from_cache)."""
        dev = self._keep["row_ptr"].device
        b = _sz()
        _check(lib().slaq_graph_autotune_workspace(self.handle, nv, m, ctypes.byref(b)))
        ws = _empty_aligned(b.value, dev)
        a = torch.empty((nv, m), dtype=torch.float64, device=dev)
        be = torch.empty_like(a)
        st = torch.empty(nv, dtype=torch.int32, device=dev)
        hit = _int()
        path = None if cache_path is None else str(cache_path).encode()
        _check(lib().slaq_graph_autotune(self.handle, nv, m, ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(a),
                                         _ptr(be), _ptr(st), _ptr(ws), ws.numel(), reps, path, ctypes.byref(hit),
                                         _stream(stream)))
        return self.settings(), bool(hit.value)

    def set_precision(self, precision):
        _check(lib().slaq_graph_set_precision(self.handle, precision))

    def precision(self):
        p = _int()
        _check(lib().slaq_graph_precision(self.handle, ctypes.byref(p)))
        return p.value

    def schedule(self):
        hm, pc, nh, npc = _int(), _int(), _i64(), _i64()
        _check(lib().slaq_graph_schedule(self.handle, ctypes.byref(hm), ctypes.byref(pc), ctypes.byref(nh),
                                         ctypes.byref(npc)))
        return {"heavy_min": hm.value, "piece": pc.value, "n_heavy": nh.value, "n_pieces": npc.value}

    def relabeled(self):
        """Whether the build relabelled the nodes (slaq_graph_internal with
        only the flag asked for: nothing is copied)."""
        rel = _int()
        _check(lib().slaq_graph_internal(self.handle, ctypes.byref(rel), None, None, None, None))
        return bool(rel.value)

    def internal(self):
        """slaq_graph_internal -> dict(relabeled, n_rows, perm, row_ptr, col_idx)
        (device tensors: label -> caller id, and the internal CSR)."""
        dev = self._keep["row_ptr"].device
        rel, nr = _int(), _i64()
        perm = torch.empty(self.n, dtype=torch.int32, device=dev)
        rp = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        _check(lib().slaq_graph_internal(self.handle, ctypes.byref(rel), ctypes.byref(nr), _ptr(perm), _ptr(rp),
                                         _ptr(ci)))
        return {"relabeled": bool(rel.value), "n_rows": nr.value, "perm": perm, "row_ptr": rp,
                "col_idx": ci[:self.nnz]}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.slaq_graph_destroy(h)
            self.handle = None


def build_graph(row_ptr, col_idx, weights=None, laplacian=SLAQ_LAP_NORMALIZED, check=False, stream=None,
                dinv=None, scratch=None, relabel=None):
    """slaq_build_graph on device CSR tensors (int64 row_ptr, int32 col_idx,
    optional float32 weights).  dinv / scratch may be passed preallocated.
    relabel: None = the library's size rule, True / False = forced."""
    _dev(row_ptr, torch.int64, "row_ptr")
    _dev(col_idx, torch.int32, "col_idx")
    if weights is not None:
        _dev(weights, torch.float32, "weights")
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    dev = row_ptr.device
    nbytes = _sz()
    _check(lib().slaq_graph_scratch_bytes(n, nnz, ctypes.byref(nbytes)))
    if dinv is None:
        dinv = torch.empty(n, dtype=torch.float32, device=dev)
    if scratch is None:
        scratch = _empty_aligned(nbytes.value, dev)
    h = _vp()
    flags = SLAQ_FLAG_CHECK if check else 0
    if relabel is not None:
        flags |= SLAQ_FLAG_RELABEL if relabel else SLAQ_FLAG_NO_RELABEL
    _check(lib().slaq_build_graph(n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(weights), laplacian,
                                  flags, _ptr(dinv), _ptr(scratch), scratch.numel(),
                                  _stream(stream), ctypes.byref(h)))
    keep = {"row_ptr": row_ptr, "col_idx": col_idx, "weights": weights, "dinv": dinv, "scratch": scratch}
    return Graph(h, n, nnz, laplacian, keep)


def lanczos_workspace(g, nv, m):
    b = _sz()
    _check(lib().slaq_lanczos_workspace(g.handle, nv, m, ctypes.byref(b)))
    return b.value


def lanczos(g, nv, m, seed, workspace=None, out=None, stream=None):
    """slaq_lanczos -> (alpha[nv, m] f64, beta[nv, m] f64, steps[nv] i32)."""
    dev = g._keep["row_ptr"].device
    need = lanczos_workspace(g, nv, m)
    if workspace is None:
        workspace = _empty_aligned(need, dev)
    if out is None:
        out = (torch.empty((nv, m), dtype=torch.float64, device=dev),
               torch.empty((nv, m), dtype=torch.float64, device=dev),
               torch.empty(nv, dtype=torch.int32, device=dev))
    alpha, beta, steps = out
    _check(lib().slaq_lanczos(g.handle, nv, m, ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(alpha), _ptr(beta),
                              _ptr(steps), _ptr(workspace), workspace.numel(), _stream(stream)))
    return alpha, beta, steps


NOALLOC_WORKSPACE_BYTES = 64 << 20
# schedule tuning cache shipped with the package (slaq_graph_autotune's JSON)
TUNING_CACHE = Path(__file__).resolve().parent / "tuning" / "schedules.json"


def lanczos_noalloc(g, nv, m, seed, out=None, stream=None):
    """slaq_lanczos_noalloc: slaq_lanczos on the library's own workspace (no
    device allocation by the library) -> (alpha, beta, steps)."""
    dev = g._keep["row_ptr"].device
    if out is None:
        out = (torch.empty((nv, m), dtype=torch.float64, device=dev),
               torch.empty((nv, m), dtype=torch.float64, device=dev),
               torch.empty(nv, dtype=torch.int32, device=dev))
    alpha, beta, steps = out
    _check(lib().slaq_lanczos_noalloc(g.handle, nv, m, ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(alpha),
                                      _ptr(beta), _ptr(steps), _stream(stream)))
    return alpha, beta, steps


def ritz(alpha, beta, steps, out=None, stream=None):
    """slaq_ritz -> (theta[nv, m], tau2[nv, m])."""
    nv, m = alpha.shape
    _dev(alpha, torch.float64, "alpha")
    _dev(beta, torch.float64, "beta")
    _dev(steps, torch.int32, "steps")
    if out is None:
        out = (torch.empty_like(alpha), torch.empty_like(alpha))
    theta, tau2 = out
    _check(lib().slaq_ritz(_ptr(alpha), _ptr(beta), _ptr(steps), nv, m, _ptr(theta), _ptr(tau2),
                           _stream(stream)))
    return theta, tau2


def signature(theta, tau2, n, t, kind=SLAQ_SIG_HEAT, out=None, stream=None):
    """slaq_signature -> double[nt] (heat or wave trace at the times t)."""
    nv, m = theta.shape
    _dev(t, torch.float64, "t")
    if out is None:
        out = torch.empty(t.numel(), dtype=torch.float64, device=theta.device)
    _check(lib().slaq_signature(_ptr(theta), _ptr(tau2), nv, m, n, _ptr(t), t.numel(), kind, _ptr(out),
                                _stream(stream)))
    return out


def vnge(g, theta, tau2, out=None, stream=None):
    """slaq_vnge -> double[1]."""
    nv, m = theta.shape
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=theta.device)
    _check(lib().slaq_vnge(g.handle, _ptr(theta), _ptr(tau2), nv, m, _ptr(out), _stream(stream)))
    return out


def lsd(alpha, beta, steps, n, t, kind=SLAQ_SIG_HEAT, out=None, stream=None):
    """slaq_lsd (Algorithm 1's SLaQ_LSD from the Lanczos coefficients, the
    eigensolve inside) -> double[nt]."""
    nv, m = alpha.shape
    _dev(alpha, torch.float64, "alpha")
    _dev(beta, torch.float64, "beta")
    _dev(steps, torch.int32, "steps")
    _dev(t, torch.float64, "t")
    if out is None:
        out = torch.empty(t.numel(), dtype=torch.float64, device=alpha.device)
    _check(lib().slaq_lsd(_ptr(alpha), _ptr(beta), _ptr(steps), nv, m, n, _ptr(t), t.numel(), kind, _ptr(out),
                          _stream(stream)))
    return out


def vnge_slq(alpha, beta, steps, n, trace, out=None, stream=None):
    """slaq_vnge_slq (Algorithm 1's SLaQ_VNGE from the Lanczos coefficients
    and tr L) -> double[1]."""
    nv, m = alpha.shape
    _dev(alpha, torch.float64, "alpha")
    _dev(beta, torch.float64, "beta")
    _dev(steps, torch.int32, "steps")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=alpha.device)
    _check(lib().slaq_vnge_slq(_ptr(alpha), _ptr(beta), _ptr(steps), nv, m, n, float(trace), _ptr(out),
                               _stream(stream)))
    return out


def device_status(clear=True, stream=None):
    """slaq_device_status: waits for the stream and returns the current
    device's SLAQ_STATUS_* bits (0 = nothing found), clearing them if asked."""
    bits = ctypes.c_uint()
    st = lib().slaq_device_status(ctypes.byref(bits), 1 if clear else 0, _stream(stream))
    if st not in (0, SLAQ_ERR_NUMERIC):
        _check(st)
    return bits.value


def graph_traces(g, out=None, stream=None):
    """slaq_graph_traces -> double[2] (tr L, tr L^2)."""
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=g._keep["row_ptr"].device)
    _check(lib().slaq_graph_traces(g.handle, _ptr(out), _stream(stream)))
    return out


def signature_cv(theta, tau2, n, traces, t, kind=SLAQ_SIG_HEAT, mode=SLAQ_CV_FITTED, out=None, stream=None):
    """slaq_signature_cv -> double[nt] (variance-reduced heat or wave trace)."""
    nv, m = theta.shape
    _dev(t, torch.float64, "t")
    if out is None:
        out = torch.empty(t.numel(), dtype=torch.float64, device=theta.device)
    _check(lib().slaq_signature_cv(_ptr(theta), _ptr(tau2), nv, m, n, _ptr(traces), _ptr(t), t.numel(), kind, mode,
                                   _ptr(out), _stream(stream)))
    return out


def vnge_cv(g, theta, tau2, traces, mode=SLAQ_CV_FITTED, out=None, stream=None):
    """slaq_vnge_cv -> double[1]."""
    nv, m = theta.shape
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=theta.device)
    _check(lib().slaq_vnge_cv(g.handle, _ptr(theta), _ptr(tau2), nv, m, _ptr(traces), mode, _ptr(out),
                              _stream(stream)))
    return out


SLAQ_BATCH_GRAPH = 1


class Batch:
    """Plan of a batch of graphs (slaq_batch_plan); keeps the device CSR
    alive and owns the library plan."""

    def __init__(self, handle, n_graphs, nv, m, nt, keep):
        self.handle = handle
        self.G = n_graphs
        self.nv, self.m, self.nt = nv, m, nt
        self._keep = keep

    def workspace_bytes(self):
        """slaq_batch_workspace: bytes the global bucket needs (0 if none)."""
        n = _sz()
        _check(lib().slaq_batch_workspace(self.handle, ctypes.byref(n)))
        return n.value

    def set_workspace(self, ws):
        """slaq_batch_set_workspace with a caller-owned device buffer (a
        256-byte aligned tensor, e.g. from _empty_aligned) or None."""
        self._keep["workspace"] = ws
        nbytes = 0 if ws is None else ws.numel() * ws.element_size()
        _check(lib().slaq_batch_set_workspace(self.handle, _ptr(ws), nbytes))

    def set_seeds(self, seeds):
        """slaq_batch_set_seeds: per-graph probe seeds (uint64-valued int64
        device tensor [G]) or None for seed + g."""
        if seeds is not None:
            _dev(seeds, torch.int64, "seeds")
            if seeds.numel() != self.G:
                raise SlaqError(SLAQ_ERR_INVALID_ARG, f"seeds needs {self.G} entries")
        self._keep["seeds"] = seeds
        _check(lib().slaq_batch_set_seeds(self.handle, _ptr(seeds)))

    def set_sign_step(self, on):
        """slaq_batch_set_sign_step: global buckets' first step from sign
        records (True, the default) or from the rows (False); same results."""
        _check(lib().slaq_batch_set_sign_step(self.handle, 1 if on else 0))

    def buckets(self):
        nb = _int()
        _check(lib().slaq_batch_buckets(self.handle, ctypes.byref(nb), None, None, None, None))
        k = nb.value
        n_hi, blocks, graphs, lds = [(ctypes.c_int * k)() for _ in range(4)]
        _check(lib().slaq_batch_buckets(self.handle, ctypes.byref(nb), n_hi, blocks, graphs, lds))
        return [{"n_hi": n_hi[i], "block": blocks[i], "graphs": graphs[i], "in_lds": bool(lds[i])}
                for i in range(k)]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.slaq_batch_destroy(h)
            self.handle = None


def _plan(row_ptr, col_idx, goff, node_off, nnz_off, nv, m, nt, bucket_blocks, growth):
    G = len(node_off) - 1
    bb = None
    nbb = 0
    if bucket_blocks is not None:
        bb = (ctypes.c_int * len(bucket_blocks))(*bucket_blocks)
        nbb = len(bucket_blocks)
    h = _vp()
    _check(lib().slaq_batch_plan_grown(G, node_off.ctypes.data_as(_vp), nnz_off.ctypes.data_as(_vp), _ptr(goff),
                                       _ptr(row_ptr), _ptr(col_idx), nv, m, nt, float(growth), bb, nbb,
                                       ctypes.byref(h)))
    return Batch(h, G, nv, m, nt, {"rp": row_ptr, "ci": col_idx, "goff": goff})


def batch_plan(union_csr, node_off, nv, m, nt, bucket_blocks=None, device="cuda", growth=2.0):
    """slaq_batch_plan (slaq_batch_plan_grown for growth != 2) for a
    block-diagonal union (inputs.disjoint_union)."""
    import numpy as np
    node_off = np.ascontiguousarray(node_off, dtype=np.int64)
    nnz_off = np.ascontiguousarray(union_csr.row_ptr[node_off], dtype=np.int64)
    rp = torch.from_numpy(union_csr.row_ptr).to(device)
    ci = torch.from_numpy(union_csr.col_idx).to(device)
    goff = torch.from_numpy(node_off).to(device)
    return _plan(rp, ci, goff, node_off, nnz_off, nv, m, nt, bucket_blocks, growth)


def _device_union_offsets(row_ptr, col_idx, node_off):
    import numpy as np
    _dev(row_ptr, torch.int64, "row_ptr")
    _dev(col_idx, torch.int32, "col_idx")
    node_off = np.ascontiguousarray(node_off, dtype=np.int64)
    goff = torch.from_numpy(node_off).to(row_ptr.device)
    nnz_off = np.ascontiguousarray(row_ptr[goff].cpu().numpy(), dtype=np.int64)
    return goff, node_off, nnz_off


def batch_plan_device(row_ptr, col_idx, node_off, nv, m, nt, bucket_blocks=None, growth=2.0):
    """slaq_batch_plan for a block-diagonal union already on the device
    (int64 row_ptr, int32 global col_idx; host int64 node offsets [G+1])."""
    goff, node_off, nnz_off = _device_union_offsets(row_ptr, col_idx, node_off)
    return _plan(row_ptr, col_idx, goff, node_off, nnz_off, nv, m, nt, bucket_blocks, growth)


def batch_autotune_edges(row_ptr, col_idx, node_off, nv, m, nt, t, reps=3, stream=None):
    """slaq_batch_autotune_edges on a device union -> (plan, growth, ms): the
    fastest of the bucket-edge growths 2, 1.5 and 3, workgroup sizes tuned."""
    goff, node_off, nnz_off = _device_union_offsets(row_ptr, col_idx, node_off)
    G = len(node_off) - 1
    h, gr, ms = _vp(), ctypes.c_double(), ctypes.c_float()
    _check(lib().slaq_batch_autotune_edges(G, node_off.ctypes.data_as(_vp), nnz_off.ctypes.data_as(_vp),
                                           _ptr(goff), _ptr(row_ptr), _ptr(col_idx), nv, m, nt, _ptr(t), reps,
                                           ctypes.byref(gr), ctypes.byref(ms), ctypes.byref(h), _stream(stream)))
    return Batch(h, G, nv, m, nt, {"rp": row_ptr, "ci": col_idx, "goff": goff}), gr.value, ms.value


def union_device(graphs):
    """Block-diagonal union of device CSRs [(row_ptr, col_idx), ...] ->
    (row_ptr, col_idx with global ids, host node offsets [G+1])."""
    import numpy as np
    rps = [g[0] for g in graphs]
    cis = [g[1] for g in graphs]
    dev = rps[0].device
    n = np.array([rp.numel() - 1 for rp in rps], dtype=np.int64)
    nnz = np.array([ci.numel() for ci in cis], dtype=np.int64)
    node_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    nnz_off = np.concatenate([[0], np.cumsum(nnz)]).astype(np.int64)
    if node_off[-1] > 2**31 - 1:
        raise SlaqError(SLAQ_ERR_INVALID_ARG, "a union needs fewer than 2^31 nodes")
    G, N, E = len(graphs), int(node_off[-1]), int(nnz_off[-1])
    # every global id is below 2^31 (checked above): the shift is added in int32,
    # in place on the concatenated copy
    ci = torch.cat(cis)
    if ci.dtype != torch.int32:
        ci = ci.to(torch.int32)
    ci += torch.repeat_interleave(torch.from_numpy(node_off[:-1].astype(np.int32)).to(dev),
                                  torch.from_numpy(nnz).to(dev), output_size=E)
    # row pointers: all G arrays concatenated (n_g + 1 entries each) and
    # shifted by their graph's nonzero offset; global node i of graph g sits at
    # position i + g, and the union's closing entry is the last one
    full = torch.cat(rps)
    full += torch.repeat_interleave(torch.from_numpy(nnz_off[:-1]).to(dev), torch.from_numpy(n + 1).to(dev),
                                    output_size=N + G)
    pos = torch.arange(N + 1, dtype=torch.int64, device=dev)
    pos[:N] += torch.repeat_interleave(torch.arange(G, dtype=torch.int64, device=dev), torch.from_numpy(n).to(dev),
                                       output_size=N)
    pos[N] = N + G - 1
    return full[pos], ci, node_off


def batch_run(b, seed, t=None, heat=True, vnge=True, ritz=False, coeffs=False, graph=False, out=None,
              stream=None):
    """slaq_batch_run -> dict of the requested outputs (device tensors)."""
    dev = b._keep["rp"].device
    o = dict(out or {})
    f64 = torch.float64
    if heat and "heat" not in o:
        o["heat"] = torch.empty((b.G, b.nt), dtype=f64, device=dev)
    if vnge and "vnge" not in o:
        o["vnge"] = torch.empty(b.G, dtype=f64, device=dev)
    if coeffs and "alpha" not in o:
        o["alpha"] = torch.empty((b.G, b.nv, b.m), dtype=f64, device=dev)
        o["beta"] = torch.empty((b.G, b.nv, b.m), dtype=f64, device=dev)
        o["steps"] = torch.empty((b.G, b.nv), dtype=torch.int32, device=dev)
    if ritz and "theta" not in o:
        o["theta"] = torch.empty((b.G, b.nv, b.m), dtype=f64, device=dev)
        o["tau2"] = torch.empty((b.G, b.nv, b.m), dtype=f64, device=dev)
        o.setdefault("steps", torch.empty((b.G, b.nv), dtype=torch.int32, device=dev))
    g = o.get
    _check(lib().slaq_batch_run(b.handle, ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(t), _ptr(g("heat")),
                                _ptr(g("vnge")), _ptr(g("alpha")), _ptr(g("beta")), _ptr(g("steps")),
                                _ptr(g("theta")), _ptr(g("tau2")), SLAQ_BATCH_GRAPH if graph else 0,
                                _stream(stream)))
    return o


def batch_autotune(b, t, reps=3, stream=None):
    """slaq_batch_autotune -> chosen workgroup size and time (ms) per bucket."""
    dev = b._keep["rp"].device
    heat = torch.empty((b.G, b.nt), dtype=torch.float64, device=dev)
    vn = torch.empty(b.G, dtype=torch.float64, device=dev)
    k = len(b.buckets())
    blocks, ms = (ctypes.c_int * k)(), (ctypes.c_float * k)()
    _check(lib().slaq_batch_autotune(b.handle, _ptr(t), _ptr(heat), _ptr(vn), reps, blocks, ms, _stream(stream)))
    return [(blocks[i], ms[i]) for i in range(k)]


CLOSURE_DIN_PAD = 32


class Closure:
    """The learned closure network (slaq_closure_*); owns its parameters."""

    def __init__(self, d_in=10, hidden=256, nt=256, seed=0, stream=None):
        h = _vp()
        _check(lib().slaq_closure_create(d_in, hidden, nt, ctypes.c_uint64(seed), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.d_in, self.hidden, self.nt = d_in, hidden, nt
        P = _i64()
        offs = (ctypes.c_int64 * 8)()
        dims = (ctypes.c_int * 5)()
        _check(lib().slaq_closure_info(h, ctypes.byref(P), offs, dims))
        self.n_params = P.value
        self.offsets = list(offs)
        self.dims = list(dims)
        self._ws = None

    def _workspace(self, batch):
        b = _sz()
        _check(lib().slaq_closure_workspace(self.handle, batch, ctypes.byref(b)))
        if self._ws is None or self._ws.numel() < b.value:
            self._ws = _empty_aligned(b.value, "cuda")
        return self._ws

    def get(self, which=0, stream=None):
        """0 weights, 1 gradients of the last train step, 2 / 3 Adam moments."""
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().slaq_closure_get(self.handle, which, _ptr(out), _stream(stream)))
        return out

    def _vector(self, v, name):
        _dev(v, torch.float32, name)
        if v.numel() != self.n_params:
            raise ValueError(f"{name} must hold {self.n_params} values, got {v.numel()}")
        return v

    def set(self, params, reset_optimizer=True, stream=None):
        self._vector(params, "params")
        _check(lib().slaq_closure_set(self.handle, _ptr(params), 1 if reset_optimizer else 0, _stream(stream)))

    def step(self):
        """Adam steps taken so far."""
        s = ctypes.c_int()
        _check(lib().slaq_closure_get_step(self.handle, ctypes.byref(s)))
        return s.value

    def set_optimizer(self, m1, m2, step, stream=None):
        """Restores the Adam moments and step count."""
        self._vector(m1, "m1")
        self._vector(m2, "m2")
        _check(lib().slaq_closure_set_optimizer(self.handle, _ptr(m1), _ptr(m2), int(step), _stream(stream)))

    def layers(self, vec=None):
        """[(W, b)] views of a parameter vector (default: the weights)."""
        v = self.get(0) if vec is None else vec
        out = []
        for l in range(4):
            wo, bo = self.offsets[2 * l], self.offsets[2 * l + 1]
            W = v[wo:bo].view(self.dims[l], self.dims[l + 1])
            out.append((W, v[bo:bo + self.dims[l + 1]]))
        return out

    def train_step(self, x, y, lr, loss=None, stream=None):
        _dev(x, torch.bfloat16, "x")
        _dev(y, torch.float32, "y")
        B = x.shape[0]
        ws = self._workspace(B)
        _check(lib().slaq_closure_train_step(self.handle, _ptr(x), _ptr(y), B, ctypes.c_float(lr), _ptr(loss),
                                             _ptr(ws), ws.numel(), _stream(stream)))

    def forward(self, x, out=None, stream=None):
        _dev(x, torch.bfloat16, "x")
        B = x.shape[0]
        if out is None:
            out = torch.empty((B, self.nt), dtype=torch.float32, device="cuda")
        ws = self._workspace(B)
        _check(lib().slaq_closure_forward(self.handle, _ptr(x), B, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.slaq_closure_destroy(h)
            self.handle = None


def closure_rules(alpha, beta, steps, mf=5, stream=None):
    """mf-node Gauss rule and (mf+1)-node Gauss-Radau rule per probe, from
    Lanczos coefficients of any length > mf (alpha/beta [..., ms])."""
    ms = alpha.shape[-1]
    count = alpha.numel() // ms
    f = dict(dtype=torch.float64, device=alpha.device)
    th, w2 = torch.empty((count, mf), **f), torch.empty((count, mf), **f)
    thr, w2r = torch.empty((count, mf + 1), **f), torch.empty((count, mf + 1), **f)
    _check(lib().slaq_closure_rules(_ptr(alpha), _ptr(beta), _ptr(steps), count, ms, mf, _ptr(th), _ptr(w2), _ptr(thr),
                                    _ptr(w2r), _stream(stream)))
    return th, w2, thr, w2r


def closure_features(theta, tau2, stream=None):
    count, mf = theta.shape
    x = torch.empty((count, CLOSURE_DIN_PAD), dtype=torch.bfloat16, device=theta.device)
    _check(lib().slaq_closure_features(_ptr(theta), _ptr(tau2), count, mf, _ptr(x), _stream(stream)))
    return x


def gauss_values(theta, tau2, t, kn=None, stream=None):
    """Q[count][nt] = sum_k tau2 exp(-t theta) over the first kn nodes."""
    ks = theta.shape[-1]
    count = theta.numel() // ks
    kn = ks if kn is None else kn
    Q = torch.empty((count, t.numel()), dtype=torch.float64, device=theta.device)
    _check(lib().slaq_closure_gauss_values(_ptr(theta), _ptr(tau2), count, kn, ks, _ptr(t), t.numel(), _ptr(Q),
                                           _stream(stream)))
    return Q


def closure_targets(q_hi, q_lo, stream=None):
    y = torch.empty(q_hi.shape, dtype=torch.float32, device=q_hi.device)
    _check(lib().slaq_closure_targets(_ptr(q_hi), _ptr(q_lo), q_hi.numel(), _ptr(y), _stream(stream)))
    return y


def closure_apply(yhat, q5, qr, graph_n, nv, tol, stream=None):
    """-> heat [G][nt] and flags [G] (1 = recompute with plain SLQ)."""
    G = graph_n.numel()
    nt = q5.shape[-1]
    heat = torch.empty((G, nt), dtype=torch.float64, device=q5.device)
    flags = torch.empty(G, dtype=torch.int32, device=q5.device)
    _check(lib().slaq_closure_apply(_ptr(yhat), _ptr(q5), _ptr(qr), G, nv, nt, _ptr(graph_n), ctypes.c_double(tol),
                                    _ptr(heat), _ptr(flags), _stream(stream)))
    return heat, flags


def hutchinson_mean(q, graph_n, nv, stream=None):
    """slaq_hutchinson_mean -> heat [G][nt] = n_g / nv sum over graph g's probes."""
    G = graph_n.numel()
    nt = q.shape[-1]
    _dev(q, torch.float64, "q")
    _dev(graph_n, torch.int64, "graph_n")
    heat = torch.empty((G, nt), dtype=torch.float64, device=q.device)
    _check(lib().slaq_hutchinson_mean(_ptr(q), G, nv, nt, _ptr(graph_n), _ptr(heat), _stream(stream)))
    return heat


def profile_enable(on=True):
    _check(lib().slaq_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().slaq_profile_reset())


def profile_read(kernel):
    """(launches, total milliseconds) recorded for a stage kernel."""
    n, ms = _i64(), ctypes.c_double()
    _check(lib().slaq_profile_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def to_device(csr, device="cuda"):
    """Host CSR (numpy) -> device tensors (row_ptr int64, col_idx int32)."""
    rp = torch.from_numpy(csr.row_ptr).to(device)
    ci = torch.from_numpy(csr.col_idx).to(device)
    return rp, ci
