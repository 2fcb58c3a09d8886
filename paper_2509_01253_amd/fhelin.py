"""Python binding of the fhelin C ABI (``include/fhelin.h``).

Argument marshalling only: every step of the encrypted path runs in the HIP
kernels of ``libfhelin.so``.  PyTorch provides device memory (tensors) and
streams; ``torch`` is imported before the library is loaded so both share one
HIP runtime.  Functions carry the C names; handles are opaque ``c_void_p``.
A non-zero status raises :class:`FhelinError`.  If the library has not been
built the import fails: there is no fallback.

Ciphertext batches are 8-byte integer tensors (int64 or uint64) on the GPU
shaped ``[n_ct][2][stride][N]`` (coefficient domain), with a host list of
levels.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the library: shared HIP runtime)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhelin.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_01253_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

_i32, _u32, _u64, _dbl, _vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
_pvp = ctypes.POINTER(ctypes.c_void_p)

FHELIN_LAYER_FC = 1
FHELIN_LAYER_CONV = 2
FHELIN_APPLY_RESCALE = 1
FHELIN_APPLY_HOIST_MODDOWN = 2

FHELIN_OK = 0
FHELIN_E_INVALID_ARG = -1
FHELIN_E_UNSUPPORTED_PARAM = -2
FHELIN_E_LEVEL_MISMATCH = -3
FHELIN_E_MISSING_GALOIS_KEY = -4
FHELIN_E_OOM = -5
FHELIN_E_BUDGET = -6
FHELIN_E_HIP = -7
FHELIN_E_UNIMPLEMENTED = -8

STATUS = {
    0: "FHELIN_OK", -1: "FHELIN_E_INVALID_ARG", -2: "FHELIN_E_UNSUPPORTED_PARAM", -3: "FHELIN_E_LEVEL_MISMATCH",
    -4: "FHELIN_E_MISSING_GALOIS_KEY", -5: "FHELIN_E_OOM", -6: "FHELIN_E_BUDGET", -7: "FHELIN_E_HIP",
    -8: "FHELIN_E_UNIMPLEMENTED",
}


class fhelin_params(ctypes.Structure):
    _fields_ = [("log_n", _i32), ("n_q", _i32), ("n_p", _i32), ("dnum", _i32),
                ("q", ctypes.POINTER(_u64)), ("p", ctypes.POINTER(_u64))]


class fhelin_layer_desc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("fc_n", _i32), ("fc_out", _i32), ("fc_in", _i32), ("n1", _i32),
                ("c_in", _i32), ("c_out", _i32), ("h", _i32), ("w", _i32), ("k", _i32)]


class fhelin_ct_batch(ctypes.Structure):
    _fields_ = [("data", _vp), ("n_ct", _i32), ("stride", _i32), ("levels", ctypes.POINTER(_i32))]


class fhelin_native_params(ctypes.Structure):
    _fields_ = [("t", _i32), ("alpha", _i32), ("gamma", _i32), ("beta", _i32), ("log_d", _i32), ("l", _i32),
                ("log_p", _i32), ("engine", _i32), ("base", _i32)]


class fhelin_tune(ctypes.Structure):
    _fields_ = [("chunk", _i32), ("ks_eg", _i32), ("mac_my", _i32), ("ntt_threads", _i32), ("persistent", _i32),
                ("fuse_baby", _i32)]


_SIGS = {
    "fhelin_primes_generate": [_i32, _i32, _i32, _vp],
    "fhelin_ctx_create": [ctypes.POINTER(fhelin_params), _pvp],
    "fhelin_ctx_destroy": [_vp],
    "fhelin_ctx_set_budget": [_vp, _u64],
    "fhelin_ctx_memory": [_vp, ctypes.POINTER(_u64)],
    "fhelin_ctx_trim": [_vp],
    "fhelin_ctx_root": [_vp, _i32, ctypes.POINTER(_u64)],
    "fhelin_keyset_load": [_vp, _vp, _i32, _i32, _vp, _i32, _vp, _pvp],
    "fhelin_keyset_release": [_vp],
    "fhelin_pt_import": [_vp, _vp, _i32, _i32, _i32, _vp, _pvp],
    "fhelin_pt_encode": [_vp, _vp, _i32, _i32, _dbl, _vp, _pvp],
    "fhelin_pt_export": [_vp, _vp, _i32, _vp, _vp],
    "fhelin_ptset_info": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "fhelin_ptset_release": [_vp],
    "fhelin_plan_create": [_vp, ctypes.POINTER(fhelin_layer_desc), _pvp],
    "fhelin_plan_destroy": [_vp],
    "fhelin_plan_info": [_vp] + [ctypes.POINTER(_i32)] * 5,
    "fhelin_plan_rotations": [_vp, _vp, _vp],
    "fhelin_plan_galois": [_vp, _vp, _i32, ctypes.POINTER(_i32)],
    "fhelin_plan_encode_weights": [_vp, _vp, _vp, _vp, _vp, _i32, _dbl, _vp, _pvp],
    "fhelin_linear_apply": [_vp, _vp, _vp, _vp, ctypes.POINTER(fhelin_ct_batch), ctypes.POINTER(fhelin_ct_batch),
                            _i32, _vp],
    "fhelin_linear_apply_noalloc": [_vp, _vp, _vp, _vp, ctypes.POINTER(fhelin_ct_batch),
                                    ctypes.POINTER(fhelin_ct_batch), _i32, _vp],
    "fhelin_plan_workspace_bytes": [_vp, _vp, _i32, _i32, ctypes.POINTER(_u64)],
    "fhelin_plan_reserve_workspace": [_vp, _vp, _i32, _i32, _vp],
    "fhelin_linear_apply_multi": [_vp, _vp, _vp, _vp, ctypes.POINTER(fhelin_ct_batch),
                                  ctypes.POINTER(fhelin_ct_batch), _i32, _vp],
    "fhelin_rescale": [_vp, ctypes.POINTER(fhelin_ct_batch), ctypes.POINTER(fhelin_ct_batch), _vp],
    "fhelin_rotate": [_vp, _vp, ctypes.POINTER(fhelin_ct_batch), _vp, ctypes.POINTER(fhelin_ct_batch), _vp],
    "fhelin_ntt": [_vp, _vp, _vp, _i32, _i32, _vp],
    "fhelin_plan_get_tune": [_vp, _vp],
    "fhelin_plan_set_tune": [_vp, _vp],
    "fhelin_plan_autotune": [_vp, _vp, _vp, _vp, ctypes.POINTER(fhelin_ct_batch), ctypes.POINTER(fhelin_ct_batch),
                             _i32, _vp, _vp, ctypes.POINTER(_dbl)],
    "fhelin_graph_capture_linear": [_vp, _vp, _vp, _vp, ctypes.POINTER(fhelin_ct_batch),
                                    ctypes.POINTER(fhelin_ct_batch), _i32, _vp, _pvp],
    "fhelin_graph_launch": [_vp, _vp],
    "fhelin_graph_destroy": [_vp],
    "fhelin_ctx_faults": [_vp, ctypes.POINTER(_u32)],
    "fhelin_native_create": [ctypes.POINTER(fhelin_native_params), _pvp],
    "fhelin_native_destroy": [_vp],
    "fhelin_native_keys_load": [_vp, _vp, _vp],
    "fhelin_native_extract": [_vp, _vp, _i32, _vp, _vp],
    "fhelin_native_linear": [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "fhelin_native_pack": [_vp, _vp, _i32, _vp, _vp],
    "fhelin_native_conv": [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp],
    "fhelin_native_pack_workspace": [_vp, _i32, ctypes.POINTER(_u64)],
    "fhelin_native_profile_enable": [_vp, _i32],
    "fhelin_native_profile_read": [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "fhelin_diag_alu_rate": [_i32, _i32, _i32, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)],
    "fhelin_profile_enable": [_vp, _i32],
    "fhelin_profile_read": [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _i32
_lib.fhelin_last_error.restype = ctypes.c_char_p
_lib.fhelin_last_error.argtypes = []
_lib.fhelin_status_string.restype = ctypes.c_char_p
_lib.fhelin_status_string.argtypes = [ctypes.c_int]


class FhelinError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def fhelin_last_error() -> str:
    return _lib.fhelin_last_error().decode()


def fhelin_status_string(status: int) -> str:
    return _lib.fhelin_status_string(status).decode()


def _check(rc: int):
    if rc != 0:
        raise FhelinError(rc, fhelin_last_error())


def _stream(stream):
    if stream is None:
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return _vp(stream.cuda_stream)
    return _vp(int(stream))


def _dev_ptr(t: torch.Tensor, dtypes, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{what} has dtype {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return _vp(t.data_ptr())


_W64 = (torch.int64, torch.uint64)


def _i32_array(vals):
    vals = [int(v) for v in vals]
    return (_i32 * max(1, len(vals)))(*vals)


# --------------------------------------------------------------------------
def fhelin_primes_generate(log_n: int, bits: int, count: int) -> list:
    out = (_u64 * count)()
    _check(_lib.fhelin_primes_generate(log_n, bits, count, ctypes.cast(out, _vp)))
    return [int(v) for v in out]


def fhelin_ctx_create(log_n: int, q, p, dnum: int):
    qa = (_u64 * len(q))(*[int(v) for v in q])
    pa = (_u64 * len(p))(*[int(v) for v in p])
    prm = fhelin_params(log_n, len(q), len(p), dnum, qa, pa)
    out = _vp()
    _check(_lib.fhelin_ctx_create(ctypes.byref(prm), ctypes.byref(out)))
    return out


def fhelin_ctx_destroy(ctx):
    _check(_lib.fhelin_ctx_destroy(ctx))


def fhelin_ctx_set_budget(ctx, nbytes: int):
    _check(_lib.fhelin_ctx_set_budget(ctx, int(nbytes)))


def fhelin_ctx_memory(ctx) -> int:
    v = _u64()
    _check(_lib.fhelin_ctx_memory(ctx, ctypes.byref(v)))
    return int(v.value)


def fhelin_ctx_trim(ctx):
    _check(_lib.fhelin_ctx_trim(ctx))


def fhelin_ctx_root(ctx, mod_index: int) -> int:
    v = _u64()
    _check(_lib.fhelin_ctx_root(ctx, mod_index, ctypes.byref(v)))
    return int(v.value)


def fhelin_keyset_load(ctx, galois, level: int, evk: torch.Tensor, stream=None):
    """evk: [n_keys][beta][2][level+K][N] 8-byte integers, GPU or CPU tensor."""
    gal = (_u32 * len(galois))(*[int(g) for g in galois])
    if evk.dtype not in _W64 or not evk.is_contiguous():
        raise ValueError("evk must be a contiguous 8-byte integer tensor")
    out = _vp()
    _check(_lib.fhelin_keyset_load(ctx, ctypes.cast(gal, _vp), len(galois), level, _vp(evk.data_ptr()),
                                   1 if evk.is_cuda else 0, _stream(stream), ctypes.byref(out)))
    return out


def fhelin_keyset_release(ks):
    _check(_lib.fhelin_keyset_release(ks))


def fhelin_pt_import(ctx, pt: torch.Tensor, level=None, stream=None):
    """pt: [n_pt][level + K][N] 8-byte integers (GPU or CPU); K = number of special primes."""
    if pt.dtype not in _W64 or not pt.is_contiguous() or pt.dim() != 3:
        raise ValueError("pt must be a contiguous [n_pt][level + K][N] 8-byte integer tensor")
    if level is None:
        raise ValueError("level is required")
    out = _vp()
    _check(_lib.fhelin_pt_import(ctx, _vp(pt.data_ptr()), pt.shape[0], level, 1 if pt.is_cuda else 0,
                                 _stream(stream), ctypes.byref(out)))
    return out


def fhelin_pt_encode(ctx, slots: torch.Tensor, level: int, scale: float, stream=None):
    """slots: GPU float64 [n_pt][N/2] (real slot values)."""
    out = _vp()
    _check(_lib.fhelin_pt_encode(ctx, _dev_ptr(slots, (torch.float64,), "slots"), slots.shape[0], level,
                                 float(scale), _stream(stream), ctypes.byref(out)))
    return out


def fhelin_pt_export(ctx, pts, level: int, out: torch.Tensor, stream=None):
    _check(_lib.fhelin_pt_export(ctx, pts, level, _dev_ptr(out, _W64, "out"), _stream(stream)))


def fhelin_ptset_info(pts):
    n, l = _i32(), _i32()
    _check(_lib.fhelin_ptset_info(pts, ctypes.byref(n), ctypes.byref(l)))
    return int(n.value), int(l.value)


def fhelin_ptset_release(pts):
    _check(_lib.fhelin_ptset_release(pts))


def fhelin_plan_create(ctx, kind: int, fc_n=0, fc_out=0, fc_in=0, n1=0, c_in=0, c_out=0, h=0, w=0, k=0):
    d = fhelin_layer_desc(kind, fc_n, fc_out, fc_in, n1, c_in, c_out, h, w, k)
    out = _vp()
    _check(_lib.fhelin_plan_create(ctx, ctypes.byref(d), ctypes.byref(out)))
    return out


def fhelin_plan_destroy(plan):
    _check(_lib.fhelin_plan_destroy(plan))


def fhelin_plan_info(plan) -> dict:
    v = [_i32() for _ in range(5)]
    _check(_lib.fhelin_plan_info(plan, *[ctypes.byref(x) for x in v]))
    return dict(zip(["n_in", "n_out", "n_baby", "n_giant", "n_pt"], [int(x.value) for x in v]))


def fhelin_plan_rotations(plan):
    info = fhelin_plan_info(plan)
    b = (_i32 * info["n_baby"])()
    g = (_i32 * info["n_giant"])()
    _check(_lib.fhelin_plan_rotations(plan, ctypes.cast(b, _vp), ctypes.cast(g, _vp)))
    return list(b), list(g)


def fhelin_plan_galois(plan) -> list:
    n = _i32()
    _check(_lib.fhelin_plan_galois(plan, None, 0, ctypes.byref(n)))
    out = (_u32 * max(1, n.value))()
    _check(_lib.fhelin_plan_galois(plan, ctypes.cast(out, _vp), n.value, ctypes.byref(n)))
    return [int(v) for v in out][: n.value]


def fhelin_plan_encode_weights(ctx, plan, weights: torch.Tensor, perm_out, perm_in, level: int, scale: float,
                               stream=None):
    po = _dev_ptr(perm_out, (torch.int32,), "perm_out") if perm_out is not None else None
    pi = _dev_ptr(perm_in, (torch.int32,), "perm_in") if perm_in is not None else None
    out = _vp()
    _check(_lib.fhelin_plan_encode_weights(ctx, plan, _dev_ptr(weights, (torch.float64,), "weights"), po, pi,
                                           level, float(scale), _stream(stream), ctypes.byref(out)))
    return out


def ct_batch(data: torch.Tensor, levels) -> fhelin_ct_batch:
    """Describe a GPU tensor [n_ct][2][stride][N] with per-ciphertext levels."""
    if data.dim() != 4 or data.shape[1] != 2:
        raise ValueError("ciphertext tensor must be [n_ct][2][stride][N]")
    lv = _i32_array(levels)
    b = fhelin_ct_batch(_dev_ptr(data, _W64, "ciphertexts"), data.shape[0], data.shape[2],
                        ctypes.cast(lv, ctypes.POINTER(_i32)))
    b._keep = lv  # keep the level array alive with the struct
    return b


def fhelin_linear_apply(ctx, plan, ks, pts, x: torch.Tensor, x_levels, y: torch.Tensor, y_levels, flags=0,
                        stream=None):
    bi, bo = ct_batch(x, x_levels), ct_batch(y, y_levels)
    _check(_lib.fhelin_linear_apply(ctx, plan, ks, pts, ctypes.byref(bi), ctypes.byref(bo), flags, _stream(stream)))


def fhelin_linear_apply_noalloc(ctx, plan, ks, pts, x: torch.Tensor, x_levels, y: torch.Tensor, y_levels, flags=0,
                                stream=None):
    """fhelin_linear_apply with the library's fixed per-GPU scratch (no device allocation)."""
    bi, bo = ct_batch(x, x_levels), ct_batch(y, y_levels)
    _check(_lib.fhelin_linear_apply_noalloc(ctx, plan, ks, pts, ctypes.byref(bi), ctypes.byref(bo), flags,
                                            _stream(stream)))


def fhelin_plan_workspace_bytes(ctx, plan, n_requests: int, flags: int) -> int:
    v = _u64()
    _check(_lib.fhelin_plan_workspace_bytes(ctx, plan, n_requests, flags, ctypes.byref(v)))
    return int(v.value)


def fhelin_plan_reserve_workspace(ctx, plan, n_requests: int, flags: int, stream=None) -> None:
    """Grow the stream's workspace now for n_requests requests (no allocation later)."""
    _check(_lib.fhelin_plan_reserve_workspace(ctx, plan, n_requests, flags, _stream(stream)))


def fhelin_linear_apply_multi(ctx, plan, ks_per_request, pts, x: torch.Tensor, x_levels, y: torch.Tensor, y_levels,
                              flags=0, stream=None):
    """linear_apply with one key set per request (requests of different clients)."""
    bi, bo = ct_batch(x, x_levels), ct_batch(y, y_levels)
    arr = (_vp * max(1, len(ks_per_request)))(*[k.value if isinstance(k, _vp) else k for k in ks_per_request])
    _check(_lib.fhelin_linear_apply_multi(ctx, plan, ctypes.cast(arr, _vp), pts, ctypes.byref(bi), ctypes.byref(bo),
                                          flags, _stream(stream)))


def fhelin_plan_get_tune(plan) -> dict:
    t = fhelin_tune()
    _check(_lib.fhelin_plan_get_tune(plan, ctypes.byref(t)))
    return {"chunk": t.chunk, "ks_eg": t.ks_eg, "mac_my": t.mac_my, "ntt_threads": t.ntt_threads,
            "persistent": t.persistent, "fuse_baby": t.fuse_baby}


def fhelin_plan_set_tune(plan, chunk: int = 0, ks_eg: int = 16, mac_my: int = 2, ntt_threads: int = 256,
                         persistent: int = 0, fuse_baby: int = 0):
    t = fhelin_tune(chunk, ks_eg, mac_my, ntt_threads, persistent, fuse_baby)
    _check(_lib.fhelin_plan_set_tune(plan, ctypes.byref(t)))


def fhelin_plan_autotune(ctx, plan, ks_per_request, pts, x: torch.Tensor, x_levels, y: torch.Tensor, y_levels,
                         flags=0, stream=None):
    """Time candidate tunes on this batch, keep the fastest in the plan; y holds the layer's
    result on return.  Returns (tune dict, best time in ms)."""
    bi, bo = ct_batch(x, x_levels), ct_batch(y, y_levels)
    arr = (_vp * max(1, len(ks_per_request)))(*[k.value if isinstance(k, _vp) else k for k in ks_per_request])
    t, ms = fhelin_tune(), _dbl()
    _check(_lib.fhelin_plan_autotune(ctx, plan, ctypes.cast(arr, _vp), pts, ctypes.byref(bi), ctypes.byref(bo),
                                     flags, _stream(stream), ctypes.byref(t), ctypes.byref(ms)))
    return {"chunk": t.chunk, "ks_eg": t.ks_eg, "mac_my": t.mac_my, "ntt_threads": t.ntt_threads,
            "persistent": t.persistent, "fuse_baby": t.fuse_baby}, float(ms.value)


def fhelin_graph_capture_linear(ctx, plan, ks, pts, x: torch.Tensor, x_levels, y: torch.Tensor, y_levels, flags=0,
                                stream=None):
    """Capture one linear_apply into a graph (stream must not be the null stream)."""
    bi, bo = ct_batch(x, x_levels), ct_batch(y, y_levels)
    out = _vp()
    _check(_lib.fhelin_graph_capture_linear(ctx, plan, ks, pts, ctypes.byref(bi), ctypes.byref(bo), flags,
                                            _stream(stream), ctypes.byref(out)))
    return out


def fhelin_graph_launch(graph, stream=None):
    _check(_lib.fhelin_graph_launch(graph, _stream(stream)))


def fhelin_graph_destroy(graph):
    _check(_lib.fhelin_graph_destroy(graph))


def fhelin_rescale(ctx, x: torch.Tensor, x_levels, y: torch.Tensor, y_levels, stream=None):
    bi, bo = ct_batch(x, x_levels), ct_batch(y, y_levels)
    _check(_lib.fhelin_rescale(ctx, ctypes.byref(bi), ctypes.byref(bo), _stream(stream)))


def fhelin_rotate(ctx, ks, x: torch.Tensor, levels, steps, y: torch.Tensor, stream=None):
    bi, bo = ct_batch(x, levels), ct_batch(y, levels)
    st = _i32_array(steps)
    _check(_lib.fhelin_rotate(ctx, ks, ctypes.byref(bi), ctypes.cast(st, _vp), ctypes.byref(bo), _stream(stream)))


def fhelin_ntt(ctx, rows: torch.Tensor, mod_index, inverse: bool, stream=None):
    mi = _i32_array(mod_index)
    if rows.dim() != 2 or rows.shape[0] != len(mod_index):
        raise ValueError("rows must be [n_rows][N] with one modulus index per row")
    _check(_lib.fhelin_ntt(ctx, _dev_ptr(rows, _W64, "rows"), ctypes.cast(mi, _vp), rows.shape[0],
                           1 if inverse else 0, _stream(stream)))


def fhelin_ctx_faults(ctx) -> int:
    """Faults of bounded device-side waits since the last call (0 = none); clears them."""
    v = _u32()
    _check(_lib.fhelin_ctx_faults(ctx, ctypes.byref(v)))
    return int(v.value)


# ---- the paper's own pipeline: RLWE over Z_{2^64}[X]/Phi_M ----------------------
def _u64_tensor(x: torch.Tensor, what: str):
    if not (x.is_cuda and x.dtype in (torch.uint64, torch.int64) and x.is_contiguous()):
        raise ValueError(f"{what}: expected a contiguous 64-bit CUDA tensor")
    return _vp(x.data_ptr())


def _i32_tensor(x: torch.Tensor, what: str):
    if not (x.is_cuda and x.dtype == torch.int32 and x.is_contiguous()):
        raise ValueError(f"{what}: expected a contiguous int32 CUDA tensor")
    return _vp(x.data_ptr())


NATIVE_ENGINE_MFMA, NATIVE_ENGINE_VALU = 0, 1


def fhelin_native_create(t: int, alpha: int, gamma: int, beta: int, log_d: int, l: int, log_p: int, engine: int = 0,
                         base: int = 0):
    prm = fhelin_native_params(t, alpha, gamma, beta, log_d, l, log_p, engine, base)
    out = _vp()
    _check(_lib.fhelin_native_create(ctypes.byref(prm), ctypes.byref(out)))
    return out


def fhelin_native_destroy(nt):
    _check(_lib.fhelin_native_destroy(nt))


def fhelin_native_keys_load(nt, ksk: torch.Tensor, stream=None):
    """ksk: [alpha-gamma][l][2][N] keys of the Galois elements 1 + t^i."""
    _check(_lib.fhelin_native_keys_load(nt, _u64_tensor(ksk, "ksk"), _stream(stream)))


def fhelin_native_extract(nt, chunks: torch.Tensor, rows: torch.Tensor, stream=None):
    """chunks [n_chunks][phi(t^gamma)][2][N] -> rows [n_chunks N][2][N]."""
    _check(_lib.fhelin_native_extract(nt, _u64_tensor(chunks, "chunks"), chunks.shape[0], _u64_tensor(rows, "rows"),
                                      _stream(stream)))


def fhelin_native_linear(nt, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, rows: torch.Tensor,
                         out: torch.Tensor, stream=None):
    """out[o] = sum val[k] rows[col[k]] over CSR row o (int32 CUDA arrays)."""
    _check(_lib.fhelin_native_linear(nt, _i32_tensor(row_ptr, "row_ptr"), _i32_tensor(col, "col"),
                                     _i32_tensor(val, "val"), out.shape[0], _u64_tensor(rows, "rows"),
                                     _u64_tensor(out, "out"), _stream(stream)))


def fhelin_native_conv(nt, c_in: int, c_out: int, h: int, w: int, k: int, stride: int, weights: torch.Tensor,
                       out_row: torch.Tensor, rows: torch.Tensor, out: torch.Tensor, stream=None):
    """Convolution on channels-last rows; output (position, co) to out[out_row[pos c_out + co]]."""
    _check(_lib.fhelin_native_conv(nt, c_in, c_out, h, w, k, stride, _i32_tensor(weights, "weights"),
                                   _i32_tensor(out_row, "out_row"), _u64_tensor(rows, "rows"), _u64_tensor(out, "out"),
                                   _stream(stream)))


def fhelin_native_pack(nt, rows: torch.Tensor, packed: torch.Tensor, stream=None):
    """rows [n][2][N] -> packed [ceil(n / phi(t^beta))][2][N]."""
    _check(_lib.fhelin_native_pack(nt, _u64_tensor(rows, "rows"), rows.shape[0], _u64_tensor(packed, "packed"),
                                   _stream(stream)))


def fhelin_native_profile_enable(nt, enable: bool = True):
    _check(_lib.fhelin_native_profile_enable(nt, 1 if enable else 0))


def fhelin_native_profile_read(nt, kernel: str):
    """(launches, total_ms, units, bytes) of one kernel class of the native pipeline."""
    n, ms, u, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.fhelin_native_profile_read(nt, kernel.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(u),
                                           ctypes.byref(by)))
    return int(n.value), float(ms.value), float(u.value), float(by.value)


def fhelin_native_pack_workspace(nt, n_rows: int) -> int:
    v = _u64()
    _check(_lib.fhelin_native_pack_workspace(nt, n_rows, ctypes.byref(v)))
    return int(v.value)


def fhelin_diag_alu_rate(op: int, waves_per_simd: int, iters: int):
    """(core GHz, clocks per wave-level op on one SIMD, lane-ops per second) of one probe."""
    g, c, o = _dbl(), _dbl(), _dbl()
    _check(_lib.fhelin_diag_alu_rate(op, waves_per_simd, iters, ctypes.byref(g), ctypes.byref(c), ctypes.byref(o)))
    return g.value, c.value, o.value


def fhelin_profile_enable(ctx, enable: bool = True):
    _check(_lib.fhelin_profile_enable(ctx, 1 if enable else 0))


def fhelin_profile_read(ctx, kernel: str):
    """(launches, total_ms, units, bytes) for one kernel class."""
    n, ms, u, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.fhelin_profile_read(ctx, kernel.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(u),
                                    ctypes.byref(by)))
    return int(n.value), float(ms.value), float(u.value), float(by.value)
