"""Python binding of libdlic, the DLIC hot path on MI355X (gfx950).

Argument marshalling only: every step of encoding and decoding runs in the
HIP kernels behind the C ABI declared in include/dlic.h.  PyTorch supplies
device memory and streams.  The functions named dlic_* mirror the C entry
points one to one; encode()/decode()/density() are conveniences that
allocate buffers with torch and call them.  There is no CPU fallback: if
libdlic.so is missing or no gfx950 device is usable, calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_char_p, c_float, c_int, c_int32, c_size_t, c_uint32, c_uint64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DLIC_LIB may name another build of the same library (e.g. an experiment).
LIB_PATH = os.environ.get("DLIC_LIB") or os.path.join(_HERE, "libdlic.so")

DLIC_OK, DLIC_ERR_ARG, DLIC_ERR_CAPACITY, DLIC_ERR_CORRUPT = 0, 1, 2, 3
DLIC_ERR_MODEL_MISMATCH, DLIC_ERR_UNSUPPORTED, DLIC_ERR_HIP, DLIC_ERR_TIMEOUT = 4, 5, 6, 7
DLIC_FP32, DLIC_BF16, DLIC_FP8_E4M3, DLIC_FP64, DLIC_FP8_W8A8 = 0, 1, 2, 3, 4
FNV_OFFSET = 0xCBF29CE484222325
HEADER_BYTES = 36
DECODE_NOALLOC_BYTES = 8 << 20  # DLIC_DECODE_NOALLOC_BYTES of dlic.h

# Every symbol include/dlic.h declares.
EXPORTS = (
    "dlic_status_string", "dlic_fnv1a64", "dlic_host_constants", "dlic_quantize_weights",
    "dlic_w8a8_multipliers", "dlic_activation_range",
    "dlic_encode_bound",
    "dlic_encode_workspace", "dlic_decode_workspace", "dlic_peek_header", "dlic_init",
    "dlic_encode", "dlic_decode", "dlic_set_spin_limit", "dlic_density",
    "dlic_rans_encode_cf", "dlic_rans_decode_tables", "dlic_set_timing", "dlic_kernel_times",
    "dlic_set_decode_profile", "dlic_nll_workspace", "dlic_nll_fwd_bwd", "dlic_adam_step",
    "dlic_batch_create", "dlic_batch_destroy", "dlic_batch_sizes", "dlic_batch_layout",
    "dlic_encode_batch", "dlic_decode_batch", "dlic_batch_capture", "dlic_batch_replay",
    "dlic_wallclock_hz", "dlic_decode_noalloc", "dlic_batch_tune", "dlic_latency_probe",
    "dlic_set_decode_delays", "dlic_deep_workspace", "dlic_deep_encode", "dlic_deep_decode",
    "dlic_deep_density", "dlic_set_deep_decode_grid", "dlic_deep_decode_grid",
    "dlic_volume_encode_bound", "dlic_volume_workspace", "dlic_volume_encode", "dlic_volume_decode",
    "dlic_volume_density", "dlic_peek_volume", "dlic_host_scale", "dlic_deep_slice_stamps",
    "dlic_net_forms",
)


class DlicError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = int(status)
        super().__init__(f"{where}: {status_string(self.status)} ({self.status})")


class dlic_model(ctypes.Structure):
    _fields_ = [("k_in", c_int32), ("h1", c_int32), ("h2", c_int32), ("n_out", c_int32),
                ("dtype", c_int32), ("reserved", c_int32), ("d_w1", c_void_p), ("d_w2", c_void_p),
                ("d_w3", c_void_p), ("d_b1", c_void_p), ("d_b2", c_void_p), ("d_b3", c_void_p),
                ("d_wscale", c_void_p), ("fingerprint", c_uint64)]


class dlic_coder(ctypes.Structure):
    """groups, lanes_per_group, strips (row strips per group; 0 or 1: one)."""
    _fields_ = [("groups", c_int32), ("lanes_per_group", c_int32), ("strips", c_int32)]


DEEP_LAYERS = 6


class dlic_deep_model(ctypes.Structure):
    _fields_ = [("hidden", c_int32), ("k_in", c_int32), ("d_w", c_void_p * DEEP_LAYERS),
                ("d_b", c_void_p * DEEP_LAYERS), ("fingerprint", c_uint64), ("depth", c_int32)]


_lib = None


def lib():
    """The loaded libdlic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2207_05152_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, S = c_void_p, c_size_t
    sig = {
        "dlic_status_string": (c_char_p, [c_int]),
        "dlic_fnv1a64": (c_uint64, [c_uint64, P, S]),
        "dlic_host_constants": (None, [P, P, P, P]),
        "dlic_quantize_weights": (c_int, [c_int32, P, S, P, P]),
        "dlic_w8a8_multipliers": (c_int, [P, P]),
        "dlic_activation_range": (c_int, [POINTER(dlic_model), P, c_int32, c_int32, P, P]),
        "dlic_encode_bound": (S, [c_int32, c_int32, POINTER(dlic_coder)]),
        "dlic_encode_workspace": (S, [c_int32, c_int32, POINTER(dlic_coder)]),
        "dlic_decode_workspace": (S, [c_int32, c_int32, POINTER(dlic_coder)]),
        "dlic_peek_header": (c_int, [P, S, POINTER(c_int32), POINTER(c_int32), POINTER(dlic_coder),
                                     POINTER(c_uint64), POINTER(c_int32), POINTER(c_int32),
                                     POINTER(c_int32)]),
        "dlic_init": (c_int, [c_int]),
        "dlic_encode": (c_int, [POINTER(dlic_model), POINTER(dlic_coder), P, c_int32, c_int32, P, S,
                                P, P, S, P]),
        "dlic_decode": (c_int, [POINTER(dlic_model), POINTER(dlic_coder), P, S, P, c_int32, c_int32,
                                P, P, S, P]),
        "dlic_decode_noalloc": (c_int, [POINTER(dlic_model), POINTER(dlic_coder), P, S, P, c_int32,
                                        c_int32, P, P]),
        "dlic_set_spin_limit": (None, [c_uint32]),
        "dlic_set_decode_delays": (None, [c_uint32, c_uint32]),
        "dlic_net_forms": (c_int, [POINTER(dlic_model), P, ctypes.c_int64, c_int32, P, P, P]),
        "dlic_density": (c_int, [POINTER(dlic_model), P, c_int32, c_int32, P, P, P, P]),
        "dlic_rans_encode_cf": (c_int, [POINTER(dlic_coder), c_int32, c_int32, P, P, S, P, P, S, P]),
        "dlic_rans_decode_tables": (c_int, [POINTER(dlic_coder), c_int32, c_int32, P, c_int32, P, P,
                                            S, P, P, P, S, P]),
        "dlic_set_timing": (None, [c_int]),
        "dlic_kernel_times": (c_int, [P, P, c_int]),
        "dlic_set_decode_profile": (None, [P]),
        "dlic_nll_workspace": (S, [ctypes.c_int64, POINTER(dlic_model)]),
        "dlic_nll_fwd_bwd": (c_int, [POINTER(dlic_model), P, c_int32, c_int32, c_int32, P,
                                     ctypes.c_int64, P, P, P, S, P]),
        "dlic_adam_step": (c_int, [ctypes.c_int64, P, P, P, P, c_int32, c_float, c_float, c_float,
                                   c_float, P]),
        "dlic_batch_create": (c_int, [POINTER(dlic_model), c_int32, P, P, c_int32, POINTER(P)]),
        "dlic_batch_destroy": (None, [P]),
        "dlic_batch_tune": (c_int, [P, c_int32, c_int32]),
        "dlic_batch_sizes": (c_int, [P, POINTER(S), POINTER(S), POINTER(S), POINTER(c_int32)]),
        "dlic_batch_layout": (c_int, [P, P, P, P]),
        "dlic_encode_batch": (c_int, [P, P, P, P, P, P, S, P]),
        "dlic_decode_batch": (c_int, [P, P, P, P, P, P, P, S, P]),
        "dlic_batch_capture": (c_int, [P, c_int32, P, P, P, P, P, P, S]),
        "dlic_batch_replay": (c_int, [P, c_int32, P]),
        "dlic_wallclock_hz": (ctypes.c_double, []),
        "dlic_latency_probe": (c_int, [P, c_int32, P, S, P]),
        "dlic_deep_workspace": (S, [POINTER(dlic_deep_model), c_int32, c_int32, P, c_int32]),
        "dlic_deep_encode": (c_int, [POINTER(dlic_deep_model), POINTER(dlic_coder), P, c_int32,
                                     c_int32, P, S, P, P, S, P]),
        "dlic_deep_decode": (c_int, [POINTER(dlic_deep_model), POINTER(dlic_coder), P, S, P,
                                     c_int32, c_int32, P, P, S, P]),
        "dlic_deep_density": (c_int, [POINTER(dlic_deep_model), P, c_int32, c_int32, P, P, P, P,
                                      S, P]),
        "dlic_set_deep_decode_grid": (None, [c_int32]),
        "dlic_deep_decode_grid": (c_int32, []),
        "dlic_volume_encode_bound": (S, [c_int32, c_int32, c_int32, POINTER(dlic_coder)]),
        "dlic_volume_workspace": (S, [POINTER(dlic_deep_model), c_int32, c_int32, c_int32, P,
                                      c_int32]),
        "dlic_host_scale": (c_int, [c_int32, P]),
        "dlic_deep_slice_stamps": (c_int, [P, c_int32]),
        "dlic_volume_encode": (c_int, [POINTER(dlic_deep_model), POINTER(dlic_coder), P, c_int32,
                                       c_int32, c_int32, c_int32, P, S, P, P, S, P]),
        "dlic_volume_decode": (c_int, [POINTER(dlic_deep_model), POINTER(dlic_coder), P, S, P,
                                       c_int32, c_int32, c_int32, c_int32, P, P, S, P]),
        "dlic_volume_density": (c_int, [POINTER(dlic_deep_model), P, c_int32, c_int32, c_int32,
                                        c_int32, P, P, P, P, S, P]),
        "dlic_peek_volume": (c_int, [P, S, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                     POINTER(c_int32), POINTER(dlic_coder)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_string(s: int) -> str:
    try:
        return lib().dlic_status_string(int(s)).decode()
    except RuntimeError:
        return f"status {s}"


def _check(rc: int, where: str):
    if rc != DLIC_OK:
        raise DlicError(rc, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ---- one-to-one wrappers of the C entry points ---------------------------------

def dlic_fnv1a64(h: int, data: bytes) -> int:
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    return int(lib().dlic_fnv1a64(h, buf, len(data)))


def dlic_quantize_weights(dtype: int, w) -> tuple:
    """Stored form of one FP32 matrix: (uint16 BF16 bits or uint8 e4m3 codes, FP32 scale)."""
    a = np.ascontiguousarray(w, dtype=np.float32)
    out = np.empty(a.shape, np.uint16 if dtype == DLIC_BF16 else np.uint8)
    sc = np.zeros(1, np.float32)
    _check(lib().dlic_quantize_weights(dtype, a.ctypes.data, a.size, out.ctypes.data,
                                       sc.ctypes.data), "dlic_quantize_weights")
    return out, np.float32(sc[0])


def dlic_w8a8_multipliers(amax) -> np.ndarray:
    a = np.ascontiguousarray(amax, dtype=np.float32)
    out = np.zeros(3, np.float32)
    _check(lib().dlic_w8a8_multipliers(a.ctypes.data, out.ctypes.data), "dlic_w8a8_multipliers")
    return out


def dlic_activation_range(model: dlic_model, d_img, h, w, d_amax, stream=None):
    _check(lib().dlic_activation_range(ctypes.byref(model), _ptr(d_img), h, w, _ptr(d_amax),
                                       _stream(stream)), "dlic_activation_range")


def dlic_host_constants():
    S = np.empty(4097, np.float32); D = np.empty(4097, np.float32)
    beta = np.empty(257, np.float32); scale = np.empty(256, np.float32)
    lib().dlic_host_constants(S.ctypes.data, D.ctypes.data, beta.ctypes.data, scale.ctypes.data)
    return S, D, beta, scale


def dlic_encode_bound(h: int, w: int, coder: dlic_coder) -> int:
    return int(lib().dlic_encode_bound(h, w, ctypes.byref(coder)))


def dlic_encode_workspace(h: int, w: int, coder: dlic_coder) -> int:
    return int(lib().dlic_encode_workspace(h, w, ctypes.byref(coder)))


def dlic_decode_workspace(h: int, w: int, coder: dlic_coder) -> int:
    return int(lib().dlic_decode_workspace(h, w, ctypes.byref(coder)))


def dlic_peek_header(head: bytes) -> dict:
    h, w, h1, h2, dt = (c_int32() for _ in range(5))
    fp = c_uint64()
    cd = dlic_coder()
    buf = ctypes.create_string_buffer(bytes(head), len(head))
    _check(lib().dlic_peek_header(buf, len(head), ctypes.byref(h), ctypes.byref(w), ctypes.byref(cd),
                                  ctypes.byref(fp), ctypes.byref(h1), ctypes.byref(h2),
                                  ctypes.byref(dt)), "dlic_peek_header")
    return dict(h=h.value, w=w.value, coder=cd, fingerprint=fp.value, h1=h1.value, h2=h2.value,
                dtype=dt.value)


def dlic_init(device: int = 0):
    _check(lib().dlic_init(device), "dlic_init")


def dlic_encode(model: dlic_model, coder: dlic_coder, d_img, h, w, d_out, out_cap, d_out_len,
                d_ws, ws_bytes, stream=None):
    _check(lib().dlic_encode(ctypes.byref(model), ctypes.byref(coder), _ptr(d_img), h, w, _ptr(d_out),
                             out_cap, _ptr(d_out_len), _ptr(d_ws), ws_bytes, _stream(stream)),
           "dlic_encode")


def dlic_decode(model: dlic_model, coder: dlic_coder, d_bits, n_bytes, d_img, h, w, d_status,
                d_ws, ws_bytes, stream=None):
    _check(lib().dlic_decode(ctypes.byref(model), ctypes.byref(coder), _ptr(d_bits), n_bytes,
                             _ptr(d_img), h, w, _ptr(d_status), _ptr(d_ws), ws_bytes,
                             _stream(stream)), "dlic_decode")


def dlic_decode_noalloc(model: dlic_model, coder: dlic_coder, d_bits, n_bytes, d_img, h, w,
                        d_status, stream=None):
    _check(lib().dlic_decode_noalloc(ctypes.byref(model), ctypes.byref(coder), _ptr(d_bits),
                                     n_bytes, _ptr(d_img), h, w, _ptr(d_status), _stream(stream)),
           "dlic_decode_noalloc")


def dlic_decode_noalloc_limit() -> int:
    """DLIC_DECODE_NOALLOC_BYTES of dlic.h: the no-alloc decode's fixed workspace."""
    return DECODE_NOALLOC_BYTES


def dlic_net_forms(model: dlic_model, d_feats, n, lanes, d_out16, d_out4, stream=None):
    _check(lib().dlic_net_forms(ctypes.byref(model), _ptr(d_feats), int(n), int(lanes),
                                _ptr(d_out16), _ptr(d_out4), _stream(stream)), "dlic_net_forms")


def dlic_set_spin_limit(polls: int):
    lib().dlic_set_spin_limit(int(polls))


def dlic_set_decode_delays(seed: int, max_cycles: int):
    lib().dlic_set_decode_delays(int(seed), int(max_cycles))


def dlic_density(model: dlic_model, d_img, h, w, d_out15=None, d_cf=None, d_tables=None,
                 stream=None):
    _check(lib().dlic_density(ctypes.byref(model), _ptr(d_img), h, w, _ptr(d_out15), _ptr(d_cf),
                              _ptr(d_tables), _stream(stream)), "dlic_density")


def dlic_rans_encode_cf(coder: dlic_coder, h, w, d_cf, d_out, out_cap, d_out_len, d_ws, ws_bytes,
                        stream=None):
    _check(lib().dlic_rans_encode_cf(ctypes.byref(coder), h, w, _ptr(d_cf), _ptr(d_out), out_cap,
                                     _ptr(d_out_len), _ptr(d_ws), ws_bytes, _stream(stream)),
           "dlic_rans_encode_cf")


def dlic_rans_decode_tables(coder: dlic_coder, h, w, d_tables, n_tables, d_tidx, d_bits, n_bytes,
                            d_sym, d_status, d_ws, ws_bytes, stream=None):
    _check(lib().dlic_rans_decode_tables(ctypes.byref(coder), h, w, _ptr(d_tables), n_tables,
                                         _ptr(d_tidx), _ptr(d_bits), n_bytes, _ptr(d_sym),
                                         _ptr(d_status), _ptr(d_ws), ws_bytes, _stream(stream)),
           "dlic_rans_decode_tables")


def dlic_set_timing(enable: bool):
    lib().dlic_set_timing(1 if enable else 0)


def dlic_set_decode_profile(d_counters):
    lib().dlic_set_decode_profile(_ptr(d_counters))


def dlic_kernel_times(max_n: int = 16):
    ms = (c_float * max_n)()
    names = (c_char_p * max_n)()
    n = lib().dlic_kernel_times(ctypes.cast(ms, c_void_p), ctypes.cast(names, c_void_p), max_n)
    return [(names[i].decode(), float(ms[i])) for i in range(n)]


# ---- conveniences (torch-allocated buffers) -------------------------------------

def default_coder(h: int, lanes: int = 4, rows_per_group: int = 24, strips: int = 1) -> dlic_coder:
    """G = ceil(h / rows_per_group) groups of `lanes` interleaved lanes, each
    coding `strips` row strips spread over the image.

    Groups of 24 rows with 4 lanes each (64 x 4 = 256 lanes on a 1536-row
    image) decode with a workgroup per group and 16 of its coder lanes per
    pixel in the symbol search.  With 2 strips per group, when a strip is
    shorter than the wavefront's band of active rows (about w/3), a group has
    rows in half as many steps at once."""
    g = max(1, math.ceil(h / rows_per_group))
    if g > 1 and h < 2 * g:
        g = max(1, h // 2)
    while strips > 1 and h < 2 * g * strips:
        strips -= 1
    return dlic_coder(g, lanes, strips)


DTYPES = {"fp32": DLIC_FP32, "bf16": DLIC_BF16, "fp8": DLIC_FP8_E4M3, "fp8a8": DLIC_FP8_W8A8}


class Model:
    """Network weights resident on a device, with their C descriptor.

    dtype 'fp32' keeps the FP32 matrices; 'bf16' and 'fp8' store them as the
    library's dlic_quantize_weights converts them (biases stay FP32)."""

    def __init__(self, weights: dict, device="cuda", dtype: str = "fp32", calibration=None):
        import torch
        code = DTYPES[dtype]
        self.dtype = dtype
        self.np = {}
        scales = []
        for k in ("W1", "W2", "W3"):
            w32 = np.ascontiguousarray(weights[k], dtype=np.float32)
            if code == DLIC_FP32:
                self.np[k], s = w32, np.float32(1.0)
            else:
                self.np[k], s = dlic_quantize_weights(
                    DLIC_FP8_E4M3 if code == DLIC_FP8_W8A8 else code, w32)
            scales.append(s)
        for k in ("b1", "b2", "b3"):
            self.np[k] = np.ascontiguousarray(weights[k], dtype=np.float32)
        self.act_max = None
        if code == DLIC_FP8_W8A8:
            # activation multipliers from the FP32 net's ranges on calibration images
            if not calibration:
                raise ValueError("dtype 'fp8a8' needs calibration images")
            ref = Model(weights, device)
            amax = torch.zeros(2, dtype=torch.float32, device=device)
            for im in calibration:
                t = im if isinstance(im, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(im))
                t = t.to(device)
                dlic_activation_range(ref.c, t.contiguous(), t.shape[0], t.shape[1], amax)
            self.act_max = np.concatenate([[1.0], amax.cpu().numpy()]).astype(np.float32)
            scales += list(dlic_w8a8_multipliers(self.act_max))
        self.scales = np.array(scales, dtype=np.float32)
        self.t = {k: torch.from_numpy(v).to(device) for k, v in self.np.items()}
        self.t_scales = torch.from_numpy(self.scales).to(device)
        h = FNV_OFFSET
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            h = dlic_fnv1a64(h, self.np[k].tobytes())
        if code in (DLIC_FP8_E4M3, DLIC_FP8_W8A8):
            h = dlic_fnv1a64(h, self.scales.tobytes())
        self.fingerprint = h
        h1, h2 = self.np["W1"].shape[0], self.np["W2"].shape[0]
        self.c = dlic_model(12, h1, h2, 15, code, 0, _ptr(self.t["W1"]), _ptr(self.t["W2"]),
                            _ptr(self.t["W3"]), _ptr(self.t["b1"]), _ptr(self.t["b2"]),
                            _ptr(self.t["b3"]),
                            _ptr(self.t_scales) if code in (DLIC_FP8_E4M3, DLIC_FP8_W8A8)
                            else None, h)


def _empty(n, dtype, device="cuda"):
    import torch
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


def encode(img, model: Model, coder: dlic_coder | None = None, stream=None):
    """Encode a [h, w] uint8 device tensor; returns the stream as a uint8 device tensor."""
    import torch
    h, w = img.shape
    coder = coder or default_coder(h)
    cap = dlic_encode_bound(h, w, coder)
    out = _empty(cap, torch.uint8, img.device)
    olen = _empty(1, torch.int64, img.device)
    wsb = dlic_encode_workspace(h, w, coder)
    ws = _empty(wsb, torch.uint8, img.device)
    dlic_encode(model.c, coder, img.contiguous(), h, w, out, cap, olen, ws, wsb, stream)
    n = int(olen.item())
    return out[:n]


def decode(bits, model: Model, stream=None, check=True):
    """Decode a stream (uint8 device tensor); returns ([h, w] uint8 tensor, status)."""
    import torch
    head = bits[:HEADER_BYTES].cpu().numpy().tobytes()
    hd = dlic_peek_header(head)
    h, w, coder = hd["h"], hd["w"], hd["coder"]
    img = torch.empty((h, w), dtype=torch.uint8, device=bits.device)
    st = torch.zeros(1, dtype=torch.int32, device=bits.device)
    wsb = dlic_decode_workspace(h, w, coder)
    ws = _empty(wsb, torch.uint8, bits.device)
    dlic_decode(model.c, coder, bits.contiguous(), bits.numel(), img, h, w, st, ws, wsb, stream)
    status = int(st.item())
    if check and status != DLIC_OK:
        raise DlicError(status, "dlic_decode (device status)")
    return img, status


def density(img, model: Model, tables=False, stream=None):
    """Raw outputs [n, 15], packed intervals [n] and optionally tables [n, 257] of an image."""
    import torch
    h, w = img.shape
    n = h * w
    out15 = torch.empty((n, 15), dtype=torch.float32, device=img.device)
    cf = torch.empty(n, dtype=torch.int32, device=img.device)
    tab = torch.empty((n, 257), dtype=torch.int32, device=img.device) if tables else None
    dlic_density(model.c, img.contiguous(), h, w, out15, cf, tab, stream)
    return out15, cf, tab


# ---- the six-layer softmax-256 network ----------------------------------------------

class DeepModel:
    """The paper's six-layer network with the softmax head, resident on a device:
    layers = [(W, b)] * 6 (FP32, W [out, in]: k -> H, H -> H x 4, H -> N with k = 12,
    or 21 for volumes with the slice below, and N = 256 levels for 8-bit samples or
    4096 for 12-bit ones).  The library's dlic_quantize_weights stores the matrices as
    BF16; biases stay FP32."""

    def __init__(self, layers, device="cuda"):
        import torch
        if len(layers) != DEEP_LAYERS:
            raise ValueError("six layers")
        self.hidden = int(np.asarray(layers[0][0]).shape[0])
        self.k_in = int(np.asarray(layers[0][0]).shape[1])
        n_out = int(np.asarray(layers[-1][0]).shape[0])
        if n_out not in (256, 4096):
            raise ValueError("256 or 4096 output levels")
        self.depth = 8 if n_out == 256 else 12
        self.w, self.b = [], []
        h = FNV_OFFSET
        for W, b in layers:
            wq, _ = dlic_quantize_weights(DLIC_BF16, np.ascontiguousarray(W, dtype=np.float32))
            bb = np.ascontiguousarray(b, dtype=np.float32)
            h = dlic_fnv1a64(h, wq.tobytes())
            h = dlic_fnv1a64(h, bb.tobytes())
            self.w.append(torch.from_numpy(wq.view(np.int16)).to(device))
            self.b.append(torch.from_numpy(bb).to(device))
        self.fingerprint = h
        self.c = dlic_deep_model(self.hidden, self.k_in,
                                 (c_void_p * DEEP_LAYERS)(*[_ptr(t) for t in self.w]),
                                 (c_void_p * DEEP_LAYERS)(*[_ptr(t) for t in self.b]), h,
                                 self.depth)


def dlic_deep_workspace(model: "DeepModel", h, w, coder, decode) -> int:
    return int(lib().dlic_deep_workspace(ctypes.byref(model.c), h, w,
                                         ctypes.byref(coder) if coder is not None else None, decode))


def dlic_volume_workspace(model: "DeepModel", z, h, w, coder, decode) -> int:
    return int(lib().dlic_volume_workspace(ctypes.byref(model.c), z, h, w,
                                           ctypes.byref(coder) if coder is not None else None,
                                           decode))


def dlic_deep_slice_stamps(n: int) -> np.ndarray:
    """Real-time stamps of the last 8-bit deep decode: [start, slice 0 done, ...]."""
    out = np.zeros(n, np.uint64)
    _check(lib().dlic_deep_slice_stamps(out.ctypes.data, int(n)), "dlic_deep_slice_stamps")
    return out


def dlic_host_scale(depth: int) -> np.ndarray:
    out = np.zeros(1 << depth, np.float32)
    _check(lib().dlic_host_scale(int(depth), out.ctypes.data), "dlic_host_scale")
    return out


def _sample_dtype(depth):
    """Device storage of samples: uint8, or int16 holding 12-bit values (< 4096)."""
    import torch
    return torch.uint8 if depth == 8 else torch.int16


def _check_samples(t, model):
    import torch
    if t.dtype != _sample_dtype(model.depth):
        want = "uint8" if model.depth == 8 else "int16 (12-bit values)"
        raise ValueError(f"samples of a {model.depth}-bit model are {want} tensors")


def deep_encode(img, model: DeepModel, coder: dlic_coder, stream=None):
    """Encode a [h, w] device tensor with the softmax network: uint8 samples, or
    int16 tensors of 12-bit values for a 4096-level network."""
    import torch
    _check_samples(img, model)
    h, w = img.shape
    cap = dlic_encode_bound(h, w, coder)
    out = _empty(cap, torch.uint8, img.device)
    olen = _empty(1, torch.int64, img.device)
    wsb = dlic_deep_workspace(model, h, w, coder, 0)
    ws = _empty(wsb, torch.uint8, img.device)
    _check(lib().dlic_deep_encode(ctypes.byref(model.c), ctypes.byref(coder),
                                  _ptr(img.contiguous()), h, w, _ptr(out), cap, _ptr(olen),
                                  _ptr(ws), wsb, _stream(stream)), "dlic_deep_encode")
    n = int(olen.item())
    if n == 0:
        raise DlicError(DLIC_ERR_ARG, "dlic_deep_encode: a sample exceeds the bit depth")
    return out[:n]


def deep_decode(bits, model: DeepModel, stream=None, check=True):
    """Decode a stream of deep_encode; returns ([h, w] tensor, status)."""
    import torch
    hd = dlic_peek_header(bits[:HEADER_BYTES].cpu().numpy().tobytes())
    h, w, coder = hd["h"], hd["w"], hd["coder"]
    img = torch.empty((h, w), dtype=_sample_dtype(model.depth), device=bits.device)
    st = torch.zeros(1, dtype=torch.int32, device=bits.device)
    wsb = dlic_deep_workspace(model, h, w, coder, 1)
    ws = _empty(wsb, torch.uint8, bits.device)
    _check(lib().dlic_deep_decode(ctypes.byref(model.c), ctypes.byref(coder),
                                  _ptr(bits.contiguous()), bits.numel(), _ptr(img), h, w,
                                  _ptr(st), _ptr(ws), wsb, _stream(stream)), "dlic_deep_decode")
    status = int(st.item())
    if check and status != DLIC_OK:
        raise DlicError(status, "dlic_deep_decode (device status)")
    return img, status


def deep_density(img, model: DeepModel, logits=True, tables=False, stream=None):
    """Logits [n, N] FP32, packed intervals [n] and optionally tables F(0..N-1)
    [n, N] (u16 in int16 storage) of every pixel of an image (N = 256 or 4096)."""
    import torch
    _check_samples(img, model)
    h, w = img.shape
    n, N = h * w, 1 << model.depth
    lg = torch.empty((n, N), dtype=torch.float32, device=img.device) if logits else None
    cf = torch.empty(n, dtype=torch.int32, device=img.device)
    tab = torch.empty((n, N), dtype=torch.int16, device=img.device) if tables else None
    wsb = dlic_deep_workspace(model, h, w, None, -1)
    ws = _empty(wsb, torch.uint8, img.device)
    _check(lib().dlic_deep_density(ctypes.byref(model.c), _ptr(img.contiguous()), h, w,
                                   _ptr(lg) if lg is not None else None, _ptr(cf),
                                   _ptr(tab) if tab is not None else None, _ptr(ws), wsb,
                                   _stream(stream)), "dlic_deep_density")
    return lg, cf, tab


def dlic_set_deep_decode_grid(workgroups: int):
    lib().dlic_set_deep_decode_grid(int(workgroups))


def dlic_deep_decode_grid() -> int:
    return int(lib().dlic_deep_decode_grid())


def dlic_peek_volume(head: bytes) -> dict:
    z, h, ws, k = (c_int32() for _ in range(4))
    cd = dlic_coder()
    buf = ctypes.create_string_buffer(bytes(head), len(head))
    _check(lib().dlic_peek_volume(buf, len(head), ctypes.byref(z), ctypes.byref(h), ctypes.byref(ws),
                                  ctypes.byref(k), ctypes.byref(cd)), "dlic_peek_volume")
    return dict(z=z.value, h=h.value, ws=ws.value, k_in=k.value, coder=cd)


def volume_encode(vol, model: DeepModel, coder: dlic_coder, ws: int = 0, stream=None):
    """Encode a [z, h, w] device tensor (slices along the first axis; samples as for
    deep_encode)."""
    import torch
    _check_samples(vol, model)
    z, h, w = vol.shape
    cap = int(lib().dlic_volume_encode_bound(z, h, w, ctypes.byref(coder)))
    if cap == 0:
        raise DlicError(DLIC_ERR_UNSUPPORTED, "dlic_volume_encode_bound")
    out = _empty(cap, torch.uint8, vol.device)
    olen = _empty(1, torch.int64, vol.device)
    wsb = dlic_volume_workspace(model, z, h, w, coder, 0)
    wsp = _empty(wsb, torch.uint8, vol.device)
    _check(lib().dlic_volume_encode(ctypes.byref(model.c), ctypes.byref(coder),
                                    _ptr(vol.contiguous()), z, h, w, ws, _ptr(out), cap, _ptr(olen),
                                    _ptr(wsp), wsb, _stream(stream)), "dlic_volume_encode")
    n = int(olen.item())
    if n == 0:
        raise DlicError(DLIC_ERR_ARG, "dlic_volume_encode: a sample exceeds the bit depth")
    return out[:n]


def volume_decode(bits, model: DeepModel, stream=None, check=True):
    """Decode a stream of volume_encode; returns ([z, h, w] tensor, status)."""
    import torch
    hd = dlic_peek_header(bits[:HEADER_BYTES].cpu().numpy().tobytes())
    hv = dlic_peek_volume(bits[:HEADER_BYTES].cpu().numpy().tobytes())
    z, h, w, ws, coder = hv["z"], hv["h"], hd["w"], hv["ws"], hv["coder"]
    vol = torch.empty((z, h, w), dtype=_sample_dtype(model.depth), device=bits.device)
    st = torch.zeros(1, dtype=torch.int32, device=bits.device)
    wsb = dlic_volume_workspace(model, z, h, w, coder, 1)
    if wsb == 0:
        raise DlicError(DLIC_ERR_UNSUPPORTED, "dlic_volume_workspace")
    wsp = _empty(wsb, torch.uint8, bits.device)
    _check(lib().dlic_volume_decode(ctypes.byref(model.c), ctypes.byref(coder),
                                    _ptr(bits.contiguous()), bits.numel(), _ptr(vol), z, h, w, ws,
                                    _ptr(st), _ptr(wsp), wsb, _stream(stream)), "dlic_volume_decode")
    status = int(st.item())
    if check and status != DLIC_OK:
        raise DlicError(status, "dlic_volume_decode (device status)")
    return vol, status


def volume_density(vol, model: DeepModel, ws: int = 0, logits=True, tables=False, stream=None):
    """As deep_density for a [z, h, w] volume (slice-major raster order)."""
    import torch
    _check_samples(vol, model)
    z, h, w = vol.shape
    n, N = z * h * w, 1 << model.depth
    lg = torch.empty((n, N), dtype=torch.float32, device=vol.device) if logits else None
    cf = torch.empty(n, dtype=torch.int32, device=vol.device)
    tab = torch.empty((n, N), dtype=torch.int16, device=vol.device) if tables else None
    wsb = dlic_volume_workspace(model, z, h, w, None, -1)
    wsp = _empty(wsb, torch.uint8, vol.device)
    _check(lib().dlic_volume_density(ctypes.byref(model.c), _ptr(vol.contiguous()), z, h, w, ws,
                                     _ptr(lg) if lg is not None else None, _ptr(cf),
                                     _ptr(tab) if tab is not None else None, _ptr(wsp), wsb,
                                     _stream(stream)), "dlic_volume_density")
    return lg, cf, tab


# ---- retraining -------------------------------------------------------------------

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def dlic_nll_workspace(n: int, model: dlic_model) -> int:
    return int(lib().dlic_nll_workspace(int(n), ctypes.byref(model)))


def dlic_nll_fwd_bwd(model: dlic_model, d_slices, n_slices, sh, sw, d_idx, n, d_loss, d_grad,
                     d_ws, ws_bytes, stream=None):
    _check(lib().dlic_nll_fwd_bwd(ctypes.byref(model), _ptr(d_slices), n_slices, sh, sw,
                                  _ptr(d_idx), int(n), _ptr(d_loss), _ptr(d_grad), _ptr(d_ws),
                                  ws_bytes, _stream(stream)), "dlic_nll_fwd_bwd")


def dlic_adam_step(n_params, d_params, d_grad, d_m, d_v, step, lr=1e-3, b1=0.9, b2=0.999,
                   eps=1e-8, stream=None):
    _check(lib().dlic_adam_step(int(n_params), _ptr(d_params), _ptr(d_grad), _ptr(d_m), _ptr(d_v),
                                int(step), lr, b1, b2, eps, _stream(stream)), "dlic_adam_step")


def param_shapes(h1: int, h2: int):
    return {"W1": (h1, 12), "b1": (h1,), "W2": (h2, h1), "b2": (h2,), "W3": (15, h2), "b3": (15,)}


def _model_over(tensors, dtype_code, h1, h2):
    return dlic_model(12, h1, h2, 15, dtype_code, 0, _ptr(tensors["W1"]), _ptr(tensors["W2"]),
                      _ptr(tensors["W3"]), _ptr(tensors["b1"]), _ptr(tensors["b2"]),
                      _ptr(tensors["b3"]), None, 0)


class TrainModel:
    """Weights in one flat device buffer (FP32 or FP64) in the gradient layout."""

    def __init__(self, weights: dict, device="cuda", dtype=None):
        import torch
        dtype = dtype or torch.float32
        h1, h2 = weights["W1"].shape[0], weights["W2"].shape[0]
        self.h1, self.h2 = h1, h2
        flat = np.concatenate([np.asarray(weights[k], dtype=np.float64).ravel() for k in PARAM_NAMES])
        self.flat = torch.from_numpy(flat).to(device=device, dtype=dtype)
        self.views = {}
        off = 0
        for k, shp in param_shapes(h1, h2).items():
            n = int(np.prod(shp))
            self.views[k] = self.flat[off:off + n].view(*shp)
            off += n
        code = DLIC_FP64 if dtype == torch.float64 else DLIC_FP32
        self.c = _model_over(self.views, code, h1, h2)


def nll(model: TrainModel, slices, idx, want_grad=True, stream=None):
    """(loss, grad) of the mean mixture NLL in bits; grad is flat in the weight layout."""
    import torch
    n = idx.shape[0]
    ns, sh, sw = slices.shape
    loss = torch.zeros(1, dtype=model.flat.dtype, device=model.flat.device)
    grad = torch.empty_like(model.flat) if want_grad else None
    wsb = dlic_nll_workspace(n, model.c)
    ws = torch.empty(wsb, dtype=torch.uint8, device=model.flat.device)
    dlic_nll_fwd_bwd(model.c, slices.contiguous(), ns, sh, sw, idx.contiguous(), n, loss, grad, ws,
                     wsb, stream)
    return loss, grad


def _autograd_fn():
    import torch

    class DLICNLL(torch.autograd.Function):
        """Mean mixture NLL (bits) with the hand-written backward kernel.

        forward(W1, b1, W2, b2, W3, b3, slices, idx) -> scalar loss.  The
        gradient is computed together with the loss by dlic_nll_fwd_bwd and
        scaled by the incoming gradient in backward.
        """

        @staticmethod
        def forward(ctx, W1, b1, W2, b2, W3, b3, slices, idx):
            tensors = {"W1": W1.contiguous(), "b1": b1.contiguous(), "W2": W2.contiguous(),
                       "b2": b2.contiguous(), "W3": W3.contiguous(), "b3": b3.contiguous()}
            code = DLIC_FP64 if W1.dtype == torch.float64 else DLIC_FP32
            m = _model_over(tensors, code, W1.shape[0], W2.shape[0])
            n = idx.shape[0]
            ns, sh, sw = slices.shape
            loss = torch.zeros(1, dtype=W1.dtype, device=W1.device)
            grad = torch.empty(sum(t.numel() for t in tensors.values()), dtype=W1.dtype,
                               device=W1.device)
            wsb = dlic_nll_workspace(n, m)
            ws = torch.empty(wsb, dtype=torch.uint8, device=W1.device)
            dlic_nll_fwd_bwd(m, slices.contiguous(), ns, sh, sw, idx.contiguous(), n, loss, grad,
                             ws, wsb)
            ctx.save_for_backward(grad)
            ctx.shapes = [t.shape for t in tensors.values()]
            return loss[0]

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            outs, off = [], 0
            for shp in ctx.shapes:
                n = int(np.prod(shp))
                outs.append((grad[off:off + n] * g).view(shp))
                off += n
            return (*outs, None, None)

    return DLICNLL


_DLICNLL = None


def DLICNLL():
    """The torch.autograd.Function class for the hand-written NLL backward."""
    global _DLICNLL
    if _DLICNLL is None:
        _DLICNLL = _autograd_fn()
    return _DLICNLL


# ---- batches ----------------------------------------------------------------------

def dlic_batch_create(model: dlic_model, sizes, coders=None, density_grid: int = 0) -> int:
    hw = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32).reshape(-1, 2))
    n = hw.shape[0]
    cd = None
    if coders is not None:
        cd = (dlic_coder * n)(*[dlic_coder(int(g), int(l)) for g, l in coders])
    out = c_void_p()
    _check(lib().dlic_batch_create(ctypes.byref(model), n, hw.ctypes.data, cd, density_grid,
                                   ctypes.byref(out)), "dlic_batch_create")
    return out.value


def dlic_batch_tune(b: int, search_lanes: int = 0, decode_grid: int = 0):
    _check(lib().dlic_batch_tune(b, int(search_lanes), int(decode_grid)), "dlic_batch_tune")


def dlic_batch_destroy(b: int):
    lib().dlic_batch_destroy(b)


def dlic_batch_sizes(b: int) -> dict:
    px, ob, ws, ni = c_size_t(), c_size_t(), c_size_t(), c_int32()
    _check(lib().dlic_batch_sizes(b, ctypes.byref(px), ctypes.byref(ob), ctypes.byref(ws),
                                  ctypes.byref(ni)), "dlic_batch_sizes")
    return dict(pixels=px.value, out_bytes=ob.value, ws_bytes=ws.value, n_items=ni.value)


def dlic_batch_layout(b: int, n_img: int):
    px = np.zeros(n_img, np.uint64)
    ob = np.zeros(n_img, np.uint64)
    cd = np.zeros((n_img, 2), np.int32)
    _check(lib().dlic_batch_layout(b, px.ctypes.data, ob.ctypes.data, cd.ctypes.data),
           "dlic_batch_layout")
    return px, ob, cd


def dlic_encode_batch(b, d_pixels, d_out, d_out_len, d_t_done, d_ws, ws_bytes, stream=None):
    _check(lib().dlic_encode_batch(b, _ptr(d_pixels), _ptr(d_out), _ptr(d_out_len), _ptr(d_t_done),
                                   _ptr(d_ws), ws_bytes, _stream(stream)), "dlic_encode_batch")


def dlic_decode_batch(b, d_bits, d_len, d_pixels, d_status, d_t_done, d_ws, ws_bytes, stream=None):
    _check(lib().dlic_decode_batch(b, _ptr(d_bits), _ptr(d_len), _ptr(d_pixels), _ptr(d_status),
                                   _ptr(d_t_done), _ptr(d_ws), ws_bytes, _stream(stream)),
           "dlic_decode_batch")


def dlic_batch_capture(b, decode, d_in, d_out, d_len, d_status, d_t_done, d_ws, ws_bytes):
    _check(lib().dlic_batch_capture(b, int(decode), _ptr(d_in), _ptr(d_out), _ptr(d_len),
                                    _ptr(d_status), _ptr(d_t_done), _ptr(d_ws), ws_bytes),
           "dlic_batch_capture")


def dlic_batch_replay(b, decode, stream=None):
    _check(lib().dlic_batch_replay(b, int(decode), _stream(stream)), "dlic_batch_replay")


def dlic_wallclock_hz() -> float:
    return float(lib().dlic_wallclock_hz())


PROBE_NAMES = ("fma_f32", "mfma_4x4x1_f32", "mfma_16x16x4_f32", "lds_store_load", "lds_load",
               "lds_flag_handoff", "dpp_reduce16", "expf", "rans_update", "ballot_popcount",
               "global_flag_handoff", "readlane")


def dlic_latency_probe(stream=None) -> dict:
    """Shader cycles per link of each primitive's dependent chain, and the shader clock."""
    import torch
    out = (ctypes.c_double * 13)()
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    _check(lib().dlic_latency_probe(out, 13, _ptr(ws), 256, _stream(stream)), "dlic_latency_probe")
    res = {n: float(out[i]) for i, n in enumerate(PROBE_NAMES)}
    res["shader_clock_mhz"] = float(out[12])
    return res


class Batch:
    """A batch plan with its torch-allocated buffers: images in, streams,
    decoded images out, lengths, statuses, completion stamps, workspace."""

    def __init__(self, model: Model, sizes, coders=None, density_grid: int = 0, device="cuda",
                 search_lanes: int = 0, decode_grid: int = 0):
        import torch
        self.model = model  # keeps the weights alive for the plan
        self.sizes = [(int(h), int(w)) for h, w in sizes]
        self.n = len(self.sizes)
        self.plan = dlic_batch_create(model.c, self.sizes, coders, density_grid)
        if search_lanes or decode_grid:
            try:
                dlic_batch_tune(self.plan, search_lanes, decode_grid)
            except DlicError:
                self.close()
                raise
        sz = dlic_batch_sizes(self.plan)
        self.n_items = sz["n_items"]
        self.px_off, self.out_off, self.coders = dlic_batch_layout(self.plan, self.n)
        self.n_pixels = sz["pixels"]
        self.pixels = torch.zeros(max(sz["pixels"], 1), dtype=torch.uint8, device=device)
        self.decoded = torch.zeros_like(self.pixels)
        self.out = torch.zeros(max(sz["out_bytes"], 1), dtype=torch.uint8, device=device)
        self.lens = torch.zeros(self.n, dtype=torch.int64, device=device)
        self.status = torch.zeros(self.n, dtype=torch.int32, device=device)
        self.t_enc = torch.zeros(self.n + 1, dtype=torch.int64, device=device)
        self.t_dec = torch.zeros(self.n + 1, dtype=torch.int64, device=device)
        self.ws_bytes = sz["ws_bytes"]
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)

    def load(self, images):
        """Copy [h, w] uint8 images (numpy or torch) into the pixel buffer."""
        import torch
        for i, im in enumerate(images):
            t = im if isinstance(im, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(im))
            o = int(self.px_off[i])
            self.pixels[o:o + t.numel()].copy_(t.reshape(-1))

    def image(self, i, decoded=True):
        h, w = self.sizes[i]
        o = int(self.px_off[i])
        return (self.decoded if decoded else self.pixels)[o:o + h * w].view(h, w)

    def intervals(self, i):
        """Packed intervals c | (f - 1) << 16 of image i from the last encode ([h, w] int32)."""
        import torch
        h, w = self.sizes[i]
        o = int(self.px_off[i])
        return self.ws[:4 * self.n_pixels].view(torch.int32)[o:o + h * w].view(h, w)

    def stream(self, i):
        o = int(self.out_off[i])
        return self.out[o:o + int(self.lens[i].item())]

    def encode(self, stream=None):
        dlic_encode_batch(self.plan, self.pixels, self.out, self.lens, self.t_enc, self.ws,
                          self.ws_bytes, stream)

    def decode(self, stream=None):
        dlic_decode_batch(self.plan, self.out, self.lens, self.decoded, self.status, self.t_dec,
                          self.ws, self.ws_bytes, stream)

    def capture(self):
        dlic_batch_capture(self.plan, 0, self.pixels, self.out, self.lens, None, self.t_enc,
                           self.ws, self.ws_bytes)
        dlic_batch_capture(self.plan, 1, self.out, self.decoded, self.lens, self.status, self.t_dec,
                           self.ws, self.ws_bytes)

    def replay(self, decode: bool, stream=None):
        dlic_batch_replay(self.plan, decode, stream)

    def latencies_s(self, decode: bool) -> np.ndarray:
        """Per-image completion time since the start of the last call (seconds)."""
        t = (self.t_dec if decode else self.t_enc).cpu().numpy().astype(np.float64)
        return (t[:self.n] - t[self.n]) / dlic_wallclock_hz()

    def close(self):
        if self.plan:
            dlic_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
