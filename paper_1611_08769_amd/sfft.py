"""ctypes binding of libsfft (include/sfft.h): same names, argument
marshalling only.  Every computation runs in the library; if the library is
not built this module raises on import."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfft.so")

SFFT_OK = 0
SFFT_EINVAL = -1
SFFT_ENOMEM = -2
SFFT_EDEVICE = -3
SFFT_ENOISE = -4
SFFT_EUNSUPPORTED = -6

GATE_NOT, GATE_AND, GATE_XOR, GATE_OR, GATE_XADD, GATE_NAND, GATE_PRODUCT = 3, 4, 5, 6, 7, 8, 9


class sfft_params(ctypes.Structure):
    _fields_ = [("n_lwe", ctypes.c_int32), ("k", ctypes.c_int32), ("m", ctypes.c_int32), ("eta", ctypes.c_int32)]


class sfft_shape(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("len", ctypes.c_int32), ("F", ctypes.c_int32), ("f", ctypes.c_int32),
                ("is_complex", ctypes.c_int32), ("nand_only", ctypes.c_int32)]


class sfft_plan_info(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("gates", ctypes.c_int64), ("products", ctypes.c_int64),
                ("exec_products", ctypes.c_int64), ("levels", ctypes.c_int64),
                ("max_level_products", ctypes.c_int64), ("n_inputs", ctypes.c_int64),
                ("n_outputs", ctypes.c_int64), ("ws_cts", ctypes.c_int64), ("exec_steps", ctypes.c_int64),
                ("k_required", ctypes.c_int32),
                ("netlist_sha256", ctypes.c_char * 65), ("tiling", ctypes.c_int32),
                ("prod_ct_reads", ctypes.c_int64), ("prod_ct_writes", ctypes.c_int64), ("ws_bytes", ctypes.c_int64),
                ("noise_bound_bits", ctypes.c_int32)]


SFFT_SERVER_DRYRUN = 1
SFFT_SERVER_SERIAL = 2
SFFT_NOALLOC_WS_BYTES = 64 << 20


class sfft_server_cfg(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("dry_bitmac_per_s", ctypes.c_double), ("fill_blocks", ctypes.c_int64)]


class sfft_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "admitted", "completed", "queued", "active", "steps",
                                              "launches", "products", "gates", "fft_points", "max_active",
                                              "peak_ws_bytes")] + [("clock_s", ctypes.c_double)]


class sfft_ring_plan_info(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("gates", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("calls", ctypes.c_int32), ("max_batch", ctypes.c_int64), ("n_inputs", ctypes.c_int64),
                ("n_outputs", ctypes.c_int64), ("ws_bytes", ctypes.c_int64)]


class SfftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sfft error %d: %s" % (code, msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("libsfft.so is not built (run paper_1611_08769_amd.build.build())")

# One HIP runtime per process: torch ships its own copy of the HIP and HSA
# runtimes under the same sonames as ROCm's.  Loading torch first makes the
# library bind to the copy already in the process; loading the library
# first would bring in a second pair of runtimes, and the one initialised
# second finds no device.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_P = ctypes.POINTER

_SIGS = {
    "sfft_last_error": (ctypes.c_char_p, []),
    "sfft_size_params": (ctypes.c_int, [_P(sfft_shape), ctypes.c_int32, _P(sfft_params)]),
    "sfft_ct_bytes": (ctypes.c_int64, [_P(sfft_params)]),
    "sfft_keygen": (ctypes.c_int, [_P(sfft_params), ctypes.c_uint64, _vp, _vp]),
    "sfft_encrypt": (ctypes.c_int, [_P(sfft_params), _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                    ctypes.c_uint64, _vp, _vp]),
    "sfft_plan_create": (ctypes.c_int, [_P(sfft_shape), _P(sfft_params), _P(_vp)]),
    "sfft_plan_info_get": (ctypes.c_int, [_vp, _P(sfft_plan_info)]),
    "sfft_analyze": (ctypes.c_int, [_P(sfft_shape), _P(sfft_params), _P(sfft_plan_info)]),
    "sfft_analyze_bounded": (ctypes.c_int, [_P(sfft_shape), _P(sfft_params), ctypes.c_int64, _P(sfft_plan_info)]),
    "sfft_plan_create_bounded": (ctypes.c_int, [_P(sfft_shape), _P(sfft_params), ctypes.c_int64, _P(_vp)]),
    "sfft_plan_workspace_bytes": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "sfft_plan_destroy": (None, [_vp]),
    "sfft_execute": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "sfft_execute_steps": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "sfft_plan_step_products": (ctypes.c_int, [_vp, _P(ctypes.c_int64), ctypes.c_int32]),
    "sfft_plan_time_products": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "sfft_execute_persistent": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "sfft_plan_persistent_timeouts": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
    "sfft_batch_workspace_bytes": (ctypes.c_int, [_P(_vp), ctypes.c_int32, _P(ctypes.c_int64)]),
    "sfft_batch_create": (ctypes.c_int, [_P(_vp), _P(_vp), _P(_vp), ctypes.c_int32, _vp, ctypes.c_int64, _P(_vp)]),
    "sfft_batch_info": (ctypes.c_int, [_vp, _P(ctypes.c_int64), _P(ctypes.c_int64)]),
    "sfft_batch_execute": (ctypes.c_int, [_vp, _vp]),
    "sfft_batch_execute_graph": (ctypes.c_int, [_vp, _vp]),
    "sfft_batch_destroy": (None, [_vp]),
    "sfft_plan_product_time": (ctypes.c_int, [_vp, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "sfft_decrypt": (ctypes.c_int, [_P(sfft_params), _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, _vp]),
    "sfft_decrypt_bits": (ctypes.c_int, [_P(sfft_params), _vp, _vp, ctypes.c_int64, ctypes.c_int, _vp]),
    "sfft_decrypt_stream": (ctypes.c_int, [_P(sfft_params), _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp]),
    "sfft_noise_bits": (ctypes.c_int, [_P(sfft_params), _vp, _vp, ctypes.c_int64, _vp, _vp, _P(ctypes.c_int32)]),
    "sfft_gate": (ctypes.c_int, [_P(sfft_params), ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "sfft_server_create": (ctypes.c_int, [_P(sfft_server_cfg), _P(_vp)]),
    "sfft_server_submit": (ctypes.c_int, [_vp, _P(sfft_shape), _P(sfft_params), _vp, _vp, _P(ctypes.c_uint64)]),
    "sfft_server_submit_plan": (ctypes.c_int, [_vp, _vp, _vp, _vp, _P(ctypes.c_uint64)]),
    "sfft_execute_graph": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "sfft_execute_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "sfft_tiling_count": (ctypes.c_int, []),
    "sfft_tiling_describe": (ctypes.c_int, [ctypes.c_int32, _P(ctypes.c_int32)]),
    "sfft_set_tiling": (ctypes.c_int, [_P(sfft_params), ctypes.c_int32]),
    "sfft_tune": (ctypes.c_int, [_P(sfft_params), ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_double), _vp]),
    "sfft_plan_tune": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _P(ctypes.c_int32),
                                      _P(ctypes.c_double), _vp]),
    "sfft_server_step": (ctypes.c_int, [_vp, _vp, _P(ctypes.c_int32)]),
    "sfft_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(ctypes.c_int32), _P(ctypes.c_double)]),
    "sfft_server_drain": (ctypes.c_int, [_vp, _vp]),
    "sfft_server_stats_get": (ctypes.c_int, [_vp, _P(sfft_server_stats)]),
    "sfft_server_destroy": (None, [_vp]),
    "sfft_ring_ct_words": (ctypes.c_int64, [ctypes.c_int32]),
    "sfft_ring_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _P(ctypes.c_int64)]),
    "sfft_ring_encrypt": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp]),
    "sfft_ring_gate": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64, _vp,
                                      ctypes.c_int64, _vp]),
    "sfft_ring_decrypt": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, ctypes.c_int64, ctypes.c_int, _vp]),
    "sfft_ring_bk_prepare": (ctypes.c_int, [ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]),
    "sfft_ring_blind_rotate": (ctypes.c_int, [ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp]),
    "sfft_ring_bootstrap_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                           _P(ctypes.c_int64)]),
    "sfft_ring_bootstrap": (ctypes.c_int, [ctypes.c_int32, _vp, ctypes.c_int64, _vp, ctypes.c_int64, _vp, _vp,
                                           ctypes.c_int64, _vp]),
    "sfft_ring_keyswitch": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp, _vp]),
    "sfft_ring_plan_analyze": (ctypes.c_int, [_P(sfft_shape), ctypes.c_int32, ctypes.c_int64, _P(sfft_ring_plan_info)]),
    "sfft_ring_plan_create": (ctypes.c_int, [_P(sfft_shape), ctypes.c_int32, ctypes.c_int64, _P(_vp)]),
    "sfft_ring_fft_execute": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "sfft_ring_plan_destroy": (None, [_vp]),
    "sfft_ring_gate_bootstrap_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                                _P(ctypes.c_int64)]),
    "sfft_ring_gate_bootstrap": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp, _vp,
                                                ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def last_error() -> str:
    return _lib.sfft_last_error().decode()


def _check(rc):
    if rc != SFFT_OK:
        raise SfftError(rc, last_error())


def params(n_lwe: int, k: int) -> sfft_params:
    return sfft_params(n_lwe, k, (n_lwe + 1) * k, 1)


def shape(dims: int, length: int, F: int, f: int, is_complex: bool, nand_only: bool = False) -> sfft_shape:
    return sfft_shape(dims, length, F, f, int(bool(is_complex)), int(bool(nand_only)))


def sfft_size_params(shp: sfft_shape, n_lwe: int) -> sfft_params:
    out = sfft_params()
    _check(_lib.sfft_size_params(ctypes.byref(shp), n_lwe, ctypes.byref(out)))
    return out


def sfft_ct_bytes(p: sfft_params) -> int:
    v = _lib.sfft_ct_bytes(ctypes.byref(p))
    if v < 0:
        raise SfftError(v, last_error())
    return v


def sfft_keygen(p: sfft_params, seed: int, pk_host_ptr: int, sk_host_ptr: int) -> None:
    _check(_lib.sfft_keygen(ctypes.byref(p), seed, pk_host_ptr, sk_host_ptr))


def sfft_encrypt(p, pk_dev_ptr, fixed_host_ptr, n_values, F, seed, first_ct_id, ct_dev_ptr, stream) -> None:
    _check(_lib.sfft_encrypt(ctypes.byref(p), pk_dev_ptr, fixed_host_ptr, n_values, F, seed, first_ct_id,
                             ct_dev_ptr, stream))


def sfft_plan_create(shp: sfft_shape, p: sfft_params) -> int:
    h = _vp()
    _check(_lib.sfft_plan_create(ctypes.byref(shp), ctypes.byref(p), ctypes.byref(h)))
    return h.value


def sfft_plan_create_bounded(shp: sfft_shape, p: sfft_params, ws_limit_bytes: int) -> int:
    h = _vp()
    _check(_lib.sfft_plan_create_bounded(ctypes.byref(shp), ctypes.byref(p), int(ws_limit_bytes), ctypes.byref(h)))
    return h.value


def sfft_analyze_bounded(shp: sfft_shape, p: sfft_params, ws_limit_bytes: int) -> sfft_plan_info:
    info = sfft_plan_info()
    _check(_lib.sfft_analyze_bounded(ctypes.byref(shp), ctypes.byref(p), int(ws_limit_bytes), ctypes.byref(info)))
    return info


def sfft_plan_info_get(plan: int) -> sfft_plan_info:
    info = sfft_plan_info()
    _check(_lib.sfft_plan_info_get(plan, ctypes.byref(info)))
    return info


def sfft_analyze(shp: sfft_shape, p: sfft_params) -> sfft_plan_info:
    info = sfft_plan_info()
    _check(_lib.sfft_analyze(ctypes.byref(shp), ctypes.byref(p), ctypes.byref(info)))
    return info


def sfft_plan_workspace_bytes(plan: int) -> int:
    v = ctypes.c_int64()
    _check(_lib.sfft_plan_workspace_bytes(plan, ctypes.byref(v)))
    return v.value


def sfft_plan_destroy(plan: int) -> None:
    _lib.sfft_plan_destroy(plan)


def sfft_execute(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_execute(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream))


def sfft_execute_noalloc(plan, ct_in_ptr, ct_out_ptr, stream) -> None:
    _check(_lib.sfft_execute_noalloc(plan, ct_in_ptr, ct_out_ptr, stream))


def sfft_execute_steps(plan, first, count, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_execute_steps(plan, first, count, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream))


def sfft_execute_persistent(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_execute_persistent(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream))


def sfft_plan_persistent_timeouts(plan) -> int:
    v = ctypes.c_int32()
    _check(_lib.sfft_plan_persistent_timeouts(plan, ctypes.byref(v)))
    return v.value


def _ptr_array(ptrs):
    return (_vp * len(ptrs))(*ptrs)


def sfft_batch_workspace_bytes(plans) -> int:
    v = ctypes.c_int64()
    _check(_lib.sfft_batch_workspace_bytes(_ptr_array(plans), len(plans), ctypes.byref(v)))
    return v.value


def sfft_batch_create(plans, ins, outs, ws_ptr, ws_bytes) -> int:
    h = _vp()
    _check(_lib.sfft_batch_create(_ptr_array(plans), _ptr_array(ins), _ptr_array(outs), len(plans), ws_ptr, ws_bytes,
                                  ctypes.byref(h)))
    return h.value


def sfft_batch_info(batch):
    st, la = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.sfft_batch_info(batch, ctypes.byref(st), ctypes.byref(la)))
    return st.value, la.value


def sfft_batch_execute(batch, stream) -> None:
    _check(_lib.sfft_batch_execute(batch, stream))


def sfft_batch_execute_graph(batch, stream) -> None:
    _check(_lib.sfft_batch_execute_graph(batch, stream))


def sfft_batch_destroy(batch) -> None:
    _lib.sfft_batch_destroy(batch)


def sfft_plan_time_products(plan, enable) -> None:
    _check(_lib.sfft_plan_time_products(plan, int(enable)))


def sfft_plan_product_time(plan):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.sfft_plan_product_time(plan, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def sfft_plan_step_products(plan, n):
    arr = (ctypes.c_int64 * n)()
    _check(_lib.sfft_plan_step_products(plan, arr, n))
    return list(arr)


def sfft_decrypt_stream(p, sk_host_ptr, ct_dev_ptr, n_values, F, stream, out_ptr) -> None:
    _check(_lib.sfft_decrypt_stream(ctypes.byref(p), sk_host_ptr, ct_dev_ptr, n_values, F, stream, out_ptr))


def sfft_noise_bits(p, sk_host_ptr, ct_dev_ptr, n_ct, mu_bits_ptr, stream) -> int:
    v = ctypes.c_int32()
    _check(_lib.sfft_noise_bits(ctypes.byref(p), sk_host_ptr, ct_dev_ptr, n_ct, mu_bits_ptr, stream, ctypes.byref(v)))
    return v.value


def sfft_decrypt(p, sk_host_ptr, ct_ptr, n_values, F, on_device, out_ptr) -> None:
    _check(_lib.sfft_decrypt(ctypes.byref(p), sk_host_ptr, ct_ptr, n_values, F, int(on_device), out_ptr))


def sfft_decrypt_bits(p, sk_host_ptr, ct_ptr, n_ct, on_device, out_ptr) -> None:
    _check(_lib.sfft_decrypt_bits(ctypes.byref(p), sk_host_ptr, ct_ptr, n_ct, int(on_device), out_ptr))


def sfft_gate(p, gate, x_ptr, y_ptr, out_ptr, stream) -> None:
    _check(_lib.sfft_gate(ctypes.byref(p), gate, x_ptr, y_ptr, out_ptr, stream))


def sfft_server_create(cfg: sfft_server_cfg) -> int:
    h = _vp()
    _check(_lib.sfft_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def sfft_server_submit(srv, shp, p, ct_in_ptr, ct_out_ptr) -> int:
    t = ctypes.c_uint64()
    _check(_lib.sfft_server_submit(srv, ctypes.byref(shp), ctypes.byref(p), ct_in_ptr, ct_out_ptr, ctypes.byref(t)))
    return t.value


def sfft_server_submit_plan(srv, plan, ct_in_ptr, ct_out_ptr) -> int:
    t = ctypes.c_uint64()
    _check(_lib.sfft_server_submit_plan(srv, plan, ct_in_ptr, ct_out_ptr, ctypes.byref(t)))
    return t.value


def sfft_tiling_count() -> int:
    return _lib.sfft_tiling_count()


def sfft_tiling_describe(tiling: int):
    f = (ctypes.c_int32 * 7)()
    _check(_lib.sfft_tiling_describe(tiling, f))
    return tuple(f)


def sfft_set_tiling(p, tiling: int) -> None:
    _check(_lib.sfft_set_tiling(ctypes.byref(p), tiling))


def sfft_tune(p, reps, stream):
    best = ctypes.c_int32()
    rates = (ctypes.c_double * sfft_tiling_count())()
    _check(_lib.sfft_tune(ctypes.byref(p), reps, ctypes.byref(best), rates, stream))
    return best.value, list(rates)


def sfft_plan_tune(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, reps, stream):
    best = ctypes.c_int32()
    rates = (ctypes.c_double * sfft_tiling_count())()
    _check(_lib.sfft_plan_tune(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, reps, ctypes.byref(best), rates, stream))
    return best.value, list(rates)


def sfft_execute_graph(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_execute_graph(plan, ct_in_ptr, ct_out_ptr, ws_ptr, ws_bytes, stream))


def sfft_server_step(srv, stream) -> int:
    pend = ctypes.c_int32()
    _check(_lib.sfft_server_step(srv, stream, ctypes.byref(pend)))
    return pend.value


def sfft_server_poll(srv, ticket):
    done, lat = ctypes.c_int32(), ctypes.c_double()
    _check(_lib.sfft_server_poll(srv, ticket, ctypes.byref(done), ctypes.byref(lat)))
    return bool(done.value), lat.value


def sfft_server_drain(srv, stream) -> None:
    _check(_lib.sfft_server_drain(srv, stream))


def sfft_server_stats_get(srv) -> sfft_server_stats:
    st = sfft_server_stats()
    _check(_lib.sfft_server_stats_get(srv, ctypes.byref(st)))
    return st


def sfft_server_destroy(srv) -> None:
    _lib.sfft_server_destroy(srv)


EXPORTED = sorted(_SIGS)


# ---- ring-GSW gates --------------------------------------------------------
SFFT_RING_P = 0x3FFFFFFFFFFF0001
SFFT_RING_ELL = 62


def sfft_ring_ct_words(d: int) -> int:
    w = _lib.sfft_ring_ct_words(d)
    if w < 0:
        raise SfftError(int(w), last_error())
    return w


def sfft_ring_workspace_bytes(d: int, n: int) -> int:
    b = ctypes.c_int64()
    _check(_lib.sfft_ring_workspace_bytes(d, n, ctypes.byref(b)))
    return b.value


def sfft_ring_encrypt(d, s_dev_ptr, a_dev_ptr, e_dev_ptr, bits_dev_ptr, n, ct_dev_ptr, stream) -> None:
    _check(_lib.sfft_ring_encrypt(d, s_dev_ptr, a_dev_ptr, e_dev_ptr, bits_dev_ptr, n, ct_dev_ptr, stream))


def sfft_ring_gate(d, gate, x_ptr, y_ptr, out_ptr, n, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_ring_gate(d, gate, x_ptr, y_ptr, out_ptr, n, ws_ptr, ws_bytes, stream))


def sfft_ring_decrypt(d, s_host_ptr, ct_ptr, n, on_device, bits_out_ptr) -> None:
    _check(_lib.sfft_ring_decrypt(d, s_host_ptr, ct_ptr, n, int(on_device), bits_out_ptr))


def sfft_ring_bk_prepare(d, bk_ptr, n, bkt_ptr, stream) -> None:
    _check(_lib.sfft_ring_bk_prepare(d, bk_ptr, n, bkt_ptr, stream))


def sfft_ring_blind_rotate(d, bkt_ptr, n, rot_ptr, acc_ptr, m, stream) -> None:
    _check(_lib.sfft_ring_blind_rotate(d, bkt_ptr, n, rot_ptr, acc_ptr, m, stream))


def sfft_ring_bootstrap_workspace_bytes(d: int, n: int, m: int) -> int:
    b = ctypes.c_int64()
    _check(_lib.sfft_ring_bootstrap_workspace_bytes(d, n, m, ctypes.byref(b)))
    return b.value


def sfft_ring_bootstrap(d, bkt_ptr, n, lwe_ptr, m, out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_ring_bootstrap(d, bkt_ptr, n, lwe_ptr, m, out_ptr, ws_ptr, ws_bytes, stream))


def sfft_ring_keyswitch(d, n, ksk_ptr, in_ptr, m, out_ptr, stream) -> None:
    _check(_lib.sfft_ring_keyswitch(d, n, ksk_ptr, in_ptr, m, out_ptr, stream))


def sfft_ring_gate_bootstrap_workspace_bytes(d: int, n: int, m: int) -> int:
    b = ctypes.c_int64()
    _check(_lib.sfft_ring_gate_bootstrap_workspace_bytes(d, n, m, ctypes.byref(b)))
    return b.value


def sfft_ring_gate_bootstrap(d, gate, bkt_ptr, n, ksk_ptr, x_ptr, y_ptr, m, out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_ring_gate_bootstrap(d, gate, bkt_ptr, n, ksk_ptr, x_ptr, y_ptr, m, out_ptr, ws_ptr, ws_bytes,
                                         stream))


def sfft_ring_plan_analyze(shp: sfft_shape, d: int, n: int) -> sfft_ring_plan_info:
    info = sfft_ring_plan_info()
    _check(_lib.sfft_ring_plan_analyze(ctypes.byref(shp), d, n, ctypes.byref(info)))
    return info


def sfft_ring_plan_create(shp: sfft_shape, d: int, n: int) -> int:
    h = _vp()
    _check(_lib.sfft_ring_plan_create(ctypes.byref(shp), d, n, ctypes.byref(h)))
    return h.value


def sfft_ring_fft_execute(plan, bkt_ptr, ksk_ptr, in_ptr, out_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(_lib.sfft_ring_fft_execute(plan, bkt_ptr, ksk_ptr, in_ptr, out_ptr, ws_ptr, ws_bytes, stream))


def sfft_ring_plan_destroy(plan) -> None:
    _lib.sfft_ring_plan_destroy(plan)
