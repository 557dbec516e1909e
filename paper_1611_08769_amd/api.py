"""Python front end: keys, encryption, plans and decryption over libsfft with
device memory owned by torch tensors.  Argument marshalling only -- every
ciphertext operation runs in the HIP library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import sfft as S


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def quantize(x, F: int, f: int) -> np.ndarray:
    """Real -> Q(F, f) by truncation (floor(x * 2^f)); must fit F bits."""
    q = np.floor(np.asarray(x, dtype=np.float64) * float(1 << f)).astype(np.int64)
    if np.any(q < -(1 << (F - 1))) or np.any(q >= (1 << (F - 1))):
        raise ValueError("value does not fit Q(%d,%d)" % (F, f))
    return q


@dataclass
class Keys:
    params: S.sfft_params
    pk_host: np.ndarray      # uint32, ct_words
    sk_host: np.ndarray      # uint32, (n+1)*k/32
    pk_dev: torch.Tensor     # int32 view of the same words, on the GPU

    @property
    def ct_words(self) -> int:
        return S.sfft_ct_bytes(self.params) // 4


def keygen(params: S.sfft_params, seed: int, device="cuda") -> Keys:
    cw = S.sfft_ct_bytes(params) // 4
    pk = np.zeros(cw, dtype=np.uint32)
    sk = np.zeros((params.n_lwe + 1) * params.k // 32, dtype=np.uint32)
    S.sfft_keygen(params, seed, pk.ctypes.data, sk.ctypes.data)
    pk_dev = torch.from_numpy(pk.view(np.int32)).to(device)
    return Keys(params, pk, sk, pk_dev)


def alloc_cts(keys_or_params, n: int, device="cuda") -> torch.Tensor:
    p = keys_or_params.params if isinstance(keys_or_params, Keys) else keys_or_params
    cw = S.sfft_ct_bytes(p) // 4
    return torch.empty((n, cw), dtype=torch.int32, device=device)


def encrypt_words(keys: Keys, words, F: int, seed: int, first_ct_id: int = 0, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """F ciphertexts per word (LSB first) on the GPU."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.int64).astype(np.int32).ravel())
    n_ct = w.size * F
    if out is None:
        out = alloc_cts(keys, n_ct)
    assert out.shape[0] >= n_ct and out.is_contiguous()
    S.sfft_encrypt(keys.params, keys.pk_dev.data_ptr(), w.ctypes.data, w.size, F, seed, first_ct_id,
                   out.data_ptr(), _stream_ptr(stream))
    return out


def decrypt_words(keys: Keys, cts: torch.Tensor, n_values: int, F: int, stream=None) -> np.ndarray:
    """Decrypted words.  Without a stream the whole device is synchronised
    first; with one, only that stream carries the copy (the caller makes sure
    the ciphertexts are complete)."""
    out = np.zeros(n_values, dtype=np.int32)
    if stream is None:
        torch.cuda.synchronize()
        S.sfft_decrypt(keys.params, keys.sk_host.ctypes.data, cts.data_ptr(), n_values, F, 1, out.ctypes.data)
    else:
        S.sfft_decrypt_stream(keys.params, keys.sk_host.ctypes.data, cts.data_ptr(), n_values, F,
                              _stream_ptr(stream), out.ctypes.data)
    return out.astype(np.int64)


def decrypt_bits(keys: Keys, cts: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    n = cts.shape[0]
    out = np.zeros(n, dtype=np.int32)
    S.sfft_decrypt_bits(keys.params, keys.sk_host.ctypes.data, cts.data_ptr(), n, 1, out.ctypes.data)
    return out


def gate(keys_or_params, g: int, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    p = keys_or_params.params if isinstance(keys_or_params, Keys) else keys_or_params
    out = torch.empty_like(x)
    S.sfft_gate(p, g, x.data_ptr(), (y if y is not None else x).data_ptr(), out.data_ptr(), _stream_ptr(stream))
    return out


class Plan:
    """A compiled encrypted FFT for one shape and parameter set."""

    def __init__(self, dims: int, length: int, F: int, f: int, is_complex: bool, params: S.sfft_params,
                 nand_only: bool = False, ws_limit_bytes: int = 0):
        """ws_limit_bytes > 0 bounds the plan's workspace (levels by list
        scheduling within it, sfft_plan_create_bounded)."""
        self.shape = S.shape(dims, length, F, f, is_complex, nand_only)
        self.params = params
        self.handle = (S.sfft_plan_create_bounded(self.shape, params, ws_limit_bytes) if ws_limit_bytes > 0
                       else S.sfft_plan_create(self.shape, params))
        self.info = S.sfft_plan_info_get(self.handle)
        self.ws_bytes = S.sfft_plan_workspace_bytes(self.handle)
        self.ct_words = S.sfft_ct_bytes(params) // 4
        self._ws = None

    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            self._ws = torch.empty(max(1, self.ws_bytes // 4), dtype=torch.int32, device="cuda")
        return self._ws

    def execute(self, ct_in: torch.Tensor, ct_out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if ct_out is None:
            ct_out = torch.empty((self.info.n_outputs, self.ct_words), dtype=torch.int32, device="cuda")
        assert ct_in.shape[0] >= self.info.n_inputs and ct_out.shape[0] >= self.info.n_outputs
        ws = self.workspace()
        S.sfft_execute(self.handle, ct_in.data_ptr(), ct_out.data_ptr(), ws.data_ptr(), ws.numel() * 4,
                       _stream_ptr(stream))
        return ct_out

    def execute_steps(self, first: int, count: int, ct_in: torch.Tensor, ct_out: torch.Tensor, stream=None):
        ws = self.workspace()
        S.sfft_execute_steps(self.handle, first, count, ct_in.data_ptr(), ct_out.data_ptr(), ws.data_ptr(),
                             ws.numel() * 4, _stream_ptr(stream))

    def execute_persistent(self, ct_in: torch.Tensor, ct_out: torch.Tensor | None = None, stream=None):
        """execute() in one persistent launch (small plans)."""
        if ct_out is None:
            ct_out = torch.empty((self.info.n_outputs, self.ct_words), dtype=torch.int32, device="cuda")
        ws = self.workspace()
        S.sfft_execute_persistent(self.handle, ct_in.data_ptr(), ct_out.data_ptr(), ws.data_ptr(), ws.numel() * 4,
                                  _stream_ptr(stream))
        return ct_out

    def time_products(self, enable: bool) -> None:
        """Record HIP events around each level's product kernel in later
        execute / execute_steps calls (product_time() collects them)."""
        S.sfft_plan_time_products(self.handle, enable)

    def product_time(self):
        """(total ms, launches) of the product kernels timed since the last
        call; waits for them."""
        return S.sfft_plan_product_time(self.handle)

    def execute_graph(self, ct_in: torch.Tensor, ct_out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """execute() through a HIP graph captured on first use for these
        buffers and replayed afterwards (stream: a torch stream other than
        the null stream; the current stream by default)."""
        if ct_out is None:
            ct_out = torch.empty((self.info.n_outputs, self.ct_words), dtype=torch.int32, device=ct_in.device)
        ws = self.workspace()
        S.sfft_execute_graph(self.handle, ct_in.data_ptr(), ct_out.data_ptr(), ws.data_ptr(), ws.numel() * 4,
                             _stream_ptr(stream))
        return ct_out

    def tune(self, ct_in: torch.Tensor, ct_out: torch.Tensor | None = None, reps: int = 3, stream=None):
        """Time the plan's widest level under every tiling that can serve it
        and switch the plan to the fastest: (tiling, {tiling: bit-MAC/s})."""
        if ct_out is None:
            ct_out = torch.empty((self.info.n_outputs, self.ct_words), dtype=torch.int32, device=ct_in.device)
        ws = self.workspace()
        best, rates = S.sfft_plan_tune(self.handle, ct_in.data_ptr(), ct_out.data_ptr(), ws.data_ptr(),
                                       ws.numel() * 4, reps, _stream_ptr(stream))
        self.info = S.sfft_plan_info_get(self.handle)
        return best, {i: r for i, r in enumerate(rates) if r > 0}

    def step_products(self):
        return S.sfft_plan_step_products(self.handle, self.info.exec_steps)

    def close(self):
        if self.handle:
            S.sfft_plan_destroy(self.handle)
            self.handle = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(params: S.sfft_params, reps: int = 3, stream=None):
    """Time every product-kernel tiling for params' geometry on the GPU and
    record the fastest for plans created afterwards: (tiling, {tiling:
    bit-MAC/s})."""
    best, rates = S.sfft_tune(params, reps, _stream_ptr(stream))
    return best, {i: r for i, r in enumerate(rates) if r > 0}


def set_tiling(params: S.sfft_params, tiling: int) -> None:
    """Record a tiling for params' geometry (-1: back to the default)."""
    S.sfft_set_tiling(params, tiling)


def size_params(dims, length, F, f, is_complex, n_lwe, nand_only: bool = False) -> S.sfft_params:
    return S.sfft_size_params(S.shape(dims, length, F, f, is_complex, nand_only), n_lwe)


def signal_words(sig) -> np.ndarray:
    """Quantised input words in ciphertext order: point-major, Re then Im."""
    re = quantize(np.asarray(sig.re).ravel(), sig.F, sig.f)
    if sig.im is None:
        return re
    im = quantize(np.asarray(sig.im).ravel(), sig.F, sig.f)
    return np.stack([re, im], 1).ravel()


class Batch:
    """A fixed batch of (plan, ct_in, ct_out) requests merged level by level
    and compiled once (sfft_batch_*); the workspace is allocated here."""

    def __init__(self, requests):
        self._keep = list(requests)
        plans = [p.handle for p, _, _ in requests]
        self.ws_bytes = S.sfft_batch_workspace_bytes(plans)
        self._ws = torch.empty(max(1, self.ws_bytes // 4), dtype=torch.int32, device="cuda")
        self.handle = S.sfft_batch_create(plans, [i.data_ptr() for _, i, _ in requests],
                                          [o.data_ptr() for _, _, o in requests], self._ws.data_ptr(),
                                          self._ws.numel() * 4)
        self.steps, self.launches = S.sfft_batch_info(self.handle)

    def execute(self, stream=None):
        S.sfft_batch_execute(self.handle, _stream_ptr(stream))

    def execute_graph(self, stream=None):
        """One graph launch (captured on first use) on `stream`, a torch
        stream other than the null stream (the current one by default)."""
        S.sfft_batch_execute_graph(self.handle, _stream_ptr(stream))

    def close(self):
        if self.handle:
            S.sfft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over libsfft's sfft_server_*."""

    def __init__(self, mem_budget_bytes: int, max_active: int = 0, dry_run: bool = False,
                 dry_bitmac_per_s: float = 0.0, fill_blocks: int = 0, serial: bool = False):
        flags = (S.SFFT_SERVER_DRYRUN if dry_run else 0) | (S.SFFT_SERVER_SERIAL if serial else 0)
        cfg = S.sfft_server_cfg(int(mem_budget_bytes), int(max_active), flags, float(dry_bitmac_per_s),
                                int(fill_blocks))
        self.dry = dry_run
        self.handle = S.sfft_server_create(cfg)
        self._keep = {}

    def submit(self, dims, length, F, f, is_complex, params, ct_in=None, ct_out=None, nand_only=False) -> int:
        shp = S.shape(dims, length, F, f, is_complex, nand_only)
        t = S.sfft_server_submit(self.handle, shp, params, ct_in.data_ptr() if ct_in is not None else None,
                                 ct_out.data_ptr() if ct_out is not None else None)
        self._keep[t] = (ct_in, ct_out)  # the buffers must outlive the request
        return t

    def submit_plan(self, plan: "Plan", ct_in: torch.Tensor, ct_out: torch.Tensor) -> int:
        """Queue a request on a plan compiled beforehand (shared; keep it open
        until the request completes)."""
        t = S.sfft_server_submit_plan(self.handle, plan.handle, ct_in.data_ptr(), ct_out.data_ptr())
        self._keep[t] = (ct_in, ct_out, plan)
        return t

    def step(self, stream=None) -> int:
        return S.sfft_server_step(self.handle, None if self.dry else _stream_ptr(stream))

    def drain(self, stream=None) -> None:
        S.sfft_server_drain(self.handle, None if self.dry else _stream_ptr(stream))

    def poll(self, ticket):
        """(done, latency_s); once done, the request's buffers are no longer
        held by the server object."""
        done, lat = S.sfft_server_poll(self.handle, ticket)
        if done:
            self._keep.pop(ticket, None)
        return done, lat

    def stats(self):
        return S.sfft_server_stats_get(self.handle)

    def close(self):
        if self.handle:
            S.sfft_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
