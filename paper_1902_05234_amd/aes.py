"""ctypes binding of libaesgpu (include/aesgpu.h), same names as the C ABI.

Argument marshalling only: every cipher step runs in the HIP kernels of
libaesgpu.so.  PyTorch supplies device memory (uint8 CUDA tensors) and
streams.  There is no fallback: if the library is missing or fails to load,
every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# another build of the library (say, one with host sanitizers) can be named in AESGPU_LIBRARY
LIBRARY = os.environ.get("AESGPU_LIBRARY") or os.path.join(HERE, "libaesgpu.so")
TUNE_FILE_ENV = "AESGPU_TUNE_FILE"  # path of an autotune record to install when the library loads
TUNE_FORCE_ENV = "AESGPU_TUNE_FORCE"  # "1": install that record even if made on another device or sources

AES_OK, AES_EINVAL, AES_EALIGN, AES_ENOMEM, AES_EHIP, AES_EBUSY, AES_ERANGE = 0, -1, -2, -3, -4, -5, -6
AES_PLACEMENT_TTABLE4, AES_PLACEMENT_TTABLE2, AES_PLACEMENT_TTABLE1, AES_PLACEMENT_BITSLICED = 0, 1, 2, 3
AES_BPT_COLUMN = 0  # Variant.bpt: one column word per lane, four lanes per block
AES_BPT_WAVE_MSG = 16  # Variant.bpt base of CBC message-set decryption with one wave per message
AES_KEY_SLOT_WORDS, AES_KEY_SLOT_ENC, AES_KEY_SLOT_DEC, AES_KEY_SLOT_NR = 128, 0, 64, 124
AES_SIZE_BUCKETS = 7

MSG_DTYPE = np.dtype([("in_block", "<u8"), ("out_block", "<u8"), ("nblocks", "<u8"),
                      ("key_slot", "<u4"), ("decrypt", "<u4")])
AES_MAX_ITEM_BLOCKS = 1 << 24  # largest work item (blocks), as in the C header
ITEM_DTYPE = np.dtype([("in_block", "<u8"), ("out_block", "<u8"), ("nblocks", "<u4"), ("key_slot", "<u4")])
CBC_MSG_DTYPE = np.dtype([("in_block", "<u8"), ("out_block", "<u8"), ("nblocks", "<u8"), ("reserved", "<u8"),
                          ("iv", "u1", (16,))])
assert MSG_DTYPE.itemsize == 32 and ITEM_DTYPE.itemsize == 24 and CBC_MSG_DTYPE.itemsize == 48


class AesError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("aesgpu error %d: %s" % (code, message))
        self.code = code


class _Variant(ctypes.Structure):
    _fields_ = [("bpt", ctypes.c_int32), ("wg", ctypes.c_int32), ("placement", ctypes.c_int32), ("grid", ctypes.c_int32)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("bpt", ctypes.c_int32), ("wg", ctypes.c_int32), ("grid", ctypes.c_int32), ("enc_groups", ctypes.c_int32),
                ("placement", ctypes.c_int32)]


@dataclass(frozen=True)
class Variant:
    bpt: int = 1
    wg: int = 1024
    placement: int = AES_PLACEMENT_TTABLE4
    grid: int = 0

    def _c(self) -> _Variant:
        return _Variant(self.bpt, self.wg, self.placement, self.grid)


_lib_obj = None
_lib_lock = threading.Lock()

_c_p = ctypes.c_void_p
_c_sz = ctypes.c_size_t
_c_i = ctypes.c_int
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def library_path() -> str:
    return LIBRARY


def _lib() -> ctypes.CDLL:
    global _lib_obj
    if _lib_obj is not None:
        return _lib_obj
    with _lib_lock:
        if _lib_obj is None:
            if not os.path.exists(LIBRARY):
                raise RuntimeError("libaesgpu.so is not built (%s); run `python -m paper_1902_05234_amd.build`" % LIBRARY)
            # torch ships its own libamdhip64.so.7; loading it first makes the
            # library's libamdhip64.so.7 dependency resolve to that same
            # runtime, so torch's streams and device pointers are valid here.
            import torch  # noqa: F401
            lib = ctypes.CDLL(LIBRARY)
            sig = {
                "aes_last_error": ([], ctypes.c_char_p),
                "aes_expand_key": ([_u8p, _c_i, _u32p, _u32p, ctypes.POINTER(_c_i)], _c_i),
                "aes_key_slot": ([_u8p, _c_i, _u32p], _c_i),
                "aes_ecb_encrypt": ([_u32p, _c_i, _c_p, _c_p, _c_sz, _c_p], _c_i),
                "aes_ecb_decrypt": ([_u32p, _c_i, _c_p, _c_p, _c_sz, _c_p], _c_i),
                "aes_ecb_crypt_variant": ([_u32p, _c_i, _c_i, _c_p, _c_p, _c_sz, ctypes.POINTER(_Variant), _c_p], _c_i),
                "aes_ctr_crypt": ([_u32p, _c_i, _u8p, ctypes.c_uint64, _c_p, _c_p, _c_sz, _c_p], _c_i),
                "aes_ctr_crypt_variant": ([_u32p, _c_i, _u8p, ctypes.c_uint64, _c_p, _c_p, _c_sz,
                                           ctypes.POINTER(_Variant), _c_p], _c_i),
                "aes_cbc_decrypt": ([_u32p, _c_i, _u8p, _c_p, _c_p, _c_sz, _c_p], _c_i),
                "aes_cbc_decrypt_variant": ([_u32p, _c_i, _u8p, _c_p, _c_p, _c_sz, ctypes.POINTER(_Variant), _c_p],
                                            _c_i),
                "aes_cbc_encrypt_msgs": ([_u32p, _c_i, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_p], _c_i),
                "aes_cbc_encrypt_msgs_variant": ([_u32p, _c_i, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p,
                                                  ctypes.POINTER(_Variant), _c_p], _c_i),
                "aes_cbc_decrypt_msgs": ([_u32p, _c_i, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_p], _c_i),
                "aes_cbc_decrypt_msgs_variant": ([_u32p, _c_i, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p,
                                                  ctypes.POINTER(_Variant), _c_p], _c_i),
                "aes_tune_set": ([_c_i, _c_i, _c_sz, ctypes.POINTER(_Variant)], _c_i),
                "aes_tune_get": ([_c_i, _c_i, _c_sz, ctypes.POINTER(_Variant)], _c_i),
                "aes_size_bucket": ([_c_sz], _c_i),
                "aes_batch_plan": ([_c_p, _c_sz, ctypes.c_uint32, _c_p, _c_sz, ctypes.POINTER(_c_sz), ctypes.POINTER(_c_sz)], _c_i),
                "aes_ecb_batch": ([_c_p, _c_sz, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p,
                                   ctypes.POINTER(_BatchConfig), _c_p], _c_i),
                "aes_batch_max_grid": ([ctypes.POINTER(_BatchConfig), ctypes.POINTER(_c_i)], _c_i),
                "aes_ecb_batch_noalloc": ([_c_p, _c_sz, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz,
                                           ctypes.POINTER(_BatchConfig), _c_p], _c_i),
                "aes_device_copy": ([_c_p, _c_p, _c_sz, _c_p], _c_i),
                "aes_roof_probe": ([_c_i, ctypes.c_uint32, _c_p, _c_sz, ctypes.POINTER(ctypes.c_uint64), _c_p], _c_i),
                "aes_host_tables": ([_u8p, _u8p, _u32p, _u32p], _c_i),
            }
            for name, (args, res) in sig.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = res
            _lib_obj = lib
            path = os.environ.get(TUNE_FILE_ENV)
            if path:
                # an autotune record (paper_1902_05234_amd.autotune --out) replaces the
                # compiled-in defaults for every size it covers; a record made on
                # another device or for other kernel sources is refused unless
                # AESGPU_TUNE_FORCE=1
                from . import autotune
                autotune.apply(autotune.load(path), force=os.environ.get(TUNE_FORCE_ENV) == "1")
    return _lib_obj


def exported_symbols():
    """Names this binding expects the library to export."""
    return ["aes_last_error", "aes_expand_key", "aes_key_slot", "aes_ecb_encrypt", "aes_ecb_decrypt",
            "aes_ecb_crypt_variant", "aes_ctr_crypt", "aes_ctr_crypt_variant", "aes_cbc_decrypt",
            "aes_cbc_decrypt_variant", "aes_cbc_encrypt_msgs", "aes_cbc_encrypt_msgs_variant", "aes_cbc_decrypt_msgs",
            "aes_cbc_decrypt_msgs_variant", "aes_tune_set", "aes_tune_get", "aes_size_bucket", "aes_batch_plan",
            "aes_ecb_batch", "aes_ecb_batch_noalloc", "aes_batch_max_grid", "aes_device_copy", "aes_roof_probe", "aes_host_tables", "aes_server_workspace_bytes",
            "aes_server_staging_bytes", "aes_server_create", "aes_server_submit", "aes_server_poll",
            "aes_server_release", "aes_server_stats", "aes_server_destroy", "aes_serve_replay", "aes_pipe_create",
            "aes_pipe_destroy", "aes_pipe_run"]


def aes_last_error() -> str:
    return _lib().aes_last_error().decode()


def _check(rc: int):
    if rc != AES_OK:
        raise AesError(rc, aes_last_error())


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _bytes_of(t, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.numel() * t.element_size()


def _blocks_of(t, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    nbytes = t.numel() * t.element_size()
    if nbytes % 16:
        raise ValueError("%s must hold whole 16-byte blocks (%d bytes)" % (name, nbytes))
    return nbytes // 16


def _u32_array(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if n is not None and a.size < n:
        raise ValueError("round-key array too short")
    return a


# --------------------------------------------------------------- key schedule
@dataclass(frozen=True)
class KeySchedule:
    rk_enc: np.ndarray
    rk_dec: np.ndarray
    nr: int
    keybits: int


def aes_expand_key(key: bytes, keybits: int | None = None) -> KeySchedule:
    key = bytes(key)
    keybits = 8 * len(key) if keybits is None else int(keybits)
    if keybits != 8 * len(key):
        raise ValueError("key is %d bytes, keybits=%d" % (len(key), keybits))
    kb = (ctypes.c_uint8 * max(1, len(key))).from_buffer_copy(key or b"\0")
    enc = np.zeros(60, dtype=np.uint32)
    dec = np.zeros(60, dtype=np.uint32)
    nr = ctypes.c_int(0)
    _check(_lib().aes_expand_key(kb, keybits, enc.ctypes.data_as(_u32p), dec.ctypes.data_as(_u32p), ctypes.byref(nr)))
    n = 4 * (nr.value + 1)
    return KeySchedule(enc[:n].copy(), dec[:n].copy(), nr.value, keybits)


def aes_key_slot(key: bytes) -> np.ndarray:
    key = bytes(key)
    kb = (ctypes.c_uint8 * max(1, len(key))).from_buffer_copy(key or b"\0")
    out = np.zeros(AES_KEY_SLOT_WORDS, dtype=np.uint32)
    _check(_lib().aes_key_slot(kb, 8 * len(key), out.ctypes.data_as(_u32p)))
    return out


# ------------------------------------------------------------------ plain ECB
def _crypt(fn, rk, nr, inp, out, nblocks, stream):
    n_in = _blocks_of(inp, "in")
    n_out = _blocks_of(out, "out")
    nblocks = n_in if nblocks is None else int(nblocks)
    if nblocks < 0 or nblocks > n_in or nblocks > n_out:
        raise ValueError("nblocks=%d is negative or exceeds a buffer (in %d, out %d blocks)" % (nblocks, n_in, n_out))
    rk = _u32_array(rk, 4 * (int(nr) + 1))
    _check(fn(rk.ctypes.data_as(_u32p), int(nr), inp.data_ptr(), out.data_ptr(), nblocks, _stream_handle(stream)))
    return out


def aes_ecb_encrypt(rk, nr: int, inp, out, nblocks: int | None = None, stream=None):
    return _crypt(_lib().aes_ecb_encrypt, rk, nr, inp, out, nblocks, stream)


def aes_ecb_decrypt(rk, nr: int, inp, out, nblocks: int | None = None, stream=None):
    return _crypt(_lib().aes_ecb_decrypt, rk, nr, inp, out, nblocks, stream)


def aes_ecb_crypt_variant(rk, nr: int, decrypt: bool, inp, out, variant: Variant, nblocks: int | None = None, stream=None):
    lib = _lib()
    v = variant._c()

    def fn(rkp, nr_, i, o, n, s):
        return lib.aes_ecb_crypt_variant(rkp, nr_, int(bool(decrypt)), i, o, n, ctypes.byref(v), s)

    return _crypt(fn, rk, nr, inp, out, nblocks, stream)


# ------------------------------------------------------------------ CTR mode
def _ctr(fn, rk, nr, iv, block_offset, inp, out, nbytes, stream, *extra):
    n_in, n_out = _bytes_of(inp, "in"), _bytes_of(out, "out")
    nbytes = n_in if nbytes is None else int(nbytes)
    if nbytes < 0 or nbytes > n_in or nbytes > n_out:
        raise ValueError("nbytes=%d exceeds a buffer (in %d, out %d bytes)" % (nbytes, n_in, n_out))
    iv = bytes(iv)
    if len(iv) != 16:
        raise ValueError("the counter block is 16 bytes, got %d" % len(iv))
    rk = _u32_array(rk, 4 * (int(nr) + 1))
    ivb = (ctypes.c_uint8 * 16).from_buffer_copy(iv)
    _check(fn(rk.ctypes.data_as(_u32p), int(nr), ivb, int(block_offset) & (2**64 - 1), inp.data_ptr(),
              out.data_ptr(), nbytes, *extra, _stream_handle(stream)))
    return out


def aes_ctr_crypt(rk, nr: int, iv: bytes, block_offset: int, inp, out, nbytes: int | None = None, stream=None):
    """CTR encryption/decryption of nbytes (default: all of ``inp``); rk is
    the encryption schedule; data block j uses counter iv + block_offset + j."""
    return _ctr(_lib().aes_ctr_crypt, rk, nr, iv, block_offset, inp, out, nbytes, stream)


def aes_ctr_crypt_variant(rk, nr: int, iv: bytes, block_offset: int, inp, out, variant: Variant,
                          nbytes: int | None = None, stream=None):
    v = variant._c()
    return _ctr(_lib().aes_ctr_crypt_variant, rk, nr, iv, block_offset, inp, out, nbytes, stream, ctypes.byref(v))


# ------------------------------------------------------------ CBC decryption
def _cbc(fn, rk, nr, iv, inp, out, nblocks, stream, *extra):
    n_in, n_out = _blocks_of(inp, "in"), _blocks_of(out, "out")
    nblocks = n_in if nblocks is None else int(nblocks)
    if nblocks < 0 or nblocks > n_in or nblocks > n_out:
        raise ValueError("nblocks=%d is negative or exceeds a buffer (in %d, out %d blocks)" % (nblocks, n_in, n_out))
    iv = bytes(iv)
    if len(iv) != 16:
        raise ValueError("the initialisation vector is 16 bytes, got %d" % len(iv))
    rk = _u32_array(rk, 4 * (int(nr) + 1))
    ivb = (ctypes.c_uint8 * 16).from_buffer_copy(iv)
    _check(fn(rk.ctypes.data_as(_u32p), int(nr), ivb, inp.data_ptr(), out.data_ptr(), nblocks, *extra,
              _stream_handle(stream)))
    return out


def aes_cbc_decrypt(rk, nr: int, iv: bytes, inp, out, nblocks: int | None = None, stream=None):
    """CBC decryption of whole blocks; rk is the decryption schedule; out
    must not overlap inp."""
    return _cbc(_lib().aes_cbc_decrypt, rk, nr, iv, inp, out, nblocks, stream)


def aes_cbc_decrypt_variant(rk, nr: int, iv: bytes, inp, out, variant: Variant, nblocks: int | None = None,
                            stream=None):
    v = variant._c()
    return _cbc(_lib().aes_cbc_decrypt_variant, rk, nr, iv, inp, out, nblocks, stream, ctypes.byref(v))


def aes_cbc_encrypt_msgs(rk, nr: int, msgs_dev, nmsgs: int, in_base, out_base, rejected_dev=None,
                         variant: Variant | None = None, stream=None):
    """CBC encryption of nmsgs independent messages described by the device
    tensor ``msgs_dev`` (CBC_MSG_DTYPE records) between the arenas ``in_base``
    and ``out_base``; rk is the encryption schedule.  ``rejected_dev`` (a
    device int32/uint32 tensor, or None) receives the count of skipped
    messages."""
    lib = _lib()
    return _cbc_msgs(lib.aes_cbc_encrypt_msgs, lib.aes_cbc_encrypt_msgs_variant, rk, nr, msgs_dev, nmsgs, in_base,
                     out_base, rejected_dev, variant, stream)


def aes_cbc_decrypt_msgs(rk, nr: int, msgs_dev, nmsgs: int, in_base, out_base, rejected_dev=None,
                         variant: Variant | None = None, stream=None):
    """CBC decryption of a message set (as aes_cbc_encrypt_msgs); rk is the
    decryption schedule."""
    lib = _lib()
    return _cbc_msgs(lib.aes_cbc_decrypt_msgs, lib.aes_cbc_decrypt_msgs_variant, rk, nr, msgs_dev, nmsgs, in_base,
                     out_base, rejected_dev, variant, stream)


def _cbc_msgs(fn, fn_variant, rk, nr, msgs_dev, nmsgs, in_base, out_base, rejected_dev, variant, stream):
    nmsgs = int(nmsgs)
    if nmsgs < 0 or _bytes_of(msgs_dev, "msgs_dev") < nmsgs * CBC_MSG_DTYPE.itemsize:
        raise ValueError("message tensor smaller than nmsgs records")
    rej = 0
    if rejected_dev is not None:
        if _bytes_of(rejected_dev, "rejected_dev") < 4:
            raise ValueError("the rejected counter needs 4 bytes")
        rej = rejected_dev.data_ptr()
    rk = _u32_array(rk, 4 * (int(nr) + 1))
    args = [rk.ctypes.data_as(_u32p), int(nr), msgs_dev.data_ptr(), nmsgs, in_base.data_ptr(),
            _blocks_of(in_base, "in_base"), out_base.data_ptr(), _blocks_of(out_base, "out_base"), rej]
    if variant is None:
        _check(fn(*args, _stream_handle(stream)))
    else:
        v = variant._c()
        _check(fn_variant(*args, ctypes.byref(v), _stream_handle(stream)))
    return out_base


def aes_tune_set(nr: int, decrypt: bool, nblocks: int, variant: Variant):
    v = variant._c()
    _check(_lib().aes_tune_set(int(nr), int(bool(decrypt)), int(nblocks), ctypes.byref(v)))


def aes_tune_get(nr: int, decrypt: bool, nblocks: int) -> Variant:
    v = _Variant()
    _check(_lib().aes_tune_get(int(nr), int(bool(decrypt)), int(nblocks), ctypes.byref(v)))
    return Variant(v.bpt, v.wg, v.placement, v.grid)


def aes_size_bucket(nblocks: int) -> int:
    return int(_lib().aes_size_bucket(int(nblocks)))


def expand_key(key: bytes) -> KeySchedule:
    """Key schedule of a 16-, 24- or 32-byte key (encryption and equivalent
    inverse), for ecb_encrypt / ecb_decrypt / ctr_crypt / cbc_decrypt."""
    return aes_expand_key(key)


def ecb_encrypt(ks: KeySchedule, x, out=None, stream=None):
    """Encrypt a uint8 CUDA tensor of whole blocks; returns ``out``."""
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_ecb_encrypt(ks.rk_enc, ks.nr, x, out, stream=stream)


def ecb_decrypt(ks: KeySchedule, x, out=None, stream=None):
    """Decrypt a uint8 CUDA tensor of whole blocks; returns ``out``."""
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_ecb_decrypt(ks.rk_dec, ks.nr, x, out, stream=stream)


def ctr_crypt(ks: KeySchedule, iv: bytes, x, out=None, block_offset: int = 0, stream=None):
    """CTR over a uint8 CUDA tensor of any length; returns ``out``."""
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_ctr_crypt(ks.rk_enc, ks.nr, iv, block_offset, x, out, stream=stream)


def cbc_decrypt(ks: KeySchedule, iv: bytes, x, out=None, stream=None):
    """CBC decryption of a uint8 CUDA tensor of whole blocks into a separate
    ``out`` (in place is refused: block b reads ciphertext block b - 1)."""
    import torch
    out = torch.empty_like(x) if out is None else out
    return aes_cbc_decrypt(ks.rk_dec, ks.nr, iv, x, out, stream=stream)


def _msgs_on_device(recs, like):
    import torch
    if isinstance(recs, torch.Tensor):
        return recs, (recs.numel() * recs.element_size()) // CBC_MSG_DTYPE.itemsize
    recs = np.ascontiguousarray(recs, dtype=CBC_MSG_DTYPE)
    return torch.from_numpy(recs.view(np.uint8)).to(like.device), recs.size


def cbc_encrypt_msgs(ks: KeySchedule, recs, x, out=None, stream=None):
    """CBC encryption of the message set ``recs`` (a host numpy array of
    CBC_MSG_DTYPE records, or a device uint8 tensor holding them) from the
    uint8 CUDA tensor ``x`` into ``out`` (a new tensor like ``x`` if None)."""
    import torch
    out = torch.empty_like(x) if out is None else out
    msgs, n = _msgs_on_device(recs, x)
    return aes_cbc_encrypt_msgs(ks.rk_enc, ks.nr, msgs, n, x, out, stream=stream)


def cbc_decrypt_msgs(ks: KeySchedule, recs, x, out=None, stream=None):
    """CBC decryption of the message set ``recs`` (as cbc_encrypt_msgs)."""
    import torch
    out = torch.empty_like(x) if out is None else out
    msgs, n = _msgs_on_device(recs, x)
    return aes_cbc_decrypt_msgs(ks.rk_dec, ks.nr, msgs, n, x, out, stream=stream)


# ---------------------------------------------------------------- batched ECB
def aes_batch_plan(msgs: np.ndarray, chunk_blocks: int):
    """Host planner: returns (items [ITEM_DTYPE], n_enc, n_dec)."""
    msgs = np.ascontiguousarray(msgs, dtype=MSG_DTYPE)
    lib = _lib()
    ne, nd = ctypes.c_size_t(0), ctypes.c_size_t(0)
    rc = lib.aes_batch_plan(msgs.ctypes.data if msgs.size else None, msgs.size, int(chunk_blocks), None, 0,
                            ctypes.byref(ne), ctypes.byref(nd))
    n = ne.value + nd.value
    if rc != AES_OK and not (rc == AES_ERANGE and n > 0):  # ERANGE with counts: only the capacity was short
        _check(rc)
    items = np.zeros(n, dtype=ITEM_DTYPE)
    if n:
        _check(lib.aes_batch_plan(msgs.ctypes.data, msgs.size, int(chunk_blocks), items.ctypes.data, n,
                                  ctypes.byref(ne), ctypes.byref(nd)))
    return items, ne.value, nd.value


@dataclass(frozen=True)
class BatchConfig:
    bpt: int = 1
    wg: int = 1024
    grid: int = 0
    enc_groups: int = -1
    placement: int = AES_PLACEMENT_TTABLE4


def aes_ecb_batch(items_dev, n_enc: int, n_dec: int, key_table_dev, in_base, out_base, counters_dev,
                  cfg: BatchConfig | None = None, stream=None):
    """One persistent launch over a device work list (tensors: uint8/int views of device memory)."""
    n_slots = (key_table_dev.numel() * key_table_dev.element_size()) // (4 * AES_KEY_SLOT_WORDS)
    if items_dev.numel() * items_dev.element_size() < (n_enc + n_dec) * ITEM_DTYPE.itemsize:
        raise ValueError("work list tensor smaller than n_enc + n_dec items")
    if counters_dev.numel() * counters_dev.element_size() < 16:
        raise ValueError("counters need 4 uint32")
    c = cfg or BatchConfig()
    bc = _BatchConfig(c.bpt, c.wg, c.grid, c.enc_groups, c.placement)
    _check(_lib().aes_ecb_batch(items_dev.data_ptr(), int(n_enc), int(n_dec), key_table_dev.data_ptr(), n_slots,
                                in_base.data_ptr(), _blocks_of(in_base, "in_base"), out_base.data_ptr(),
                                _blocks_of(out_base, "out_base"), counters_dev.data_ptr(), ctypes.byref(bc),
                                _stream_handle(stream)))


def aes_ecb_batch_noalloc(items_dev, n_enc: int, n_dec: int, key_table_dev, in_base, out_base,
                          cfg: BatchConfig | None = None, stream=None):
    """aes_ecb_batch with the claim counters in the library's per-device
    scratch (no counters argument; the call allocates nothing)."""
    n_slots = (key_table_dev.numel() * key_table_dev.element_size()) // (4 * AES_KEY_SLOT_WORDS)
    if items_dev.numel() * items_dev.element_size() < (n_enc + n_dec) * ITEM_DTYPE.itemsize:
        raise ValueError("work list tensor smaller than n_enc + n_dec items")
    c = cfg or BatchConfig()
    bc = _BatchConfig(c.bpt, c.wg, c.grid, c.enc_groups, c.placement)
    _check(_lib().aes_ecb_batch_noalloc(items_dev.data_ptr(), int(n_enc), int(n_dec), key_table_dev.data_ptr(),
                                        n_slots, in_base.data_ptr(), _blocks_of(in_base, "in_base"),
                                        out_base.data_ptr(), _blocks_of(out_base, "out_base"), ctypes.byref(bc),
                                        _stream_handle(stream)))


def aes_batch_max_grid(cfg: BatchConfig | None = None) -> int:
    """Workgroups a batch launch with cfg uses at most (the persistent grid)."""
    c = cfg or BatchConfig()
    g = _c_i(0)
    _check(_lib().aes_batch_max_grid(ctypes.byref(_BatchConfig(c.bpt, c.wg, c.grid, c.enc_groups, c.placement)),
                                     ctypes.byref(g)))
    return g.value


def aes_device_copy(inp, out, nbytes: int | None = None, stream=None):
    nbytes = inp.numel() * inp.element_size() if nbytes is None else int(nbytes)
    _check(_lib().aes_device_copy(inp.data_ptr(), out.data_ptr(), nbytes, _stream_handle(stream)))


AES_PROBE_LDS = 0
AES_PROBE_VALU = 1


def aes_roof_probe(which: int, iters: int, out, stream=None) -> int:
    """Launch a roofline probe (AES_PROBE_LDS / AES_PROBE_VALU) writing into the
    device tensor ``out``; returns the operations it performs (time it with events)."""
    work = ctypes.c_uint64(0)
    _check(_lib().aes_roof_probe(int(which), int(iters), out.data_ptr(), out.numel() * out.element_size(),
                                 ctypes.byref(work), _stream_handle(stream)))
    return work.value


def aes_host_tables():
    """(sbox, inv_sbox, te0, td0) as numpy arrays, from the library's host copy."""
    sbox = np.zeros(256, dtype=np.uint8)
    inv = np.zeros(256, dtype=np.uint8)
    te0 = np.zeros(256, dtype=np.uint32)
    td0 = np.zeros(256, dtype=np.uint32)
    _check(_lib().aes_host_tables(sbox.ctypes.data_as(_u8p), inv.ctypes.data_as(_u8p), te0.ctypes.data_as(_u32p),
                                  td0.ctypes.data_as(_u32p)))
    return sbox, inv, te0, td0


# -------------------------------------------------------------- native serving
REQUEST_DTYPE = np.dtype([("in_block", "<u8"), ("nblocks", "<u8"), ("key_slot", "<u4"), ("decrypt", "<u4")])
SERVED_DTYPE = np.dtype([("id", "<u8"), ("arrival_s", "<f8"), ("admitted_s", "<f8"), ("done_s", "<f8"),
                         ("out_block", "<u8"), ("nblocks", "<u8"), ("status", "<i4"), ("batch", "<i4")])
assert REQUEST_DTYPE.itemsize == 24 and SERVED_DTYPE.itemsize == 56
AES_SERVED_DONE, AES_SERVED_REJECTED, AES_SERVED_FAILED = 0, 1, 2
AES_SERVE_COMPLETION_AUTO, AES_SERVE_COMPLETION_EVENTS = 0, 1


class _ServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("chunk_blocks", ctypes.c_uint32),
                ("max_batch_items", ctypes.c_uint32), ("nslots", ctypes.c_int32), ("bpt", ctypes.c_int32),
                ("wg", ctypes.c_int32), ("grid", ctypes.c_int32), ("auto_release", ctypes.c_int32),
                ("dry_run", ctypes.c_int32), ("dry_run_seconds", ctypes.c_double), ("placement", ctypes.c_int32),
                ("completion", ctypes.c_int32), ("small_item_blocks", ctypes.c_uint32),
                ("size_classes", ctypes.c_int32)]


class _ServeStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("max_device_bytes_in_use", ctypes.c_uint64),
                ("arena_blocks_in_use", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("direct_batches", ctypes.c_uint64), ("launch_ns", ctypes.c_uint64)]


def _serve_sigs(lib):
    if getattr(lib, "_serve_sigs", False):
        return
    cfgp = ctypes.POINTER(_ServeConfig)
    lib.aes_server_workspace_bytes.argtypes = [cfgp]
    lib.aes_server_workspace_bytes.restype = _c_sz
    lib.aes_server_staging_bytes.argtypes = [cfgp]
    lib.aes_server_staging_bytes.restype = _c_sz
    lib.aes_server_create.argtypes = [cfgp, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz, _c_p, _c_sz,
                                      ctypes.POINTER(_c_p)]
    lib.aes_server_create.restype = _c_i
    lib.aes_server_submit.argtypes = [_c_p, _c_p, _c_sz, ctypes.POINTER(ctypes.c_uint64)]
    lib.aes_server_submit.restype = _c_i
    lib.aes_server_poll.argtypes = [_c_p, _c_p, _c_sz, ctypes.POINTER(_c_sz)]
    lib.aes_server_poll.restype = _c_i
    lib.aes_server_release.argtypes = [_c_p, _c_p, _c_sz]
    lib.aes_server_release.restype = _c_i
    lib.aes_server_stats.argtypes = [_c_p, ctypes.POINTER(_ServeStats)]
    lib.aes_server_stats.restype = _c_i
    lib.aes_server_destroy.argtypes = [_c_p]
    lib.aes_server_destroy.restype = _c_i
    lib.aes_serve_replay.argtypes = [_c_p, _c_p, _c_p, _c_sz, _c_p]
    lib.aes_serve_replay.restype = _c_i
    lib._serve_sigs = True


class Server:
    """The native continuous-batching engine (aes_server_* in aesgpu.h).

    Device buffers are torch tensors owned by the caller (kept alive here);
    the work-list workspace and pinned staging are allocated here with torch.
    ``dry_run`` runs the admission policy with no device work (CPU only).
    ``size_classes`` (on by default) keeps requests of at most ``chunk_blocks``
    blocks and larger ones in separate batches.
    """

    def __init__(self, key_table_dev=None, in_pool=None, out_arena=None, *, n_slots=None, in_blocks=None,
                 out_blocks=None, budget_bytes=32 << 30, chunk_blocks=2048, max_batch_items=1 << 18, nslots=4,
                 bpt=4, wg=1024, grid=0, auto_release=True, dry_run=False, dry_run_seconds=0.0,
                 placement=AES_PLACEMENT_TTABLE4, completion=0, small_item_blocks=None, size_classes=True):
        lib = _lib()
        _serve_sigs(lib)
        self._lib = lib
        self.cfg = _ServeConfig(int(budget_bytes), int(chunk_blocks), int(max_batch_items), int(nslots), int(bpt),
                                int(wg), int(grid), int(bool(auto_release)), int(bool(dry_run)), float(dry_run_seconds),
                                int(placement), int(completion),
                                # default: one wave unit (64 lanes x bpt blocks) per item of a small request
                                int(min(64 * bpt, chunk_blocks) if small_item_blocks is None else small_item_blocks),
                                int(bool(size_classes)))
        ws = lib.aes_server_workspace_bytes(ctypes.byref(self.cfg))
        st = lib.aes_server_staging_bytes(ctypes.byref(self.cfg))
        self._keep = [key_table_dev, in_pool, out_arena]
        if dry_run:
            self._ws = np.zeros(max(ws, 1), dtype=np.uint8)
            self._st = np.zeros(max(st, 1), dtype=np.uint8)
            ws_ptr, st_ptr = self._ws.ctypes.data, self._st.ctypes.data
        else:
            import torch
            self._ws = torch.empty(ws, dtype=torch.uint8, device="cuda")
            self._st = torch.empty(st, dtype=torch.uint8, pin_memory=True)
            ws_ptr, st_ptr = self._ws.data_ptr(), self._st.data_ptr()
            torch.cuda.synchronize()

        def ptr(t):
            return None if t is None else t.data_ptr()

        n_slots = n_slots if n_slots is not None else key_table_dev.numel() // AES_KEY_SLOT_WORDS
        in_blocks = in_blocks if in_blocks is not None else in_pool.numel() // 16
        out_blocks = out_blocks if out_blocks is not None else out_arena.numel() // 16
        self.out_blocks = out_blocks
        h = _c_p()
        _check_rc(lib.aes_server_create(ctypes.byref(self.cfg), ptr(key_table_dev), n_slots, ptr(in_pool), in_blocks,
                                        ptr(out_arena), out_blocks, ws_ptr, ws, st_ptr, st, ctypes.byref(h)),
                  "aes_server_create")
        self._h = h

    def submit(self, reqs) -> int:
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        first = ctypes.c_uint64(0)
        _check_rc(self._lib.aes_server_submit(self._h, reqs.ctypes.data if reqs.size else None, reqs.size,
                                              ctypes.byref(first)), "aes_server_submit")
        return first.value

    def poll(self, cap: int = 4096) -> np.ndarray:
        out = np.zeros(cap, dtype=SERVED_DTYPE)
        n = ctypes.c_size_t(0)
        _check_rc(self._lib.aes_server_poll(self._h, out.ctypes.data, cap, ctypes.byref(n)), "aes_server_poll")
        return out[:n.value]

    def release(self, served: np.ndarray):
        served = np.ascontiguousarray(served, dtype=SERVED_DTYPE)
        _check_rc(self._lib.aes_server_release(self._h, served.ctypes.data if served.size else None, served.size),
                  "aes_server_release")

    def stats(self) -> dict:
        s = _ServeStats()
        _check_rc(self._lib.aes_server_stats(self._h, ctypes.byref(s)), "aes_server_stats")
        return {"batches": s.batches, "max_device_bytes_in_use": s.max_device_bytes_in_use,
                "arena_blocks_in_use": s.arena_blocks_in_use, "pending": s.pending,
                "direct_batches": s.direct_batches, "launch_ns": s.launch_ns}

    def replay(self, reqs, arrival_s) -> np.ndarray:
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        out = np.zeros(reqs.size, dtype=SERVED_DTYPE)
        _check_rc(self._lib.aes_serve_replay(self._h, reqs.ctypes.data, arr.ctypes.data, reqs.size,
                                             out.ctypes.data), "aes_serve_replay")
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.aes_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def _check_rc(rc: int, what: str):
    if rc != AES_OK:
        raise AesError(rc, "%s failed (%s)" % (what, aes_last_error() or "see argument checks"))


# ------------------------------------------------------- host-inclusive path
AES_PIPE_ECB_ENCRYPT = 0
AES_PIPE_ECB_DECRYPT = 1
AES_PIPE_CTR = 2
AES_PIPE_HOST_PINNED = 1
AES_PIPE_MAX_SLOTS = 8


class _PipeConfig(ctypes.Structure):
    _fields_ = [("dev", _c_p), ("dev_bytes", ctypes.c_uint64), ("pinned", _c_p), ("pinned_bytes", ctypes.c_uint64),
                ("chunk_bytes", ctypes.c_uint64), ("nslots", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _pipe_sigs(lib):
    if getattr(lib, "_pipe_sigs", False):
        return
    lib.aes_pipe_create.argtypes = [ctypes.POINTER(_PipeConfig), ctypes.POINTER(_c_p)]
    lib.aes_pipe_create.restype = _c_i
    lib.aes_pipe_destroy.argtypes = [_c_p]
    lib.aes_pipe_destroy.restype = _c_i
    lib.aes_pipe_run.argtypes = [_c_p, _c_i, _u32p, _c_i, _u8p, _c_p, _c_p, _c_sz, _c_i]
    lib.aes_pipe_run.restype = _c_i
    lib._pipe_sigs = True


def _host_view(a, name):
    """(pointer, nbytes, pinned) of a host uint8 numpy array or CPU torch tensor."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.uint8 or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("%s must be a contiguous uint8 array" % name)
        return a.ctypes.data, a.size, False
    import torch
    if isinstance(a, torch.Tensor):
        if a.is_cuda or a.dtype != torch.uint8 or not a.is_contiguous():
            raise ValueError("%s must be a contiguous uint8 CPU tensor" % name)
        return a.data_ptr(), a.numel(), bool(a.is_pinned())
    raise TypeError("%s must be a numpy array or a CPU torch tensor" % name)


class HostPipe:
    """The host-inclusive path (aes_pipe_* in aesgpu.h): host buffers in and
    out, chunks pipelined over ``nslots`` streams.  The device workspace and
    the pinned staging are allocated here with torch and kept alive."""

    def __init__(self, chunk_bytes: int = 32 << 20, nslots: int = 2, staging: bool = True):
        import torch
        lib = _lib()
        _pipe_sigs(lib)
        self._lib = lib
        n = int(chunk_bytes) * int(nslots)
        self._dev = torch.empty(n, dtype=torch.uint8, device="cuda")
        self._pin = torch.empty(n, dtype=torch.uint8, pin_memory=True) if staging else None
        torch.cuda.synchronize()
        self.cfg = _PipeConfig(self._dev.data_ptr(), n, None if self._pin is None else self._pin.data_ptr(),
                               0 if self._pin is None else n, int(chunk_bytes), int(nslots), 0)
        h = _c_p()
        _check(lib.aes_pipe_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h

    def run(self, op: int, ks: KeySchedule, src, out=None, iv: bytes | None = None):
        """Encrypt (AES_PIPE_ECB_ENCRYPT), decrypt (AES_PIPE_ECB_DECRYPT) or
        CTR-process (AES_PIPE_CTR, with ``iv``) a host buffer; returns ``out``
        (a new numpy array if not given).  Pinned CPU tensors on both sides are
        copied without staging."""
        if self._h is None:
            raise RuntimeError("pipe is closed")
        if out is None:
            out = np.empty(src.size if isinstance(src, np.ndarray) else src.numel(), dtype=np.uint8)
        sp, sn, spin = _host_view(src, "src")
        op_, on, opin = _host_view(out, "out")
        if on < sn:
            raise ValueError("out holds %d bytes, src %d" % (on, sn))
        rk = ks.rk_dec if op == AES_PIPE_ECB_DECRYPT else ks.rk_enc
        rk = _u32_array(rk, 4 * (ks.nr + 1))
        ivb = None
        if op == AES_PIPE_CTR:
            iv = bytes(iv if iv is not None else bytes(16))
            if len(iv) != 16:
                raise ValueError("the counter block is 16 bytes")
            ivb = (ctypes.c_uint8 * 16).from_buffer_copy(iv)
        flags = AES_PIPE_HOST_PINNED if (spin and opin) else 0
        _check(self._lib.aes_pipe_run(self._h, int(op), rk.ctypes.data_as(_u32p), int(ks.nr), ivb, sp, op_, sn, flags))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.aes_pipe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
