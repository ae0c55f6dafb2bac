"""ctypes front end of the CPU AES oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.

The oracle computes AES-128/192/256 ECB byte by byte with GF(2^8) arithmetic
(see ``aes_oracle.c`` for the section of Wang & Chu, arXiv:1902.05234, or of
FIPS-197 that each step follows).
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

from . import build as _build

_u8 = ctypes.c_uint8
_p8 = ctypes.POINTER(ctypes.c_uint8)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_p8)


class Oracle:
    """One loaded copy of an oracle library (the default one, or a test build)."""

    def __init__(self, path: str):
        self.path = path
        lib = ctypes.CDLL(path)
        self._lib = lib
        lib.oracle_xtime.argtypes = [_u8]
        lib.oracle_xtime.restype = _u8
        lib.oracle_gf_mul.argtypes = [_u8, _u8]
        lib.oracle_gf_mul.restype = _u8
        lib.oracle_gf_inv.argtypes = [_u8]
        lib.oracle_gf_inv.restype = _u8
        for name in ("oracle_gf_mul_table", "oracle_sbox", "oracle_inv_sbox",
                     "oracle_mix_matrix", "oracle_inv_mix_matrix",
                     "oracle_sub_bytes", "oracle_inv_sub_bytes", "oracle_shift_rows",
                     "oracle_inv_shift_rows", "oracle_mix_columns", "oracle_inv_mix_columns"):
            getattr(lib, name).argtypes = [_p8]
            getattr(lib, name).restype = None
        lib.oracle_add_round_key.argtypes = [_p8, _p8]
        lib.oracle_add_round_key.restype = None
        lib.oracle_expand_key.argtypes = [_p8, ctypes.c_int, _p8, ctypes.POINTER(ctypes.c_int)]
        lib.oracle_expand_key.restype = ctypes.c_int
        for name in ("oracle_ecb_encrypt", "oracle_ecb_decrypt"):
            f = getattr(lib, name)
            f.argtypes = [_p8, ctypes.c_int, _p8, _p8, ctypes.c_uint64, ctypes.c_int]
            f.restype = ctypes.c_int
        lib.oracle_ctr_crypt.argtypes = [_p8, ctypes.c_int, _p8, ctypes.c_uint64, _p8, _p8, ctypes.c_uint64,
                                         ctypes.c_int]
        lib.oracle_ctr_crypt.restype = ctypes.c_int
        lib.oracle_cbc_encrypt.argtypes = [_p8, ctypes.c_int, _p8, _p8, _p8, ctypes.c_uint64]
        lib.oracle_cbc_encrypt.restype = ctypes.c_int
        lib.oracle_cbc_decrypt.argtypes = [_p8, ctypes.c_int, _p8, _p8, _p8, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_cbc_decrypt.restype = ctypes.c_int

    # -- field ------------------------------------------------------------
    def xtime(self, a: int) -> int:
        return int(self._lib.oracle_xtime(a))

    def gf_mul(self, a: int, b: int) -> int:
        return int(self._lib.oracle_gf_mul(a, b))

    def gf_inv(self, a: int) -> int:
        return int(self._lib.oracle_gf_inv(a))

    def gf_mul_table(self) -> np.ndarray:
        out = np.zeros(65536, dtype=np.uint8)
        self._lib.oracle_gf_mul_table(_ptr(out))
        return out.reshape(256, 256)

    # -- tables -----------------------------------------------------------
    def _table(self, name: str, n: int) -> np.ndarray:
        out = np.zeros(n, dtype=np.uint8)
        getattr(self._lib, name)(_ptr(out))
        return out

    def sbox(self) -> np.ndarray:
        return self._table("oracle_sbox", 256)

    def inv_sbox(self) -> np.ndarray:
        return self._table("oracle_inv_sbox", 256)

    def mix_matrix(self) -> np.ndarray:
        return self._table("oracle_mix_matrix", 16).reshape(4, 4)

    def inv_mix_matrix(self) -> np.ndarray:
        return self._table("oracle_inv_mix_matrix", 16).reshape(4, 4)

    # -- single-block transforms (input byte order) -----------------------
    def _block_op(self, name: str, block) -> bytes:
        buf = np.frombuffer(bytes(block), dtype=np.uint8).copy()
        assert buf.size == 16
        getattr(self._lib, name)(_ptr(buf))
        return buf.tobytes()

    def sub_bytes(self, b): return self._block_op("oracle_sub_bytes", b)
    def inv_sub_bytes(self, b): return self._block_op("oracle_inv_sub_bytes", b)
    def shift_rows(self, b): return self._block_op("oracle_shift_rows", b)
    def inv_shift_rows(self, b): return self._block_op("oracle_inv_shift_rows", b)
    def mix_columns(self, b): return self._block_op("oracle_mix_columns", b)
    def inv_mix_columns(self, b): return self._block_op("oracle_inv_mix_columns", b)

    def add_round_key(self, block, rk) -> bytes:
        buf = np.frombuffer(bytes(block), dtype=np.uint8).copy()
        k = np.frombuffer(bytes(rk), dtype=np.uint8).copy()
        self._lib.oracle_add_round_key(_ptr(buf), _ptr(k))
        return buf.tobytes()

    # -- key schedule and ECB ---------------------------------------------
    def expand_key(self, key: bytes, keybits: int | None = None):
        """Returns (schedule bytes, Nr); the schedule is 16*(Nr+1) bytes."""
        keybits = 8 * len(key) if keybits is None else keybits
        k = np.frombuffer(bytes(key), dtype=np.uint8).copy()
        out = np.zeros(240, dtype=np.uint8)
        nr = ctypes.c_int(0)
        rc = self._lib.oracle_expand_key(_ptr(k), keybits, _ptr(out), ctypes.byref(nr))
        if rc != 0:
            raise ValueError("bad key size %r" % keybits)
        return out[: 16 * (nr.value + 1)].tobytes(), nr.value

    def _ecb(self, name, key, data, nthreads):
        key = bytes(key)
        src = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray, memoryview)) else data, dtype=np.uint8).reshape(-1)
        if src.size % 16:
            raise ValueError("ECB input must be whole 16-byte blocks")
        out = np.empty_like(src)
        k = np.frombuffer(key, dtype=np.uint8).copy()
        nthreads = nthreads or (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
        rc = getattr(self._lib, name)(_ptr(k), 8 * len(key), _ptr(src), _ptr(out), src.size // 16, int(nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the key (%d bytes)" % len(key))
        return out

    def ecb_encrypt(self, key: bytes, data, nthreads: int | None = None) -> np.ndarray:
        """AES ECB encryption of whole blocks; returns a uint8 array."""
        return self._ecb("oracle_ecb_encrypt", key, data, nthreads)

    def ecb_decrypt(self, key: bytes, data, nthreads: int | None = None) -> np.ndarray:
        return self._ecb("oracle_ecb_decrypt", key, data, nthreads)

    def ctr_crypt(self, key: bytes, iv: bytes, data, offset: int = 0, nthreads: int | None = None) -> np.ndarray:
        """AES CTR of any number of bytes (encryption and decryption are the
        same); data block j uses counter iv + offset + j, 128-bit big-endian."""
        key, iv = bytes(key), bytes(iv)
        if len(iv) != 16:
            raise ValueError("the counter block is 16 bytes")
        src = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray, memoryview)) else data, dtype=np.uint8).reshape(-1)
        out = np.empty_like(src)
        k = np.frombuffer(key, dtype=np.uint8).copy()
        c = np.frombuffer(iv, dtype=np.uint8).copy()
        nthreads = nthreads or (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
        rc = self._lib.oracle_ctr_crypt(_ptr(k), 8 * len(key), _ptr(c), int(offset) & (2**64 - 1), _ptr(src),
                                        _ptr(out), src.size, int(nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the key (%d bytes)" % len(key))
        return out

    def _cbc_args(self, key, iv, data):
        key, iv = bytes(key), bytes(iv)
        if len(iv) != 16:
            raise ValueError("the initialisation vector is 16 bytes")
        src = np.ascontiguousarray(np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray, memoryview)) else data, dtype=np.uint8).reshape(-1)
        if src.size % 16:
            raise ValueError("CBC input must be whole 16-byte blocks")
        return (np.frombuffer(key, dtype=np.uint8).copy(), np.frombuffer(iv, dtype=np.uint8).copy(), src,
                np.empty_like(src))

    def cbc_encrypt(self, key: bytes, iv: bytes, data) -> np.ndarray:
        """CBC encryption (sequential) of whole blocks."""
        k, c, src, out = self._cbc_args(key, iv, data)
        rc = self._lib.oracle_cbc_encrypt(_ptr(k), 8 * k.size, _ptr(c), _ptr(src), _ptr(out), src.size // 16)
        if rc != 0:
            raise ValueError("oracle rejected the key (%d bytes)" % k.size)
        return out

    def cbc_decrypt(self, key: bytes, iv: bytes, data, nthreads: int | None = None) -> np.ndarray:
        """CBC decryption of whole blocks (threaded over block ranges)."""
        k, c, src, out = self._cbc_args(key, iv, data)
        nthreads = nthreads or (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
        rc = self._lib.oracle_cbc_decrypt(_ptr(k), 8 * k.size, _ptr(c), _ptr(src), _ptr(out), src.size // 16,
                                          int(nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the key (%d bytes)" % k.size)
        return out


_default = None
_lock = threading.Lock()


def load() -> Oracle:
    """The oracle built from ``aes_oracle.c`` (compiled with gcc on first use)."""
    global _default
    with _lock:
        if _default is None:
            if _build.is_stale():
                _build.build()
            _default = Oracle(_build.LIBRARY)
        return _default
