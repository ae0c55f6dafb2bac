"""MI355X-native AES-128/192/256 ECB (Wang & Chu, arXiv:1902.05234).

The compute path is the HIP library ``libaesgpu.so`` built from ``csrc/``;
``paper_1902_05234_amd.aes`` is its thin ctypes binding.  Importing this
package loads nothing: the library is opened on first use, and every entry
point raises if it is missing.
"""

__all__ = ["aes", "inputs"]
