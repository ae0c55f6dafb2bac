"""The plain entry points inside a captured HIP graph: ECB encrypt/decrypt
(every placement), CTR and CBC decryption are captured once and replayed
several times, with eager work and synchronisations between the replays;
every replay must equal the eager result (and the oracle)."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_plain_paths_replay_in_a_graph(oracle_lib):
    torch = cuda()
    key = inputs.random_key(950, 192)
    iv = inputs.random_bytes(951, 16).tobytes()
    ks = aes.aes_expand_key(key)
    n = 16 * 70001
    x = inputs.random_bytes(952, n)
    xd = to_dev(x)
    outs = {name: torch.empty_like(xd) for name in ("enc4", "enc2", "enc1", "encb", "encc", "dec", "ctr", "cbc")}
    cd = to_dev(oracle_lib.ecb_encrypt(key, x))
    cbc_in = to_dev(oracle_lib.cbc_encrypt(key, iv, x))

    def work():
        aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, xd, outs["enc4"], aes.Variant(bpt=4, wg=1024, placement=0))
        aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, xd, outs["enc2"], aes.Variant(bpt=2, wg=1024, placement=1))
        aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, xd, outs["enc1"], aes.Variant(bpt=1, wg=512, placement=2))
        aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, xd, outs["encb"], aes.Variant(bpt=1, wg=256, placement=3))
        aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, xd, outs["encc"],
                                  aes.Variant(bpt=aes.AES_BPT_COLUMN, wg=512, placement=1))
        aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, cd, outs["dec"])
        aes.aes_ctr_crypt(ks.rk_enc, ks.nr, iv, 5, xd, outs["ctr"])
        aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, iv, cbc_in, outs["cbc"])

    work()
    torch.cuda.synchronize()
    eager = {k: to_host(v).copy() for k, v in outs.items()}
    want_enc = oracle_lib.ecb_encrypt(key, x)
    for k in ("enc4", "enc2", "enc1", "encb", "encc"):
        assert first_mismatch(eager[k], want_enc) is None, k
    assert first_mismatch(eager["dec"], x) is None
    assert first_mismatch(eager["ctr"], oracle_lib.ctr_crypt(key, iv, x, offset=5)) is None
    assert first_mismatch(eager["cbc"], x) is None

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            work()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        for v in outs.values():
            v.zero_()                                   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert first_mismatch(to_host(v), eager[k]) is None, "replay %d, %s" % (rep, k)
    del g
