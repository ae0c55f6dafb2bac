"""The benchmark's measurement arithmetic, on the CPU with synthetic timings:
the published roofs, the algorithmic work per block, and the roofline object
bench.py prints (achieved = lookups per launch / mean launch time, frac =
achieved / peak)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_published_roofs(bench):
    assert bench.LDS_PEAK == pytest.approx(256 * 32 * 2.4e9)          # 19.66 T lookups/s
    assert bench.VALU_PEAK == pytest.approx(78.6e12, rel=1e-3)        # half the fp32 vector FLOP rate
    assert bench.HBM_PEAK_BPS == 8.0e12


def test_work_per_block(bench):
    assert [bench.lookups_per_block(n) for n in (10, 12, 14)] == [160, 192, 224]
    assert [bench.valu_floor_per_block(n) for n in (10, 12, 14)] == [252, 300, 348]


def test_roofline_object(bench):
    from paper_1902_05234_amd import aes
    nblocks = bench.GiB // 16
    b = {"nbytes": bench.GiB, "enc_ms": [0.70, 0.74, 0.72], "dec_ms": [0.73]}
    r = bench.roofline(b, 2.1478e9, aes)
    t = 0.72e-3
    lookups = 160 * nblocks
    assert r["bound"] == "lds" and r["unit"] == "Glookup/s" and r["traffic"] == 2.1478e9
    assert r["per_launch"]["blocks"] == nblocks and r["per_launch"]["lookups"] == lookups
    assert r["per_launch"]["hbm_bytes_algorithmic"] == 32 * nblocks
    assert r["achieved"] == pytest.approx(lookups / t / 1e9, rel=1e-3)
    assert r["peak"] == pytest.approx(19660.8, rel=1e-4)
    assert r["frac"] == pytest.approx(lookups / t / bench.LDS_PEAK, abs=1e-4)
    assert r["roofs"]["hbm"]["achieved_GB_s"] == pytest.approx(32 * nblocks / t / 1e9, rel=1e-3)
    assert r["roofs"]["payload_roof_GB_s"] == pytest.approx(bench.LDS_PEAK * 16 / 160 / 1e9, rel=1e-3)
    # decryption is reported beside encryption, with the same lookups per block
    td = 0.73e-3
    assert r["decrypt"]["achieved"] == pytest.approx(lookups / td / 1e9, rel=1e-3)
    assert r["decrypt"]["frac"] == pytest.approx(lookups / td / bench.LDS_PEAK, abs=1e-4)
    assert r["per_launch"]["mean_ms"] == pytest.approx(0.72) and r["per_launch"]["median_ms"] == 0.72
    assert r["per_launch"]["launches"] == 3 and r["decrypt"]["launches"] == 1
