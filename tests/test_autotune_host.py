"""Host-side logic of the autotuner (CPU): the sizes timed for each tuning
bucket lie in that bucket, and a bucket's winner is the variant with the best
worst-case ratio to the fastest variant over the bucket's sizes."""
from paper_1902_05234_amd import aes, autotune


def test_bucket_sizes_lie_in_their_buckets():
    assert len(autotune.BUCKET_SIZES) == aes.AES_SIZE_BUCKETS
    for b, sizes in enumerate(autotune.BUCKET_SIZES):
        assert sizes and all(n % 16 == 0 for n in sizes)
        assert {aes.aes_size_bucket(n // 16) for n in sizes} == {b}


def _row(bpt, wg, pl, gbs):
    return {"bpt": bpt, "wg": wg, "placement": pl, "GB_s": gbs, "ms": 1.0 / gbs}


def test_bucket_winner_maximises_the_worst_ratio():
    # v1 wins the large size, v2 is close there but far ahead at the small one
    per_size = {
        2 << 20: [_row(2, 1024, 1, 100.0), _row(1, 1024, 1, 50.0), _row(1, 512, 2, 80.0)],
        8 << 20: [_row(2, 1024, 1, 90.0), _row(1, 1024, 1, 100.0), _row(1, 512, 2, 60.0)],
    }
    w = autotune.bucket_winner(per_size)
    assert (w["bpt"], w["wg"], w["placement"]) == (2, 1024, 1)
    assert abs(w["worst_ratio"] - 0.9) < 1e-9


def test_bucket_winner_ignores_variants_missing_at_some_size():
    per_size = {
        1 << 20: [_row(1, 512, 2, 100.0), _row(4, 1024, 0, 99.0)],
        2 << 20: [_row(1, 512, 2, 100.0)],
    }
    w = autotune.bucket_winner(per_size)
    assert (w["bpt"], w["wg"], w["placement"]) == (1, 512, 2)


def test_source_hashes_cover_the_tuned_kernels_and_their_headers():
    """The record's plain hash reads the plain kernels and every csrc header
    they include, its batch hash the batched kernel's, and nothing else:
    device code the record does not time (CTR, CBC, probes) can change
    without voiding it, and the batched kernel can change without voiding
    the plain timings."""
    import os
    import re
    from paper_1902_05234_amd import autotune
    csrc = os.path.join(os.path.dirname(autotune.__file__), "csrc")
    for kernels in (autotune.PLAIN_KERNELS, autotune.BATCH_KERNELS):
        files = autotune.tuned_sources(kernels)
        assert set(kernels) <= set(files)
        for f in files:  # closed under local includes
            for inc in re.findall(r'^\s*#\s*include\s+"([^"/]+)"', open(os.path.join(csrc, f)).read(), re.M):
                assert inc in files, (f, inc)
        for other in ("aes_ctr.hip", "aes_cbc.hip", "aes_microbench.hip", "aes_abi.cpp", "aes_serve.cpp"):
            assert other not in files
    assert "aes_batch.hip" not in autotune.tuned_sources()
    os.makedirs(os.path.join(csrc, "__pycache__"), exist_ok=True)
    h = autotune.source_hash()
    assert len(h) == 16 and int(h, 16) >= 0 and h != autotune.source_hash(autotune.BATCH_KERNELS)
    assert autotune.source_hash() == h