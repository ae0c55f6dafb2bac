"""The committed MI355X tuning record (paper_1902_05234_amd/tuning/
mi355x_sweep.json) was made on the library's current kernel sources, and
the library's compiled-in defaults are its winners: the generated default
table equals what the record produces, and aes_tune_get returns the
record's variant for every key size, direction and size bucket."""
import os

from paper_1902_05234_amd import aes, autotune


def _record():
    return autotune.load(autotune.RECORD)


def test_record_is_for_the_current_kernel_sources():
    rec = _record()
    assert rec["source_hash"] == autotune.source_hash(), (
        "the kernel sources changed since the record was made: re-run the autotuner on an MI355X")
    assert rec["batch"]["source_hash"] == autotune.source_hash(autotune.BATCH_KERNELS), (
        "the batched kernel changed since its entry was timed: re-run the autotuner with --batch-only")
    assert rec.get("arch", "").startswith("gfx950")


def test_generated_default_table_is_the_records():
    assert open(autotune.DEFAULTS_INC).read() == autotune.emit_defaults(_record())


def test_compiled_defaults_are_the_record_winners():
    w = autotune.winners(_record())
    assert len(w) == 3 * 2 * aes.AES_SIZE_BUCKETS
    for (nr, dec, bucket), want in w.items():
        for n in autotune.BUCKET_SIZES[bucket]:
            v = aes.aes_tune_get(nr, dec, n // 16)
            assert (v.bpt, v.wg, v.placement) == want, (nr, dec, bucket, n)


def test_largest_bucket_winner_was_timed_under_sustained_load():
    rec = _record()
    for k, v in rec["plain"].items():
        if max(v["sizes"]) > autotune.GRAPH_TIMED_MAX:
            rows = v["all"][str(max(v["sizes"]))]
            best = rows[0]
            assert best["timing"] == "sustained", k
            assert (best["bpt"], best["wg"], best["placement"]) == (
                v["winner"]["bpt"], v["winner"]["wg"], v["winner"]["placement"]), k


def test_record_has_a_batch_winner_from_the_full_search():
    rec = _record()
    chunk, cfg = autotune.batch_winner(rec)
    stale = dict(rec, batch=dict(rec["batch"], source_hash="0000000000000000"))
    assert autotune.batch_winner(stale) is None, "a batch entry timed on other sources is not used"
    assert chunk in autotune.BATCH_CHUNKS and cfg.placement in autotune.BATCH_PLACEMENTS
    seen = {(r["chunk_blocks"], r["bpt"], r["wg"], r["placement"]) for r in rec["batch"]["all"]}
    assert seen == {(c, v.bpt, v.wg, v.placement) for c, v in autotune.batch_variants()}


def test_record_mismatch_names_every_difference():
    rec = {"source_hash": "aaaa", "device": "dev A", "arch": "gfx950:sramecc+:xnack-", "hip": "7.0.1"}
    assert autotune.record_mismatch(rec, "dev A", "gfx950:sramecc+:xnack-", src_hash="aaaa", hip="7.0.1") == []
    why = autotune.record_mismatch(rec, "dev B", "gfx942", src_hash="bbbb", hip="6.4.0")
    assert len(why) == 4
    assert any("kernel sources" in w for w in why) and any("device" in w for w in why)
    assert any("architecture" in w for w in why) and any("HIP runtime" in w for w in why)
    # no device to compare with: only the sources are checked
    assert autotune.record_mismatch(rec, None, None, src_hash="aaaa") == []


def test_apply_refuses_a_record_for_other_sources_unless_forced():
    rec = dict(_record(), source_hash="0000000000000000")
    v0 = aes.aes_tune_get(10, False, 1 << 20)
    try:
        autotune.apply(rec)
    except autotune.RecordMismatch as e:
        assert "kernel sources" in str(e)
    else:
        raise AssertionError("a record for other kernel sources was installed")
    v1 = aes.aes_tune_get(10, False, 1 << 20)
    assert v1 == v0
    assert autotune.apply(rec, force=True) == 3 * 2 * aes.AES_SIZE_BUCKETS
