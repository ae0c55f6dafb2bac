"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle's source (a dropped term, a wrong constant, sign, index or operand
order) must make at least one pin fail.  Mutants are compiled on the CPU into
a temporary directory; the real oracle is never modified."""
import os

import pytest

import oracle
from oracle import build as obuild
from tests import pins

MUTANTS = [
    ("xtime_modulus", "((a & 0x80) ? 0x1B : 0x00)", "((a & 0x80) ? 0x1D : 0x00)"),
    ("mul_skips_top_bit", "for (int i = 0; i < 8; ++i) {\n        if (b & (1u << i))",
     "for (int i = 0; i < 7; ++i) {\n        if (b & (1u << i))"),
    ("inverse_exponent", "unsigned e = 254;", "unsigned e = 253;"),
    ("affine_dropped_term", "^ bit(b, i + 6) ^ bit(b, i + 7) ^ bit(c, i)", "^ bit(b, i + 6) ^ bit(c, i)"),
    ("affine_constant", "const uint8_t c = 0x63;", "const uint8_t c = 0x62;"),
    ("affine_rotation_sign", "bit(b, i) ^ bit(b, i + 4) ^ bit(b, i + 5) ^ bit(b, i + 6) ^ bit(b, i + 7)",
     "bit(b, i) ^ bit(b, i - 4) ^ bit(b, i - 5) ^ bit(b, i - 6) ^ bit(b, i - 7)"),
    ("mix_row_transposed", "{0x02, 0x03, 0x01, 0x01},\n    {0x01, 0x02, 0x03, 0x01},\n    {0x01, 0x01, 0x02, 0x03},\n    {0x03, 0x01, 0x01, 0x02},",
     "{0x02, 0x01, 0x01, 0x03},\n    {0x03, 0x02, 0x01, 0x01},\n    {0x01, 0x03, 0x02, 0x01},\n    {0x01, 0x01, 0x03, 0x02},"),
    ("state_map_transposed_consistently", "s[r][c] = in[r + 4 * c];", "s[r][c] = in[4 * r + c];"),
    ("shift_rows_direction_consistent", "t[r][c] = s[r][(r + c) % 4];", "t[r][c] = s[r][(c - r + 4) % 4];"),
    ("inv_shift_rows_only", "t[r][(r + c) % 4] = s[r][c];", "t[r][c] = s[r][(r + c) % 4];"),
    ("round_key_byte_order", "s[r][c] ^= rk[4 * c + r];", "s[r][c] ^= rk[4 * r + c];"),
    ("rcon_without_reduction", "rcon = gf_xtime(rcon);", "rcon = (uint8_t)(rcon << 1);"),
    ("rot_word_direction", "temp[0] = SBOX[temp[1]];\n            temp[1] = SBOX[temp[2]];\n            temp[2] = SBOX[temp[3]];\n            temp[3] = SBOX[t0];",
     "temp[0] = SBOX[temp[3]];\n            temp[3] = SBOX[temp[2]];\n            temp[2] = SBOX[temp[1]];\n            temp[1] = SBOX[t0];"),
    ("aes256_missing_subword", "} else if (nk == 8 && i % nk == 4) {", "} else if (nk == 8 && i % nk == 5) {"),
    ("rounds_192", "case 192: return 12;", "case 192: return 11;"),
    ("final_round_with_mixcolumns", "    sub_bytes(s);\n    shift_rows(s);\n    add_round_key(s, w + 16 * nr);",
     "    sub_bytes(s);\n    shift_rows(s);\n    mix_columns(s);\n    add_round_key(s, w + 16 * nr);"),
    ("inv_cipher_step_order", "add_round_key(s, w + 16 * round);\n        inv_mix_columns(s);",
     "inv_mix_columns(s);\n        add_round_key(s, w + 16 * round);"),
    ("inv_cipher_key_index", "add_round_key(s, w + 16 * nr);\n    for (int round = nr - 1;",
     "add_round_key(s, w + 16 * (nr - 1));\n    for (int round = nr - 1;"),
    ("ctr_counter_little_endian", "for (int i = 15; i >= 0; --i) {\n        unsigned v = (unsigned)c[i] + (unsigned)(add & 0xffu) + carry;\n        out[i]",
     "for (int i = 0; i < 16; ++i) {\n        unsigned v = (unsigned)c[i] + (unsigned)(add & 0xffu) + carry;\n        out[i]"),
    ("ctr_carry_dropped", "        carry = v >> 8;\n        add >>= 8;", "        carry = 0;\n        add >>= 8;"),
    ("ctr_partial_block_dropped", "        if (n > 16)\n            n = 16;", "        if (n < 16)\n            n = 0;\n        if (n > 16)\n            n = 16;"),
    ("ctr_offset_ignored", "counter_add(iv, offset, ctr0);", "counter_add(iv, 0, ctr0);"),
    ("ctr_first_block_counter_plus_one", "counter_add(j->ctr0, b, ctr);", "counter_add(j->ctr0, b + 1, ctr);"),
    ("cbc_chain_not_updated", "        cipher_block(w, nr, x, chain);\n        memcpy(out + 16 * b, chain, 16);",
     "        uint8_t y[16];\n        cipher_block(w, nr, x, y);\n        memcpy(out + 16 * b, y, 16);"),
    ("cbc_dec_xor_with_own_block", "const uint8_t *prev = b == 0 ? j->iv : j->in + 16 * (b - 1);",
     "const uint8_t *prev = b == 0 ? j->iv : j->in + 16 * b;"),
    ("cbc_dec_first_block_without_iv", "const uint8_t *prev = b == 0 ? j->iv : j->in + 16 * (b - 1);",
     "static const uint8_t zero16[16];\n        const uint8_t *prev = b == 0 ? zero16 : j->in + 16 * (b - 1);"),
    ("ecb_last_block_skipped", "for (uint64_t b = j->first; b < j->first + j->count; ++b) {",
     "for (uint64_t b = j->first; b + 1 < j->first + j->count; ++b) {"),
]


@pytest.mark.parametrize("name,orig,mutated", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, mutated):
    src = open(obuild.SOURCE).read()
    assert src.count(orig) == 1, "mutation anchor for %s must occur exactly once" % name
    path = tmp_path / ("mutant_%s.c" % name)
    path.write_text(src.replace(orig, mutated))
    lib = obuild.build(str(path), str(tmp_path / ("libmutant_%s.so" % name)), extra_flags=["-Wno-error"])
    o = oracle.Oracle(lib)
    failed = []
    for pin in pins.ALL_PINS:
        if pin in pins.OPENSSL_PINS and not pins.openssl_available():
            continue
        try:
            pin(o)
        except (AssertionError, ValueError, IndexError) as e:  # a pin caught it
            failed.append(pin.__name__)
            break
    assert failed, "mutant %s passed every pin" % name


def test_real_oracle_source_unchanged_by_mutants():
    assert os.path.exists(obuild.SOURCE)
    assert "MUTANT" not in open(obuild.SOURCE).read()
