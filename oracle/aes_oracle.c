/*
 * aes_oracle.c -- plain CPU oracle for AES-128/192/256 ECB.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, table or generator with
 * the GPU library.
 *
 * What it computes: AES as defined byte by byte, with GF(2^8) arithmetic done
 * by shift-and-conditional-XOR, never with the T-table shortcut the GPU path
 * uses.  Section references are to Wang & Chu, "GPU Accelerated AES
 * Algorithm" (arXiv:1902.05234); where that paper leaves a step out, the step
 * follows the AES standard (FIPS-197), which the paper names as Rijndael
 * (section 3.2).
 *
 *   - field element = polynomial over GF(2) stored as a byte      (sec 3.2.1, eq 6)
 *   - addition = XOR                                               (Def. 1, eq 7)
 *   - xtime = shift plus conditional XOR with m(x) = 0x11B         (Def. 3, eqs 8, 15-17)
 *   - multiplication = repeated xtime over the bits of one factor  (Def. 2, eqs 9-14)
 *   - inverse = a^254, square-and-multiply; inverse(0) = 0         (FIPS-197 5.1.1)
 *   - S-box = affine map of the inverse, constant 0x63             (Def. 4; FIPS-197 5.1.1)
 *   - state s[r][c] = in[r + 4c]                                   (FIPS-197 3.4)
 *   - ShiftRows s'[r][c] = s[r][(r + c) mod 4]                     (Def. 5, eq 19)
 *   - MixColumns: column <- A x column, A = circ(02,03,01,01)      (Def. 6, eq 20)
 *   - InvMixColumns: A^-1 found by Gauss-Jordan elimination on A over GF(2^8)
 *   - AddRoundKey: state XOR round key                             (Def. 7, eq 21)
 *   - key expansion: 4(Nr+1) words, Nb words per round key        (sec 3.2.2; FIPS-197 5.2)
 *   - Cipher: one initial AddRoundKey, Nr-1 full rounds, final round without
 *     MixColumns (Algorithm 1 read as the standard's Cipher)
 *   - InvCipher: the standard's straightforward inverse, using the ENCRYPTION
 *     schedule (FIPS-197 5.3), deliberately not the equivalent-inverse form
 *   - ECB: every block independent                                 (sec 3.1.1, eq 1)
 *
 * Blocks are shared out to threads in contiguous ranges; that changes nothing
 * about the result because ECB blocks are independent.
 *
 * Parity is pinned by the test suite: the paper's worked field examples,
 * field axioms checked exhaustively, S-box invariants, an independent
 * known-answer implementation (the OpenSSL command-line tool) on seeded keys
 * and data, and a round trip (tests/pins.py); tests/test_oracle_mutants.py
 * shows each of those pins catches planted mistakes.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)

/* ---------------------------------------------------------------- GF(2^8) */

/* Multiplication by x (Def. 3): shift left one place; if a term x^8 appears,
 * reduce it with m(x) = x^8 + x^4 + x^3 + x + 1 (eq 8), i.e. XOR 0x1B. */
static uint8_t gf_xtime(uint8_t a)
{
    return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1B : 0x00));
}

/* Multiplication (Def. 2): a * b = XOR over the set bits i of b of x^i * a,
 * each power obtained by repeated xtime. */
static uint8_t gf_mul(uint8_t a, uint8_t b)
{
    uint8_t acc = 0;
    for (int i = 0; i < 8; ++i) {
        if (b & (1u << i))
            acc ^= a;
        a = gf_xtime(a);
    }
    return acc;
}

/* Multiplicative inverse: a^254 = a^-1 for a != 0 since the multiplicative
 * group has order 255; 0 maps to 0. */
static uint8_t gf_inv(uint8_t a)
{
    uint8_t result = 1, base = a;
    unsigned e = 254;
    while (e) {
        if (e & 1u)
            result = gf_mul(result, base);
        base = gf_mul(base, base);
        e >>= 1;
    }
    return result;
}

/* ------------------------------------------------------------------ S-box */

static uint8_t bit(uint8_t v, int i) { return (uint8_t)((v >> (i & 7)) & 1u); }

/* Affine map over GF(2): b'_i = b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i
 * (indices mod 8), c = 0x63. */
static uint8_t affine(uint8_t b)
{
    const uint8_t c = 0x63;
    uint8_t out = 0;
    for (int i = 0; i < 8; ++i) {
        uint8_t v = bit(b, i) ^ bit(b, i + 4) ^ bit(b, i + 5) ^ bit(b, i + 6) ^ bit(b, i + 7) ^ bit(c, i);
        out |= (uint8_t)(v << i);
    }
    return out;
}

static uint8_t SBOX[256];
static uint8_t INV_SBOX[256];
static uint8_t INV_MIX[4][4];

/* MixColumns matrix of eq 20, rows as printed. */
static const uint8_t MIX[4][4] = {
    {0x02, 0x03, 0x01, 0x01},
    {0x01, 0x02, 0x03, 0x01},
    {0x01, 0x01, 0x02, 0x03},
    {0x03, 0x01, 0x01, 0x02},
};

/* Gauss-Jordan elimination over GF(2^8) on [A | I]; leaves A^-1 in INV_MIX. */
static void invert_mix_matrix(void)
{
    uint8_t m[4][8];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 8; ++c)
            m[r][c] = (c < 4) ? MIX[r][c] : (uint8_t)((c - 4) == r);
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        while (m[piv][col] == 0)
            ++piv; /* A is invertible, so a pivot exists */
        if (piv != col)
            for (int c = 0; c < 8; ++c) {
                uint8_t t = m[col][c];
                m[col][c] = m[piv][c];
                m[piv][c] = t;
            }
        uint8_t scale = gf_inv(m[col][col]);
        for (int c = 0; c < 8; ++c)
            m[col][c] = gf_mul(m[col][c], scale);
        for (int r = 0; r < 4; ++r) {
            if (r == col || m[r][col] == 0)
                continue;
            uint8_t f = m[r][col];
            for (int c = 0; c < 8; ++c)
                m[r][c] ^= gf_mul(f, m[col][c]);
        }
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            INV_MIX[r][c] = m[r][c + 4];
}

static pthread_once_t init_once = PTHREAD_ONCE_INIT;

static void init_tables(void)
{
    for (int a = 0; a < 256; ++a)
        SBOX[a] = affine(gf_inv((uint8_t)a));
    for (int a = 0; a < 256; ++a)
        INV_SBOX[SBOX[a]] = (uint8_t)a;
    invert_mix_matrix();
}

static void ensure_init(void) { pthread_once(&init_once, init_tables); }

/* ---------------------------------------------------------- state transforms */

typedef uint8_t state_t[4][4]; /* [row][column] */

static void load_state(state_t s, const uint8_t in[16])
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            s[r][c] = in[r + 4 * c];
}

static void store_state(uint8_t out[16], state_t s)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            out[r + 4 * c] = s[r][c];
}

/* Def. 4, eq 18 */
static void sub_bytes(state_t s)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            s[r][c] = SBOX[s[r][c]];
}

static void inv_sub_bytes(state_t s)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            s[r][c] = INV_SBOX[s[r][c]];
}

/* Def. 5, eq 19: s'[r][c] = s[r][(r + c) mod 4] */
static void shift_rows(state_t s)
{
    state_t t;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            t[r][c] = s[r][(r + c) % 4];
    memcpy(s, t, sizeof(t));
}

/* inverse of eq 19: s'[r][(r + c) mod 4] = s[r][c] */
static void inv_shift_rows(state_t s)
{
    state_t t;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            t[r][(r + c) % 4] = s[r][c];
    memcpy(s, t, sizeof(t));
}

/* column <- M x column over GF(2^8) */
static void mat_columns(state_t s, const uint8_t m[4][4])
{
    for (int c = 0; c < 4; ++c) {
        uint8_t col[4], res[4];
        for (int r = 0; r < 4; ++r)
            col[r] = s[r][c];
        for (int r = 0; r < 4; ++r) {
            uint8_t acc = 0;
            for (int k = 0; k < 4; ++k)
                acc ^= gf_mul(m[r][k], col[k]);
            res[r] = acc;
        }
        for (int r = 0; r < 4; ++r)
            s[r][c] = res[r];
    }
}

/* Def. 6, eq 20 */
static void mix_columns(state_t s) { mat_columns(s, MIX); }
static void inv_mix_columns(state_t s) { mat_columns(s, (const uint8_t(*)[4])INV_MIX); }

/* Def. 7, eq 21. rk points at the 16 bytes of one round key, which are the
 * 4 schedule words in order, each word = one state column top to bottom. */
static void add_round_key(state_t s, const uint8_t *rk)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            s[r][c] ^= rk[4 * c + r];
}

/* ------------------------------------------------------------ key schedule */

static int rounds_for(int keybits)
{
    switch (keybits) {
    case 128: return 10;
    case 192: return 12;
    case 256: return 14;
    default: return -1;
    }
}

/* Key expansion into 4(Nr+1) four-byte words w[0..], stored as bytes
 * (w[i] = out[4i..4i+3]).  Section 3.2.2 fixes only the sizes and that round
 * key k is words Nb*k .. Nb*k+Nb-1; the recurrence is FIPS-197 5.2. */
static int expand_key(const uint8_t *key, int keybits, uint8_t *w, int *nr_out)
{
    int nr = rounds_for(keybits);
    if (nr < 0 || key == NULL || w == NULL)
        return ORACLE_EINVAL;
    ensure_init();
    const int nk = keybits / 32;
    const int total = 4 * (nr + 1);
    memcpy(w, key, (size_t)(4 * nk));
    uint8_t rcon = 0x01;
    for (int i = nk; i < total; ++i) {
        uint8_t temp[4];
        memcpy(temp, w + 4 * (i - 1), 4);
        if (i % nk == 0) {
            /* RotWord, SubWord, then XOR (Rcon, 0, 0, 0) */
            uint8_t t0 = temp[0];
            temp[0] = SBOX[temp[1]];
            temp[1] = SBOX[temp[2]];
            temp[2] = SBOX[temp[3]];
            temp[3] = SBOX[t0];
            temp[0] ^= rcon;
            rcon = gf_xtime(rcon);
        } else if (nk == 8 && i % nk == 4) {
            for (int b = 0; b < 4; ++b)
                temp[b] = SBOX[temp[b]];
        }
        for (int b = 0; b < 4; ++b)
            w[4 * i + b] = (uint8_t)(w[4 * (i - nk) + b] ^ temp[b]);
    }
    if (nr_out)
        *nr_out = nr;
    return ORACLE_OK;
}

/* ------------------------------------------------------------ block cipher */

static void cipher_block(const uint8_t *w, int nr, const uint8_t in[16], uint8_t out[16])
{
    state_t s;
    load_state(s, in);
    add_round_key(s, w);
    for (int round = 1; round < nr; ++round) {
        sub_bytes(s);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w + 16 * round);
    }
    sub_bytes(s);
    shift_rows(s);
    add_round_key(s, w + 16 * nr);
    store_state(out, s);
}

static void inv_cipher_block(const uint8_t *w, int nr, const uint8_t in[16], uint8_t out[16])
{
    state_t s;
    load_state(s, in);
    add_round_key(s, w + 16 * nr);
    for (int round = nr - 1; round >= 1; --round) {
        inv_shift_rows(s);
        inv_sub_bytes(s);
        add_round_key(s, w + 16 * round);
        inv_mix_columns(s);
    }
    inv_shift_rows(s);
    inv_sub_bytes(s);
    add_round_key(s, w);
    store_state(out, s);
}

/* ------------------------------------------------------------- ECB driver */

typedef struct {
    const uint8_t *w;
    int nr;
    int decrypt;
    const uint8_t *in;
    uint8_t *out;
    uint64_t first, count;
} ecb_job;

static void *ecb_worker(void *arg)
{
    const ecb_job *j = (const ecb_job *)arg;
    for (uint64_t b = j->first; b < j->first + j->count; ++b) {
        uint8_t tmp[16];
        if (j->decrypt)
            inv_cipher_block(j->w, j->nr, j->in + 16 * b, tmp);
        else
            cipher_block(j->w, j->nr, j->in + 16 * b, tmp);
        memcpy(j->out + 16 * b, tmp, 16); /* tmp allows in == out */
    }
    return NULL;
}

static int ecb(const uint8_t *key, int keybits, const uint8_t *in, uint8_t *out,
               uint64_t nblocks, int nthreads, int decrypt)
{
    uint8_t w[16 * 15];
    int nr;
    if (expand_key(key, keybits, w, &nr) != ORACLE_OK)
        return ORACLE_EINVAL;
    if (nblocks == 0)
        return ORACLE_OK;
    if (in == NULL || out == NULL)
        return ORACLE_EINVAL;
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > nblocks)
        nthreads = (int)nblocks;
    ecb_job *jobs = (ecb_job *)calloc((size_t)nthreads, sizeof(ecb_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return ORACLE_EINVAL;
    }
    uint64_t per = nblocks / (uint64_t)nthreads, extra = nblocks % (uint64_t)nthreads, next = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t cnt = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (ecb_job){w, nr, decrypt, in, out, next, cnt};
        next += cnt;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tid[t], NULL, ecb_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    ecb_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tid[t], NULL);
    /* any range whose thread could not be started runs here */
    for (int t = started + 1; t < nthreads; ++t)
        ecb_worker(&jobs[t]);
    free(jobs);
    free(tid);
    return ORACLE_OK;
}

/* ------------------------------------------------------------- CTR driver
 *
 * Counter mode (section 3.1.5, eq 5): block i of the output is block i of
 * the input XOR the cipher of a counter block, and counter blocks of
 * successive data blocks are successive integers.  Reading of the paper's
 * counter (its range for R is garbled): the counter block is one 128-bit
 * big-endian integer, data block j (counted from 0) uses iv + offset + j
 * modulo 2^128, so the paper's R is iv + offset - 1.  A partial last block
 * uses the leading bytes of its key-stream block.  Decryption is the same
 * operation.
 */

/* out = c + add (mod 2^128), both big-endian, one byte at a time */
static void counter_add(const uint8_t c[16], uint64_t add, uint8_t out[16])
{
    unsigned carry = 0;
    for (int i = 15; i >= 0; --i) {
        unsigned v = (unsigned)c[i] + (unsigned)(add & 0xffu) + carry;
        out[i] = (uint8_t)(v & 0xffu);
        carry = v >> 8;
        add >>= 8;
    }
}

typedef struct {
    const uint8_t *w;
    int nr;
    const uint8_t *ctr0; /* counter of data block 0 */
    const uint8_t *in;
    uint8_t *out;
    uint64_t nbytes;
    uint64_t first, count; /* block range */
} ctr_job;

static void *ctr_worker(void *arg)
{
    const ctr_job *j = (const ctr_job *)arg;
    const uint64_t end = j->first + j->count;
    for (uint64_t b = j->first; b < end; ++b) {
        uint8_t ctr[16], ks[16];
        counter_add(j->ctr0, b, ctr);
        cipher_block(j->w, j->nr, ctr, ks);
        uint64_t n = j->nbytes - 16 * b;
        if (n > 16)
            n = 16;
        for (uint64_t k = 0; k < n; ++k)
            j->out[16 * b + k] = (uint8_t)(j->in[16 * b + k] ^ ks[k]);
    }
    return NULL;
}

static int ctr(const uint8_t *key, int keybits, const uint8_t iv[16], uint64_t offset, const uint8_t *in,
               uint8_t *out, uint64_t nbytes, int nthreads)
{
    uint8_t w[16 * 15], ctr0[16];
    int nr;
    if (expand_key(key, keybits, w, &nr) != ORACLE_OK || iv == NULL)
        return ORACLE_EINVAL;
    if (nbytes == 0)
        return ORACLE_OK;
    if (in == NULL || out == NULL)
        return ORACLE_EINVAL;
    counter_add(iv, offset, ctr0);
    uint64_t nblocks = (nbytes + 15) / 16;
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > nblocks)
        nthreads = (int)nblocks;
    ctr_job *jobs = (ctr_job *)calloc((size_t)nthreads, sizeof(ctr_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return ORACLE_EINVAL;
    }
    uint64_t per = nblocks / (uint64_t)nthreads, extra = nblocks % (uint64_t)nthreads, next = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t cnt = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (ctr_job){w, nr, ctr0, in, out, nbytes, next, cnt};
        next += cnt;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tid[t], NULL, ctr_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    ctr_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tid[t], NULL);
    for (int t = started + 1; t < nthreads; ++t)
        ctr_worker(&jobs[t]);
    free(jobs);
    free(tid);
    return ORACLE_OK;
}

/* ------------------------------------------------------------- CBC driver
 *
 * Cipher block chaining (section 3.1.2, eq 2).  The printed equation lacks
 * the block cipher; the reading is the standard chain: C_i = cipher(P_i XOR
 * C_{i-1}) with C_0 the initialisation vector, so decryption is P_i =
 * invcipher(C_i) XOR C_{i-1}.  Encryption is sequential by definition and
 * runs block after block on one thread; decryption of each block needs only
 * two ciphertext blocks and is threaded over block ranges.  Whole blocks
 * only.
 */
static int cbc_encrypt(const uint8_t *key, int keybits, const uint8_t iv[16], const uint8_t *in, uint8_t *out,
                       uint64_t nblocks)
{
    uint8_t w[16 * 15], chain[16];
    int nr;
    if (expand_key(key, keybits, w, &nr) != ORACLE_OK || iv == NULL)
        return ORACLE_EINVAL;
    if (nblocks == 0)
        return ORACLE_OK;
    if (in == NULL || out == NULL)
        return ORACLE_EINVAL;
    memcpy(chain, iv, 16);
    for (uint64_t b = 0; b < nblocks; ++b) {
        uint8_t x[16];
        for (int k = 0; k < 16; ++k)
            x[k] = (uint8_t)(in[16 * b + k] ^ chain[k]);
        cipher_block(w, nr, x, chain);
        memcpy(out + 16 * b, chain, 16);
    }
    return ORACLE_OK;
}

typedef struct {
    const uint8_t *w;
    int nr;
    const uint8_t *iv;
    const uint8_t *in;
    uint8_t *out;
    uint64_t first, count;
} cbc_job;

static void *cbc_dec_worker(void *arg)
{
    const cbc_job *j = (const cbc_job *)arg;
    const uint64_t stop = j->first + j->count;
    for (uint64_t b = j->first; b < stop; ++b) {
        uint8_t x[16];
        const uint8_t *prev = b == 0 ? j->iv : j->in + 16 * (b - 1);
        inv_cipher_block(j->w, j->nr, j->in + 16 * b, x);
        for (int k = 0; k < 16; ++k)
            j->out[16 * b + k] = (uint8_t)(x[k] ^ prev[k]);
    }
    return NULL;
}

static int cbc_decrypt(const uint8_t *key, int keybits, const uint8_t iv[16], const uint8_t *in, uint8_t *out,
                       uint64_t nblocks, int nthreads)
{
    uint8_t w[16 * 15];
    int nr;
    if (expand_key(key, keybits, w, &nr) != ORACLE_OK || iv == NULL)
        return ORACLE_EINVAL;
    if (nblocks == 0)
        return ORACLE_OK;
    if (in == NULL || out == NULL || in == out)
        return ORACLE_EINVAL; /* block b reads ciphertext block b - 1: no in-place */
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > nblocks)
        nthreads = (int)nblocks;
    cbc_job *jobs = (cbc_job *)calloc((size_t)nthreads, sizeof(cbc_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return ORACLE_EINVAL;
    }
    uint64_t per = nblocks / (uint64_t)nthreads, extra = nblocks % (uint64_t)nthreads, next = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t cnt = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t] = (cbc_job){w, nr, iv, in, out, next, cnt};
        next += cnt;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tid[t], NULL, cbc_dec_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    cbc_dec_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tid[t], NULL);
    for (int t = started + 1; t < nthreads; ++t)
        cbc_dec_worker(&jobs[t]);
    free(jobs);
    free(tid);
    return ORACLE_OK;
}

/* ---------------------------------------------------------- exported API */

uint8_t oracle_xtime(uint8_t a) { return gf_xtime(a); }
uint8_t oracle_gf_mul(uint8_t a, uint8_t b) { return gf_mul(a, b); }
uint8_t oracle_gf_inv(uint8_t a) { return gf_inv(a); }

/* full 256 x 256 product table, out[256*a + b] = a*b */
void oracle_gf_mul_table(uint8_t *out)
{
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b)
            out[256 * a + b] = gf_mul((uint8_t)a, (uint8_t)b);
}

void oracle_sbox(uint8_t out[256])
{
    ensure_init();
    memcpy(out, SBOX, 256);
}

void oracle_inv_sbox(uint8_t out[256])
{
    ensure_init();
    memcpy(out, INV_SBOX, 256);
}

void oracle_mix_matrix(uint8_t out[16]) { memcpy(out, MIX, 16); }

void oracle_inv_mix_matrix(uint8_t out[16])
{
    ensure_init();
    memcpy(out, INV_MIX, 16);
}

/* single transforms on one 16-byte block in input byte order */
#define ORACLE_BLOCK_OP(name, body)                                              \
    void name(uint8_t blk[16])                                                   \
    {                                                                            \
        state_t s;                                                               \
        ensure_init();                                                           \
        load_state(s, blk);                                                      \
        body(s);                                                                 \
        store_state(blk, s);                                                     \
    }
ORACLE_BLOCK_OP(oracle_sub_bytes, sub_bytes)
ORACLE_BLOCK_OP(oracle_inv_sub_bytes, inv_sub_bytes)
ORACLE_BLOCK_OP(oracle_shift_rows, shift_rows)
ORACLE_BLOCK_OP(oracle_inv_shift_rows, inv_shift_rows)
ORACLE_BLOCK_OP(oracle_mix_columns, mix_columns)
ORACLE_BLOCK_OP(oracle_inv_mix_columns, inv_mix_columns)

void oracle_add_round_key(uint8_t blk[16], const uint8_t rk[16])
{
    state_t s;
    load_state(s, blk);
    add_round_key(s, rk);
    store_state(blk, s);
}

/* w_out: 16*(Nr+1) bytes (at most 240). Returns 0, or -1 for a bad keybits. */
int oracle_expand_key(const uint8_t *key, int keybits, uint8_t *w_out, int *nr)
{
    return expand_key(key, keybits, w_out, nr);
}

int oracle_ecb_encrypt(const uint8_t *key, int keybits, const uint8_t *in, uint8_t *out,
                       uint64_t nblocks, int nthreads)
{
    return ecb(key, keybits, in, out, nblocks, nthreads, 0);
}

int oracle_ecb_decrypt(const uint8_t *key, int keybits, const uint8_t *in, uint8_t *out,
                       uint64_t nblocks, int nthreads)
{
    return ecb(key, keybits, in, out, nblocks, nthreads, 1);
}

/* CTR encryption or decryption of nbytes (any length); counter of data
 * block j is iv + offset + j (128-bit big-endian, mod 2^128). */
int oracle_ctr_crypt(const uint8_t *key, int keybits, const uint8_t iv[16], uint64_t offset,
                     const uint8_t *in, uint8_t *out, uint64_t nbytes, int nthreads)
{
    return ctr(key, keybits, iv, offset, in, out, nbytes, nthreads);
}

/* CBC over nblocks whole blocks with initialisation vector iv (C_0). */
int oracle_cbc_encrypt(const uint8_t *key, int keybits, const uint8_t iv[16], const uint8_t *in, uint8_t *out,
                       uint64_t nblocks)
{
    return cbc_encrypt(key, keybits, iv, in, out, nblocks);
}

int oracle_cbc_decrypt(const uint8_t *key, int keybits, const uint8_t iv[16], const uint8_t *in, uint8_t *out,
                       uint64_t nblocks, int nthreads)
{
    return cbc_decrypt(key, keybits, iv, in, out, nblocks, nthreads);
}
