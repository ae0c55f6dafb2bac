/*
 * aesgpu.h -- C ABI of libaesgpu: AES-128/192/256 ECB on AMD MI355X (gfx950).
 *
 * The operations follow Wang & Chu, "GPU Accelerated AES Algorithm"
 * (arXiv:1902.05234): ECB mode (section 3.1.1, eq 1) over whole 16-byte
 * blocks, one AES state per GPU thread (section 4.1), T-table rounds
 * (section 3.2.3, eqs 22-26), round keys from one cipher key (section 3.2.2,
 * Algorithm 1).  Where the paper is silent (key-expansion recurrence,
 * decryption tables, byte order) the library follows FIPS-197.
 *
 * Conventions
 *   - Every function returns an int status (AES_OK or a negative AES_E* code)
 *     and never aborts; aes_last_error() gives a message for the calling
 *     thread's last failure.
 *   - "device pointer" = memory of the current HIP device (hipMalloc, or a
 *     torch tensor's data_ptr()); "host pointer" = ordinary process memory.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  Device
 *     work is enqueued asynchronously on it; the call returns without waiting.
 *   - The caller owns every buffer it passes.  No entry point allocates or
 *     frees device memory.  Besides its immutable tables and the static
 *     scratch array of aes_ecb_batch_noalloc (both in the code object) and
 *     the tuning table set by aes_tune_set, the library holds only what a
 *     pipe or server handle creates (streams, events, a worker thread, the
 *     pipe's 256-byte pinned completion page), released by its destroy call.
 *   - A 16-byte block is processed byte-for-byte as FIPS-197's input array:
 *     byte r + 4c is state row r, column c.  No padding is applied: callers
 *     pass whole blocks.
 */
#ifndef AESGPU_H
#define AESGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AES_OK 0
#define AES_EINVAL (-1) /* bad argument: key size, Nr, null pointer, overlap */
#define AES_EALIGN (-2) /* buffer not 16-byte aligned */
#define AES_ENOMEM (-3) /* host memory for the serving engine's or pipe's bookkeeping ran out
                            (no entry point allocates device memory) */
#define AES_EHIP (-4)   /* HIP runtime or launch error */
#define AES_EBUSY (-5)  /* reserved for callers' admission control */
#define AES_ERANGE (-6) /* a count or capacity out of range */

#define AES_MAX_ROUND_KEY_WORDS 60 /* 4 * (14 + 1) */

/* Message for the calling thread's last non-OK status ("" if none). */
const char *aes_last_error(void);

/*
 * aes_expand_key -- key schedule (section 3.2.2; Algorithm 1 keyExpansion).
 *   key:     host pointer to keybits/8 bytes.
 *   keybits: 128, 192 or 256.
 *   rk_enc:  host array of >= 4*(Nr+1) uint32 (may be NULL): the expanded key;
 *            round key k is words 4k..4k+3 (Nb = 4 words per round key, so
 *            4*(10+1) words = 1408 bits for AES-128).  Word i holds key bytes
 *            4i..4i+3 little-endian (byte 4i in bits 0..7).
 *   rk_dec:  host array of >= 4*(Nr+1) uint32 (may be NULL): the schedule of
 *            the equivalent inverse cipher (FIPS-197 5.3.5): rk_dec round 0 =
 *            rk_enc round Nr, round Nr = rk_enc round 0, rounds 1..Nr-1 =
 *            InvMixColumns(rk_enc round Nr-r).
 *   nr:      receives Nr = 10/12/14 (may be NULL).
 * Host only, thread-safe.  AES_EINVAL for a bad keybits or NULL key.
 */
int aes_expand_key(const uint8_t *key, int keybits, uint32_t *rk_enc, uint32_t *rk_dec, int *nr);

/*
 * aes_ecb_encrypt / aes_ecb_decrypt -- ECB over nblocks whole blocks
 * (section 3.1.1, eq 1: C_i = cipher(P_i), each block independently).
 *   rk:      host pointer to the 4*(nr+1)-word schedule from aes_expand_key
 *            (rk_enc for encryption, rk_dec for decryption).  Copied into the
 *            launch, so it may be freed when the call returns.
 *   nr:      10, 12 or 14.
 *   in, out: device pointers, 16-byte aligned, nblocks*16 bytes each.
 *            in == out (in place) is allowed; any other overlap is AES_EINVAL.
 *   nblocks: number of 16-byte blocks; 0 is a no-op returning AES_OK.
 * The kernel variant comes from the tuning table (aes_tune_get/aes_tune_set),
 * one entry per key size, direction and size bucket.
 */
int aes_ecb_encrypt(const uint32_t *rk, int nr, const void *in, void *out, size_t nblocks, void *stream);
int aes_ecb_decrypt(const uint32_t *rk, int nr, const void *in, void *out, size_t nblocks, void *stream);

/* Kernel variant of the plain path (the autotuner's search space). */
#define AES_PLACEMENT_TTABLE4 0 /* four T-tables, 32 replicas each, in LDS (128 KiB) */
#define AES_PLACEMENT_TTABLE2 1 /* T0 and T2 (= T0 rotated 16), 32 replicas (64 KiB) */
#define AES_PLACEMENT_TTABLE1 2 /* T0 only, 32 replicas (32 KiB); rotations on the VALU */
#define AES_PLACEMENT_BITSLICED 3 /* no tables: 32 blocks per lane as 128 bit slices, the S-box as a
                                     Boolean circuit; ECB only, bpt is ignored (512 bytes per thread),
                                     wg at most 256 */
/* One column word per lane (4 bytes per thread): the four lanes of a quad
 * hold the four columns of one block and exchange them each round, so a
 * lane issues four lookups per round instead of sixteen.  For launches bound
 * by the latency of one block's rounds (small buffers). */
#define AES_BPT_COLUMN 0
/* CBC message-set decryption with one wave per message:
 * bpt = AES_BPT_WAVE_MSG + 1 or 2 (blocks per lane per 64-lane unit). */
#define AES_BPT_WAVE_MSG 16
typedef struct {
    int32_t bpt;       /* blocks per thread per iteration: 1, 2, 4 (16/32/64 bytes), or
                          AES_BPT_COLUMN: a quarter block, four lanes per block (ECB, table
                          placements only) */
    int32_t wg;        /* workgroup size: multiple of 64 in [64, 1024] */
    int32_t placement; /* AES_PLACEMENT_* */
    int32_t grid;      /* workgroups; 0 = persistent (compute units x workgroups that fit on one) */
} aes_variant;

/* Same as aes_ecb_encrypt/decrypt (decrypt != 0 selects decryption) with an
 * explicit variant.  AES_EINVAL for a variant outside the search space. */
int aes_ecb_crypt_variant(const uint32_t *rk, int nr, int decrypt, const void *in, void *out, size_t nblocks,
                          const aes_variant *variant, void *stream);

/* Tuning table used by aes_ecb_encrypt/decrypt: one variant per (nr,
 * direction, size bucket of nblocks).  Buckets: <=256 blocks (4 KiB),
 * <=4096 (64 KiB), <=32768 (512 KiB), <=131072 (2 MiB), <=524288 (8 MiB),
 * <=2097152 (32 MiB), larger.
 * aes_tune_set is process-wide and thread-safe; grid is ignored. */
#define AES_SIZE_BUCKETS 7
int aes_tune_set(int nr, int decrypt, size_t nblocks, const aes_variant *v);
int aes_tune_get(int nr, int decrypt, size_t nblocks, aes_variant *v);
int aes_size_bucket(size_t nblocks);

/*
 * aes_ctr_crypt -- counter mode (section 3.1.5, eq 5; parallel per Table 1):
 * output byte k of data block j is input byte k XOR byte k of
 * cipher(counter c0 + j), counters being 128-bit big-endian integers taken
 * modulo 2^128.  Encryption and decryption are the same call.
 *   rk:           host pointer to the ENCRYPTION schedule (rk_enc) of
 *                 aes_expand_key, 4*(nr+1) words, copied into the launch.
 *   nr:           10, 12 or 14.
 *   iv:           host pointer to the 16-byte initial counter block.
 *   block_offset: c0 = iv + block_offset (a 128-bit addition), so a long
 *                 message can be processed in pieces: a piece starting at
 *                 byte 16*k of the message passes block_offset = k.  The
 *                 paper's R (counter of block i = R + i, i from 1) is
 *                 c0 - 1.
 *   in, out:      device pointers, 16-byte aligned, nbytes each; in == out
 *                 is allowed, any other overlap is AES_EINVAL.
 *   nbytes:       any length; a partial last block uses the leading bytes
 *                 of its key-stream block.  0 is a no-op returning AES_OK.
 * The variant is the encryption entry of the tuning table for
 * ceil(nbytes/16) blocks.  Asynchronous on stream.
 */
int aes_ctr_crypt(const uint32_t *rk, int nr, const uint8_t *iv, uint64_t block_offset, const void *in, void *out,
                  size_t nbytes, void *stream);
/* Same with an explicit variant (AES_EINVAL outside the search space). */
int aes_ctr_crypt_variant(const uint32_t *rk, int nr, const uint8_t *iv, uint64_t block_offset, const void *in,
                          void *out, size_t nbytes, const aes_variant *variant, void *stream);

/*
 * aes_cbc_decrypt -- CBC decryption (section 3.1.2, eq 2, read as
 * C_i = cipher(P_i XOR C_{i-1}) with C_0 = iv): P_i = invcipher(C_i) XOR
 * C_{i-1}.  Every block is independent, so this is the parallel direction
 * of CBC; encryption is sequential within a message (aes_cbc_encrypt_msgs
 * runs many messages side by side).
 *   rk:      host pointer to the DECRYPTION schedule (rk_dec), copied.
 *   nr:      10, 12 or 14.
 *   iv:      host pointer to the 16-byte initialisation vector (C_0).  To
 *            continue a message, pass its last ciphertext block so far.
 *   in, out: device pointers, 16-byte aligned, nblocks*16 bytes; they must
 *            not overlap at all (in == out is AES_EINVAL: block b reads
 *            ciphertext block b - 1).
 *   nblocks: whole blocks; 0 is a no-op returning AES_OK.
 * The variant is the decryption entry of the tuning table.
 */
int aes_cbc_decrypt(const uint32_t *rk, int nr, const uint8_t *iv, const void *in, void *out, size_t nblocks,
                    void *stream);
int aes_cbc_decrypt_variant(const uint32_t *rk, int nr, const uint8_t *iv, const void *in, void *out, size_t nblocks,
                            const aes_variant *variant, void *stream);

/*
 * aes_cbc_encrypt_msgs -- CBC encryption (section 3.1.2, eq 2, read as
 * C_i = cipher(P_i XOR C_{i-1}) with C_0 = iv) of many independent messages
 * under one key, in one launch.  Within a message each block needs the
 * previous ciphertext block, so a message cannot be split (Table 1 marks
 * CBC encryption unsuitable for parallel work); the parallelism is across
 * messages: each message is one chain, walked by one GPU lane.
 *   rk:        host pointer to the ENCRYPTION schedule (rk_enc), copied.
 *   nr:        10, 12 or 14.
 *   msgs_dev:  device array of nmsgs aes_cbc_msg, 16-byte aligned.  Message
 *              m encrypts blocks [in_block, in_block + nblocks) of the input
 *              arena into blocks [out_block, out_block + nblocks) of the
 *              output arena, starting its chain from iv (C_0; to continue a
 *              message, pass its last ciphertext block so far).
 *   in_base, in_blocks / out_base, out_blocks: device arenas, 16-byte
 *              aligned, sizes in blocks.  The same arena for both is
 *              allowed; any other overlap of the two is AES_EINVAL.  A
 *              message may run in place (equal ranges in one arena); the
 *              output range of a message must not overlap another message's
 *              input or output range (not checked: such messages get
 *              undefined results, and no access leaves the arenas).
 *   rejected_dev: NULL or a device uint32 (4-byte aligned) to which the
 *              kernel adds the number of messages it skipped: a range
 *              outside its arena or a nonzero reserved field.  A skipped
 *              message's output is left untouched.
 *   nmsgs:     0 is a no-op returning AES_OK.
 * One chain has one block in flight, so a launch keeps every compute unit
 * busy only with about 2^17 messages or more; fewer are bound by the latency
 * of a block's rounds.  The consecutive entries that one wave walks (64, or
 * 16 for short lists) take as long as the longest of them: list messages of
 * similar length together.
 * Asynchronous on stream.
 */
typedef struct {
    uint64_t in_block;
    uint64_t out_block;
    uint64_t nblocks;
    uint64_t reserved; /* 0 */
    uint8_t iv[16];
} aes_cbc_msg;
int aes_cbc_encrypt_msgs(const uint32_t *rk, int nr, const aes_cbc_msg *msgs_dev, size_t nmsgs, const void *in_base,
                         size_t in_blocks, void *out_base, size_t out_blocks, uint32_t *rejected_dev, void *stream);
/* Same with an explicit variant: bpt = blocks a lane loads and stores at once
 * (1, 2, 4 or 8; one lane walks one message), or AES_BPT_COLUMN (four lanes
 * share a message, one column word each, 16 messages per wave: shorter
 * rounds for short lists); wg, a table placement (not bitsliced), grid (0 =
 * as many workgroups as fit on every compute unit, no more than the messages
 * need).  AES_EINVAL outside that.  aes_cbc_encrypt_msgs takes the 4-table
 * placement, bpt 8 when there are at least 8 one-lane waves per compute unit
 * (2^17 messages on 256 CUs) and AES_BPT_COLUMN below that, and the smallest
 * workgroup (up to 1024 threads) that gives every compute unit the same
 * number of waves. */
int aes_cbc_encrypt_msgs_variant(const uint32_t *rk, int nr, const aes_cbc_msg *msgs_dev, size_t nmsgs,
                                 const void *in_base, size_t in_blocks, void *out_base, size_t out_blocks,
                                 uint32_t *rejected_dev, const aes_variant *variant, void *stream);

/*
 * aes_cbc_decrypt_msgs -- CBC decryption (section 3.1.2, eq 2 read as above:
 * P_i = invcipher(C_i) XOR C_{i-1}, C_0 = iv) of the same kind of message
 * set, under one key, in one launch: one message per lane, its blocks
 * independent of each other, each XORed with the preceding ciphertext block.
 *   rk:       host pointer to the DECRYPTION schedule (rk_dec), copied.
 *   Other arguments, checks, skipped messages and errors as for
 *   aes_cbc_encrypt_msgs; a message may run in place (equal ranges in one
 *   arena).  For one long message aes_cbc_decrypt is the faster call (every
 *   block of it in parallel); this call is for many messages at once.
 * Two kernels: one message per lane (bpt = blocks a lane decrypts at once:
 * 1, 2 or 4), for short messages, or one wave per message (bpt =
 * AES_BPT_WAVE_MSG + 1 or 2 blocks per lane per 64-block unit, every
 * access of the wave contiguous), for messages of 64 blocks or more.  The
 * _variant form takes that bpt, wg, a table placement (not bitsliced) and
 * grid.  The default uses 4 tables, one wave per message with 2 blocks per
 * lane when the input arena averages at least 64 blocks per message (one
 * lane per message with 4 otherwise), and the smallest workgroup (up to 1024
 * threads) that gives every compute unit the same number of waves.
 * Asynchronous on stream.
 */
int aes_cbc_decrypt_msgs(const uint32_t *rk, int nr, const aes_cbc_msg *msgs_dev, size_t nmsgs, const void *in_base,
                         size_t in_blocks, void *out_base, size_t out_blocks, uint32_t *rejected_dev, void *stream);
int aes_cbc_decrypt_msgs_variant(const uint32_t *rk, int nr, const aes_cbc_msg *msgs_dev, size_t nmsgs,
                                 const void *in_base, size_t in_blocks, void *out_base, size_t out_blocks,
                                 uint32_t *rejected_dev, const aes_variant *variant, void *stream);

/*
 * aes_roof_probe -- the measured roofs beside the published ones.
 *   which = AES_PROBE_LDS:  conflict-free ds_read_b32 lookups with per-lane
 *           random entries in a 32-replica table laid out like the T-tables,
 *           32 waves per CU (the cipher's binding unit);
 *   which = AES_PROBE_VALU: independent full-rate v_bitop3_b32 chains, 32
 *           waves per CU.
 *   iters:  loop count in [1, 2^24]; each thread does 16 operations per loop.
 *   out_dev, out_bytes: device scratch of one 32-bit word per probe thread
 *           (compute units x 2048 threads), written with a checksum.
 *   work:   if not NULL, receives the number of lookups / lane-operations
 *           the launch performs; the caller times the launch on stream.
 * The copy roof is aes_device_copy.  Diagnostic only; asynchronous.
 */
#define AES_PROBE_LDS 0
#define AES_PROBE_VALU 1
int aes_roof_probe(int which, uint32_t iters, void *out_dev, size_t out_bytes, uint64_t *work, void *stream);

/*
 * Host-inclusive path (aes_pipe_*): host buffer in, host buffer out.  The
 * paper's GPU timings are of files in host memory (section 5, Tables 4-5),
 * i.e. they include the copies over the host link; this path measures and
 * serves that regime.  A buffer is cut into pieces of at most chunk_bytes
 * (smaller, down to 1 MiB, when that gives every slot two pieces); piece i
 * runs on slot i mod nslots (one stream): copy to the device, the kernel in
 * place, copy back, so copies and kernels of different pieces overlap.  Two
 * slots keep one copy in each direction in flight, which is what the host
 * link rewards (on MI355X 2 x 32 MiB reached 0.90 of the link's two-way
 * rate, 4 or 8 slots less).
 *
 * aes_pipe_config (all memory provided and owned by the caller):
 *   dev, dev_bytes:         device workspace, 16-byte aligned, at least
 *                           nslots * chunk_bytes bytes.
 *   pinned, pinned_bytes:   pinned host staging (hipHostMalloc / page-locked)
 *                           of at least nslots * chunk_bytes bytes; used for
 *                           pageable host buffers.  May be NULL when every
 *                           run passes AES_PIPE_HOST_PINNED.
 *   chunk_bytes:            positive multiple of 16.
 *   nslots:                 1..AES_PIPE_MAX_SLOTS streams (chunks in flight).
 * aes_pipe_create records the current device and creates the streams, the
 * events and one 256-byte page of pinned host memory (hipHostMalloc) that
 * holds the single-launch path's completion word; aes_pipe_destroy waits for
 * the streams and frees all three (not the caller's memory).
 *
 * aes_pipe_run(p, op, rk, nr, iv, host_in, host_out, nbytes, flags):
 *   op:      AES_PIPE_ECB_ENCRYPT / AES_PIPE_ECB_DECRYPT (rk = rk_enc /
 *            rk_dec, nbytes a multiple of 16) or AES_PIPE_CTR (rk = rk_enc,
 *            iv = first counter block, any nbytes; each piece continues the
 *            counter at iv + (its offset)/16).
 *   host_in, host_out: host pointers; host_in == host_out is allowed, any
 *            other overlap is AES_EINVAL.
 *   flags:   AES_PIPE_HOST_PINNED if both host buffers are page-locked (then
 *            they are copied directly, no staging).
 * A buffer of at most one chunk and 4 MiB runs as a single kernel launch on
 * host memory when the device maps it (the caller's pinned buffers, or the
 * pipe's pinned staging): each range must lie inside one page-locked
 * allocation mapped at the same address; otherwise it takes the copy path.
 * That launch is followed by a one-thread kernel that writes a completion
 * word into the pipe's pinned page, which the call polls (falling back to
 * the runtime's wait after 2 ms, or when the page could not be allocated);
 * a pageable buffer of 512 KiB or more goes through the staging in up to
 * four pieces, so the CPU copies of one overlap the kernel of another.
 * Synchronous: returns when host_out holds the result.  Calls on one pipe
 * are serialised.  Errors: AES_EINVAL for bad arguments, AES_EHIP for a
 * failed copy or launch (all slots are drained before returning).
 */
#define AES_PIPE_MAX_SLOTS 8
#define AES_PIPE_ECB_ENCRYPT 0
#define AES_PIPE_ECB_DECRYPT 1
#define AES_PIPE_CTR 2
#define AES_PIPE_HOST_PINNED 1
typedef struct aes_pipe aes_pipe;
typedef struct {
    void *dev;
    uint64_t dev_bytes;
    void *pinned;
    uint64_t pinned_bytes;
    uint64_t chunk_bytes;
    int32_t nslots;
    int32_t reserved; /* 0 */
} aes_pipe_config;
int aes_pipe_create(const aes_pipe_config *cfg, aes_pipe **out);
int aes_pipe_destroy(aes_pipe *p);
int aes_pipe_run(aes_pipe *p, int op, const uint32_t *rk, int nr, const uint8_t *iv, const void *host_in,
                 void *host_out, size_t nbytes, int flags);

/*
 * Batched ECB: many independent messages, each with its own key, key size
 * and direction, in one persistent launch (not in the paper; the same
 * per-block cipher as aes_ecb_encrypt/decrypt).
 *
 * Key table: device array of key slots, AES_KEY_SLOT_WORDS uint32 each:
 *   words [0, 60)   encryption schedule, [64, 124) decryption schedule,
 *   word 124        Nr.  aes_key_slot() fills one slot image on the host.
 */
#define AES_KEY_SLOT_WORDS 128
#define AES_KEY_SLOT_ENC 0
#define AES_KEY_SLOT_DEC 64
#define AES_KEY_SLOT_NR 124
int aes_key_slot(const uint8_t *key, int keybits, uint32_t *slot);

/* One message: blocks [in_block, in_block+nblocks) of the input arena go to
 * blocks [out_block, ...) of the output arena (units of 16 bytes). */
typedef struct {
    uint64_t in_block;
    uint64_t out_block;
    uint64_t nblocks;
    uint32_t key_slot;
    uint32_t decrypt; /* 0 = encrypt, nonzero = decrypt */
} aes_msg;

/* One work item: a chunk of at most chunk_blocks blocks of one message. */
typedef struct {
    uint64_t in_block;
    uint64_t out_block;
    uint32_t nblocks;
    uint32_t key_slot;
} aes_work_item;

/* Largest work item, in blocks (256 MiB).  One wave walks an item alone, so
 * items are meant to be small: the batched launch and the serving engine are
 * tuned at 2048-4096 blocks. */
#define AES_MAX_ITEM_BLOCKS (1u << 24)

/*
 * aes_batch_plan -- host only.  Splits msgs[0..nmsgs) into work items of at
 * most chunk_blocks blocks, all encryption items first, then all decryption
 * items, in message order.  items: host array of cap entries.  *n_enc and
 * *n_dec receive the item counts even when the capacity is too small
 * (AES_ERANGE), so a caller can size the array.  Messages with nblocks == 0
 * produce no items.  Errors: chunk_blocks outside [1, AES_MAX_ITEM_BLOCKS] or a
 * message whose in_block + nblocks or out_block + nblocks passes 2^64:
 * AES_EINVAL with both counts 0; more than 2^32 - 1 items in all: AES_ERANGE
 * with both counts 0.  Nothing is written to items unless the call succeeds.
 */
int aes_batch_plan(const aes_msg *msgs, size_t nmsgs, uint32_t chunk_blocks, aes_work_item *items, size_t cap,
                   size_t *n_enc, size_t *n_dec);

typedef struct {
    int32_t bpt;        /* 1, 2, 4 */
    int32_t wg;         /* multiple of 64 in [64, 1024] */
    int32_t grid;       /* 0 = as many workgroups as fit on every compute unit at once */
    int32_t enc_groups; /* workgroups starting on the encryption list; <0 = by item share */
    int32_t placement;  /* AES_PLACEMENT_TTABLE4 (0, the default), _TTABLE2 or _TTABLE1 */
} aes_batch_config;

/*
 * aes_ecb_batch -- one persistent launch over a planned work list.
 *   items_dev:     device copy of the planned items (n_enc + n_dec entries).
 *   key_table_dev: device key table of n_slots slots.
 *   in_base/out_base: device arenas of in_blocks / out_blocks blocks, 16-byte
 *                  aligned; the same arena for both is allowed (in place),
 *                  any other overlap of [in_base, +16*in_blocks) and
 *                  [out_base, +16*out_blocks) is refused (AES_EINVAL).
 *   counters_dev:  device array of 4 uint32, all zero before the first launch:
 *                  [0],[1] claim counters, [2] finished workgroups (the last
 *                  workgroup resets [0..2] to zero, so the launch can be
 *                  replayed, e.g. from a captured HIP graph), [3] the number of
 *                  items rejected by the in-kernel checks (slot out of range,
 *                  blocks outside an arena, more than AES_MAX_ITEM_BLOCKS
 *                  blocks); [3] is never reset by the kernel.
 *   cfg:           may be NULL for defaults.
 * Launches that share counters_dev must not overlap in time.
 */
int aes_ecb_batch(const aes_work_item *items_dev, size_t n_enc, size_t n_dec, const uint32_t *key_table_dev,
                  size_t n_slots, const void *in_base, size_t in_blocks, void *out_base, size_t out_blocks,
                  uint32_t *counters_dev, const aes_batch_config *cfg, void *stream);

/*
 * aes_ecb_batch_noalloc -- aes_ecb_batch for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): the same launch, with the four claim counters in a
 * scratch array of AES_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device (a static device array, kept until the process ends) instead of a
 * caller's counters_dev.  The caller still passes the work list, key table
 * and arenas, with the meaning, checks and errors of aes_ecb_batch.  The call
 * allocates nothing: it enqueues a one-workgroup kernel that zeroes the
 * counters, then the batch kernel, both on `stream` (so a captured graph
 * holds two kernel nodes and no memset).  A launch needs 16 bytes of the
 * scratch whatever its sizes, so no size exceeds it.  Rejected items are
 * skipped as in aes_ecb_batch but their count is not reported.  Every call on
 * one device shares that device's scratch: calls whose launches overlap in
 * time on one device (different streams, or graphs replayed concurrently)
 * race on the counters and must not be issued.  The first call on each
 * device looks up the scratch's device address (hipGetSymbolAddress) and the
 * chosen variant's occupancy: a caller that captures the launch in a HIP
 * graph makes one call on that device, with that configuration, before it
 * begins the capture.  AES_EHIP if the scratch's device address cannot be
 * obtained or a launch fails.
 */
#define AES_NOALLOC_SCRATCH_BYTES 256
int aes_ecb_batch_noalloc(const aes_work_item *items_dev, size_t n_enc, size_t n_dec, const uint32_t *key_table_dev,
                          size_t n_slots, const void *in_base, size_t in_blocks, void *out_base, size_t out_blocks,
                          const aes_batch_config *cfg, void *stream);

/* Workgroups a launch of aes_ecb_batch with cfg (NULL: defaults) uses at most:
 * cfg->grid if positive, else as many as fit on every compute unit at once
 * (the occupancy of that bpt / placement / workgroup size).  A caller that
 * splits the workgroups by bytes (enc_groups) sizes the split with it.
 * AES_EINVAL for a config aes_ecb_batch refuses; AES_EHIP if the device
 * cannot be queried. */
int aes_batch_max_grid(const aes_batch_config *cfg, int *grid);

/*
 * Serving: a native continuous-batching engine over aes_ecb_batch (not in the
 * paper).  Requests read blocks of one device input pool and get their
 * output placed in a device output arena by the engine.  A worker thread
 * admits requests in arrival order while the device budget (input + output
 * bytes of admitted, unfinished requests) and the arena allow, and whenever
 * one of nslots stream slots is free it runs everything admitted so far as
 * one batched launch; requests arriving meanwhile join the next batch, and
 * batches on different slots overlap on the device.
 *
 * Memory: the caller provides every buffer: key table, input pool, output
 * arena, a device workspace of aes_server_workspace_bytes(cfg) bytes (work
 * lists and counters) and pinned host staging of aes_server_staging_bytes(cfg)
 * bytes (e.g. hipHostMalloc).  The engine creates nslots streams and events
 * on the current device.  All of them must outlive the server.
 */
typedef struct {
    uint64_t in_block;  /* first block of the request in the input pool */
    uint64_t nblocks;   /* > 0 */
    uint32_t key_slot;  /* index into the key table */
    uint32_t decrypt;   /* 0 = encrypt, nonzero = decrypt */
} aes_request;

#define AES_SERVED_DONE 0
#define AES_SERVED_REJECTED 1 /* can never run: empty, over budget/arena, more work items than
                                 max_batch_items, bad slot, outside the pool */
#define AES_SERVED_FAILED 2   /* its batch failed to launch or run */
typedef struct {
    uint64_t id;          /* submission order, from 0 */
    double arrival_s;     /* seconds on the server's clock (replay: scheduled arrival) */
    double admitted_s;
    double done_s;        /* when the engine saw the batch complete */
    uint64_t out_block;   /* output position in the arena (valid when DONE) */
    uint64_t nblocks;
    int32_t status;       /* AES_SERVED_* */
    int32_t batch;        /* index of the batch that ran the request */
} aes_served;

/* AUTO: when the device maps the pinned staging, the batch kernel's last
 * workgroup writes a completion word into it (after every workgroup's output
 * stores) and the worker reads it with a plain load; otherwise, and with EVENTS, the
 * worker queries an event recorded after the kernel.  Either way a batch not
 * seen complete within 2 ms is also checked with the runtime, which reports
 * a failed kernel (AES_SERVED_FAILED). */
#define AES_SERVE_COMPLETION_AUTO 0
#define AES_SERVE_COMPLETION_EVENTS 1
typedef struct {
    uint64_t budget_bytes;     /* cap on input + output bytes of admitted, unfinished requests */
    uint32_t chunk_blocks;     /* work-item size, 1..AES_MAX_ITEM_BLOCKS */
    uint32_t max_batch_items;  /* work items per batch (sizes the workspace) */
    int32_t nslots;            /* batches in flight, 1..16 (one stream each) */
    int32_t bpt, wg, grid;     /* batch kernel shape (grid 0 = as many workgroups as fit on every CU) */
    int32_t auto_release;      /* nonzero: output space is freed when a request completes */
    int32_t dry_run;           /* nonzero: no device work; batches complete after dry_run_seconds */
    double dry_run_seconds;
    int32_t placement;         /* table placement of the batch kernel, as in aes_batch_config */
    int32_t completion;        /* AES_SERVE_COMPLETION_*: how the worker sees a batch finish */
    uint32_t small_item_blocks; /* work-item size for requests of at most chunk_blocks blocks, so that
                                   several waves share a small request (0: chunk_blocks for all);
                                   at most chunk_blocks */
    int32_t size_classes;      /* nonzero: a batch holds only requests of at most chunk_blocks blocks or
                                  only larger ones (the head of the queue picks; the other class keeps
                                  its order for the next slot), so small requests do not wait for
                                  large ones in their batch; 0: one FIFO for all */
} aes_serve_config;

typedef struct {
    uint64_t batches;
    uint64_t max_device_bytes_in_use;
    uint64_t arena_blocks_in_use;
    uint64_t pending;
    uint64_t direct_batches; /* batches whose kernel read the work list from the pinned staging
                                (device-mapped staging, at most 4096 items: no copy) */
    uint64_t launch_ns;      /* worker time spent in the runtime calls that launch batches
                                (work-list copy, kernel, completion word or event), all batches */
} aes_serve_stats;

typedef struct aes_server aes_server;

size_t aes_server_workspace_bytes(const aes_serve_config *cfg);
size_t aes_server_staging_bytes(const aes_serve_config *cfg);
/* AES_EINVAL bad config or null buffer; AES_ERANGE workspace/staging too small;
 * AES_EHIP stream/event creation failed. */
int aes_server_create(const aes_serve_config *cfg, const uint32_t *key_table_dev, size_t n_slots, const void *in_pool,
                      size_t in_blocks, void *out_arena, size_t out_blocks, void *workspace_dev,
                      size_t workspace_bytes, void *staging_host, size_t staging_bytes, aes_server **out);
/* Thread-safe; requests get consecutive ids starting at *first_id. */
int aes_server_submit(aes_server *s, const aes_request *reqs, size_t n, uint64_t *first_id);
/* Moves up to cap finished requests (any order of ids) into out; *n = count. */
int aes_server_poll(aes_server *s, aes_served *out, size_t cap, size_t *n);
/* Frees the output space of finished requests (no-op with auto_release).
 * Records with status AES_SERVED_DONE whose (out_block, nblocks) the engine
 * does not hold as an unreleased output (released already, or never handed
 * out) are skipped, and the call returns AES_EINVAL; the others are freed. */
int aes_server_release(aes_server *s, const aes_served *done, size_t n);
int aes_server_stats(aes_server *s, aes_serve_stats *stats);
/* Finishes every submitted request, then frees the engine (not the buffers).
 * Without auto_release, queued requests that cannot get output space while
 * nothing runs (the caller still holds outputs and, being inside this call,
 * releases no more) are finished as AES_SERVED_REJECTED instead of waiting. */
int aes_server_destroy(aes_server *s);
/* Open-loop replay on an auto_release server: request i is submitted at
 * arrival_s[i] seconds after the call starts; returns when all have finished,
 * with results[i] for request i (arrival_s = scheduled arrival). */
int aes_serve_replay(aes_server *s, const aes_request *reqs, const double *arrival_s, size_t n, aes_served *results);

/* Host copies of the library's source tables (for inspection and tests):
 * sbox/inv_sbox 256 bytes each; te0/td0 256 column words each (eqs 22 and
 * its decryption counterpart; T_k = rotl(T_0, 8k)).  Any pointer may be NULL. */
int aes_host_tables(uint8_t *sbox, uint8_t *inv_sbox, uint32_t *te0, uint32_t *td0);

/* Plain device copy of nbytes (multiple of 16, 16-byte aligned); the memory
 * reference kernel used to calibrate HBM traffic counters. */
int aes_device_copy(const void *in, void *out, size_t nbytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* AESGPU_H */
