/*
 * bbfc.h -- C ABI of the MI355X (gfx950) library for Blocked Bloom filters
 * with choices (Schmitz, Zentgraf, Rahmann, arXiv 2501.18977).
 *
 * The filter (Section 3.1): M blocks of 512 bits, c candidate blocks per
 * key chosen by block hashes h_1..h_c, k bit hashes f_1..f_k into a block.
 * insert(x) sets F(x) = { f_i(x) } in the candidate block of lowest cost
 * (Section 3.2, App. A), or does nothing if a candidate already holds F(x);
 * query(x) answers true iff F(x) lies inside some candidate block. A query
 * of an inserted key always answers true; a key never inserted may answer
 * true with the filter's false-positive rate (Section 1).
 *
 * Conventions shared by every entry point
 *   - Status: every call returns BBFC_OK (0) or a negative bbfc_status.
 *     Argument errors are detected before anything is enqueued and return
 *     BBFC_EINVAL with nothing done; bbfc_last_error() then describes the
 *     problem (thread-local text, valid until the next call on the thread).
 *   - Device work is enqueued on the caller's HIP stream and is asynchronous;
 *     only bbfc_download, bbfc_upload and bbfc_destroy synchronise.
 *     A null stream means the legacy default stream.
 *   - Ownership: the library owns the filter memory (hipMalloc in create,
 *     hipFree in destroy). The caller owns key and output buffers, which are
 *     device pointers on the filter's device and must stay valid until the
 *     stream has executed the work that reads or writes them.
 *   - A call takes at most 2^56 keys (BBFC_EINVAL beyond).
 *   - Keys are 64-bit unsigned integers, hashed as u = 64-bit words
 *     (Section 3.4) whatever their meaningful width (a canonical 31-mer
 *     uses 62 bits).
 *   - Bit layout: bit f in [0, 512) of block b is bit (f mod 64) of 64-bit
 *     word 8*b + f/64 of the filter; words are little-endian.
 *   - A handle may be used from one host thread at a time. Concurrent
 *     insert and query launches on different streams are allowed: bits are
 *     only ever set, so a query sees some subset of the in-flight inserts.
 */
#ifndef BBFC_H
#define BBFC_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bbfc_filter *bbfc_handle;

typedef enum {
    BBFC_OK = 0,
    BBFC_EINVAL = -1,      /* bad argument; nothing was enqueued             */
    BBFC_ENOMEM = -2,      /* device allocation failed                       */
    BBFC_EHIP = -3,        /* a HIP runtime call or kernel launch failed     */
    BBFC_EUNSUPPORTED = -4, /* valid request the library does not implement  */
    BBFC_EBUSY = -5         /* not now: admission full or not finished yet    */
} bbfc_status;

/* Cost functions for block selection (App. A; Section 3.2):
 *   MIX  sigma*k*(j/256)^k + a        (eq. cost:mix)
 *   LA   k*((j + mu*k)/256)^k + a     (eq. cost:la; lookahead)
 *   EXP  beta^(j/128) + a/k           (eq. cost:exp)
 * where j is the number of bits set in the block after the insertion and a
 * the number of those that are new (Section 3.2). Costs are IEEE-754 double,
 * evaluated left to right as written; equal doubles tie, and on a tie the
 * lower choice index wins. NONE is required for, and only allowed with,
 * one choice (a Blocked Bloom filter, Section 2.2). */
typedef enum {
    BBFC_COST_NONE = 0,
    BBFC_COST_MIX = 1,
    BBFC_COST_LA = 2,
    BBFC_COST_EXP = 3
} bbfc_cost_kind;

/* kind plus its parameter (sigma, mu or beta). A NaN param selects the
 * paper's value: sigma 2.5 for k <= 10 and 50 for k >= 11 (the printed
 * values are 2.5 at k = 7 and 50 at k = 14, App. C), mu 3.5 (App. C),
 * beta (1 + sqrt 5)/2 (Section 4). Ignored for BBFC_COST_NONE. */
typedef struct {
    int32_t kind; /* a bbfc_cost_kind */
    double param;
} bbfc_cost;

/* Limits of the library. */
#define BBFC_MAX_CHOICES 4u
#define BBFC_MAX_BITS_PER_KEY 32u

/* How a key's k bit addresses F(x) are chosen (Section 3.3):
 *   RANDOM    f_i(x), i = 1..k, are independent hashes into [512] (the top
 *             9 bits of a_i * x); two of them may coincide, so a key can
 *             set and test fewer than k distinct bits.
 *   DISTINCT  App. B: f_i is hashed into [512 - i + 1] and names the f_i-th
 *             address not taken by f_1..f_{i-1}, so every key sets exactly
 *             k distinct bits, a uniform k-subset of [512]. The bit hash
 *             multipliers must be coprime to their moduli 512 - i + 1. It
 *             costs k(k-1)/2 compare steps per key in the hashing phase. */
typedef enum {
    BBFC_BITS_RANDOM = 0,
    BBFC_BITS_DISTINCT = 1
} bbfc_bit_selection;

/* Everything that defines a filter, for bbfc_create_config.
 *
 * Sub-arrays (Section 3.4, Parallelization): with subarrays = T > 1 the
 * n_blocks blocks form T sub-arrays of S = n_blocks / T blocks (T must
 * divide n_blocks). A key's sub-array is h_0(x), the linear hash into [T]
 * with multiplier sub_mult; its candidates are blocks h_0(x) S + h_i(x) with
 * the block hashes h_i into [S]. subarrays 0 or 1 is a single array. The
 * layout changes which blocks a key uses, not the method; it is what lets
 * bbfc_bulk_insert stage a whole sub-array in on-chip memory. */
typedef struct {
    uint64_t n_blocks;
    uint32_t choices;
    uint32_t bits_per_key;
    bbfc_cost cost;
    int32_t bit_selection;      /* a bbfc_bit_selection */
    uint64_t seed;              /* multiplier stream (see bbfc_create_seeded) */
    const uint64_t *block_mult; /* host [choices], or null: drawn from seed */
    const uint64_t *bit_mult;   /* host [bits_per_key], or null: drawn from seed */
    uint64_t subarrays;         /* T; 0 or 1: one array */
    uint64_t sub_mult;          /* multiplier of h_0 (coprime to T), or 0: drawn from seed */
} bbfc_config;

/* Create an empty filter of n_blocks 512-bit blocks (64 bytes each, the
 * allocation is 256-byte aligned) on the current HIP device, with `choices`
 * candidate blocks per key (c, Section 3.1) and `bits_per_key` bit hashes
 * (k, Section 3.1: the number of hashes, not the space per key; the space
 * is fixed by n_blocks). Hash multipliers are drawn from seed 0 (see
 * bbfc_create_seeded).
 *   n_blocks >= 1; 1 <= choices <= 4; 1 <= bits_per_key <= 32;
 *   cost.kind == NONE iff choices == 1.
 * On success *out receives the handle; on failure *out is left untouched.
 * Errors: EINVAL (ranges, null out), ENOMEM (filter does not fit), EHIP. */
bbfc_status bbfc_create(uint64_t n_blocks, uint32_t choices, uint32_t bits_per_key, bbfc_cost cost,
                        bbfc_handle *out);

/* As bbfc_create, with the linear hashes' multipliers (Section 3.4: "a
 * random large integer a, coprime with b") drawn from a SplitMix64 stream
 * (Steele, Lea, Flood 2014) started at `seed`: each draw is made odd, draws
 * below 2^32 or sharing a factor with the modulus are skipped; the first
 * `choices` accepted draws (modulus n_blocks) are the block multipliers,
 * the next `bits_per_key` (modulus 512) the bit multipliers. */
bbfc_status bbfc_create_seeded(uint64_t n_blocks, uint32_t choices, uint32_t bits_per_key, bbfc_cost cost,
                               uint64_t seed, bbfc_handle *out);

/* As bbfc_create, with explicit multipliers: block_mult[choices] (each must
 * be coprime to n_blocks) and bit_mult[bits_per_key] (each must be odd).
 * Both arrays are host memory, copied; the caller keeps ownership. */
bbfc_status bbfc_create_with_multipliers(uint64_t n_blocks, uint32_t choices, uint32_t bits_per_key,
                                         bbfc_cost cost, const uint64_t *block_mult,
                                         const uint64_t *bit_mult, bbfc_handle *out);

/* The general constructor: shape and cost as bbfc_create, the bit
 * selection strategy, the sub-array layout, and multipliers given or drawn.
 * Multipliers are drawn as in bbfc_create_seeded, except that block
 * multipliers are coprime to S = n_blocks / subarrays, that with DISTINCT
 * the i-th bit multiplier (i from 1) is drawn coprime to 512 - i + 1, and
 * that with subarrays > 1 one more draw, coprime to T, is the multiplier of
 * h_0. Given multipliers are checked (block ones coprime to S, bit ones to
 * their moduli, sub_mult to T) and copied. Errors: as bbfc_create, plus
 * EINVAL for a null cfg, an unknown bit_selection or a subarrays that does
 * not divide n_blocks. */
bbfc_status bbfc_create_config(const bbfc_config *cfg, bbfc_handle *out);

/* Synchronise the device, then free the filter. A null handle is EINVAL. */
bbfc_status bbfc_destroy(bbfc_handle h);

/* Insert d_keys[0..n) (device memory) with racing atomic inserts
 * (Sections 3.1, 3.2). Every key's mask ends up in one of its candidates,
 * so every inserted key queries true afterwards. Keys inserted by the same
 * call decide on block contents that may miss the bits of keys still in
 * flight, so the filter may differ from a one-key-at-a-time build; the
 * library bounds the keys in flight to a fraction of n_blocks (see
 * BBFC_OPT_INSERT_INFLIGHT) so that the false-positive rate stays within
 * about 1% of the sequential build's. With choices == 1 the result equals
 * the sequential build bit for bit, and the keys in flight are not bounded. n == 0 is a no-op. Errors: EINVAL (null handle, null
 * keys with n > 0), EHIP. */
bbfc_status bbfc_insert(bbfc_handle h, const uint64_t *d_keys, uint64_t n, hipStream_t stream);

/* Checking hook: bbfc_insert (same kernels' schedule, shape and keys in
 * flight) that also records each key's decision in d_decisions[0..n)
 * (device memory, caller-owned, one byte per key, must not overlap the
 * keys): the index i in [0, choices) of the candidate h_(i+1)(x) whose block
 * received F(x), or BBFC_DECISION_PRESENT (0xFF) when the key found F(x)
 * already held by a candidate and wrote nothing (Sections 3.1, 3.2). With
 * these, the filter after the call is the OR, over the keys that wrote, of
 * F(x) placed in the recorded candidate, on top of what the filter held
 * before. bbfc_insert itself records nothing. Errors as bbfc_insert, and
 * EINVAL for null or overlapping decisions with n > 0. */
#define BBFC_DECISION_PRESENT 0xFFu
bbfc_status bbfc_insert_recorded(bbfc_handle h, const uint64_t *d_keys, uint64_t n, uint8_t *d_decisions,
                                 hipStream_t stream);

/* Insert d_keys[0..n) with exactly the sequential semantics: the result is
 * the filter obtained by inserting the keys one at a time in index order
 * (Section 3.2 applied key by key), on any layout. Each step decides
 * together every pending key that no older pending key shares a candidate
 * block with: on one workgroup below 2^16 keys, else on the whole device in
 * windows of 2^16 or 2^18 keys. The first large call allocates scratch that
 * the filter keeps until bbfc_destroy: 33 MB, or 130 MB for filters of 2^24
 * blocks or more. Calls on one filter must not overlap.
 * For filters with sub-arrays, bbfc_bulk_insert gives the same result
 * faster. Errors as bbfc_insert, and ENOMEM if the scratch cannot be
 * allocated. */
bbfc_status bbfc_insert_deterministic(bbfc_handle h, const uint64_t *d_keys, uint64_t n,
                                      hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * bbfc_insert_deterministic with the same result, bit for bit, that never
 * allocates. Its scratch is a static device array of 34,144,512 bytes per
 * device (a 2^22-entry claim table and one window of 2^16 keys), held on
 * every device the library runs on until the process ends; the claim table
 * is cleared by a fill kernel on the caller's stream at the first call on a
 * device. Every n fits: the call walks the keys in windows of 2^16 (inputs
 * below 2^16 keys use no scratch), so no key count exceeds the scratch.
 * All calls on one device share the array, so calls that overlap on a
 * device race and corrupt each other's results: order them (one stream, or
 * synchronise between calls), across filters too. Errors as
 * bbfc_insert_deterministic except ENOMEM; EUNSUPPORTED on a device index
 * of 64 or more. */
bbfc_status bbfc_insert_deterministic_noalloc(bbfc_handle h, const uint64_t *d_keys, uint64_t n,
                                              hipStream_t stream);

/* Query d_keys[0..n) (Section 3.1). Writes ceil(n/64) words to d_out_bits
 * (device memory): bit t mod 64 of word t/64, least significant first, is
 * the answer for d_keys[t]; bits past n in the last word are zero. The
 * output must not overlap the keys. Errors: EINVAL (null handle, null
 * pointers with n > 0), EHIP. */
bbfc_status bbfc_query(bbfc_handle h, const uint64_t *d_keys, uint64_t n, uint64_t *d_out_bits,
                       hipStream_t stream);

/* Bulk insert for filters with sub-arrays (Section 3.4, Parallelization):
 * the same result as bbfc_insert_deterministic, i.e. as inserting
 * d_keys[0..n) one at a time in index order (Section 3.2), built the way
 * the paper parallelises insertion: the keys are routed to their
 * sub-arrays by a stable partition on h_0, and each sub-array is filled by a
 * single writer (one wavefront holding the sub-array in LDS). Needs at most
 * 1024 blocks per sub-array (n_blocks / subarrays <= 1024; a filter without
 * sub-arrays qualifies when n_blocks <= 1024). d_workspace is device memory
 * of at least bbfc_bulk_insert_workspace(h, n) bytes (about 16 bytes per
 * key, for at most 2^31 keys; larger n is inserted in consecutive pieces),
 * owned by the caller and free again when the stream reaches the end of the
 * call. Errors: EINVAL (null handle or pointers, workspace too small),
 * EUNSUPPORTED (sub-arrays too large for LDS), EHIP. */
bbfc_status bbfc_bulk_insert(bbfc_handle h, const uint64_t *d_keys, uint64_t n, void *d_workspace,
                             uint64_t workspace_bytes, hipStream_t stream);

/* Workspace bytes bbfc_bulk_insert needs for n keys (*bytes; 0 for n = 0).
 * Errors: EINVAL (null handle or output), EUNSUPPORTED as bbfc_bulk_insert. */
bbfc_status bbfc_bulk_insert_workspace(bbfc_handle h, uint64_t n, uint64_t *bytes);

/* Set every filter bit to zero (stream-ordered, uses a fill kernel). */
bbfc_status bbfc_clear(bbfc_handle h, hipStream_t stream);

/* Copy all 8*n_blocks filter words from / to host memory. Both synchronise
 * `stream` before returning. Used to checkpoint and restore a filter. */
bbfc_status bbfc_upload(bbfc_handle h, const uint64_t *h_words, hipStream_t stream);
bbfc_status bbfc_download(bbfc_handle h, uint64_t *h_words, hipStream_t stream);

/* Filter shape and hash parameters. Any output pointer may be null;
 * block_mult receives `choices` words and bit_mult `bits_per_key` words.
 * cost->param receives the resolved value (never NaN). */
bbfc_status bbfc_get_params(bbfc_handle h, uint64_t *n_blocks, uint32_t *choices, uint32_t *bits_per_key,
                            bbfc_cost *cost, uint64_t *block_mult, uint64_t *bit_mult);

/* The filter's bbfc_bit_selection. */
bbfc_status bbfc_get_bit_selection(bbfc_handle h, int32_t *bit_selection);

/* The sub-array layout: *subarrays = T (1 for a single array) and
 * *sub_mult = the multiplier of h_0 (0 when T = 1). Either pointer may be
 * null. */
bbfc_status bbfc_get_subarrays(bbfc_handle h, uint64_t *subarrays, uint64_t *sub_mult);

/* Load histogram (App. C, the per-block load figure): d_hist[j], j = 0..512
 * (device memory, 513 uint64, caller-owned) receives the number of blocks
 * with exactly j bits set. The call overwrites d_hist with a fill kernel and
 * accumulates with atomics, stream-ordered on `stream`. */
bbfc_status bbfc_load_histogram(bbfc_handle h, uint64_t *d_hist, hipStream_t stream);

/* Device address of the filter words (8*n_blocks uint64, owned by the
 * library, valid until bbfc_destroy). */
bbfc_status bbfc_get_words(bbfc_handle h, uint64_t **d_words);

/* Launch options of one filter (all have defaults; none changes a result
 * except where stated):
 *   BBFC_OPT_INSERT_INFLIGHT  upper bound on keys a racing insert keeps in
 *       flight; 0 (default) means n_blocks/(8(choices-1)), at least one
 *       wavefront of 64, and no bound with one choice. The bound matters
 *       only where it is below what the GPU holds resident (about 2.6e5
 *       keys, so filters under about 2^21 blocks with two choices): there
 *       the insert is bound by memory latency and its rate grows with the
 *       bound, at the price of decisions on staler block contents (the
 *       filter can differ, its false-positive rate drifts upwards; zero
 *       false negatives holds).
 *   BBFC_OPT_QUERY_EARLY_EXIT  1 (default): a query reads candidate i+1
 *       only for keys that candidates 1..i did not answer; 0: every
 *       candidate is read. Answers are identical either way.
 *   BBFC_OPT_INSERT_TILE  keys per wavefront tile of the racing insert.
 *       0 (default): chosen by the bound on keys in flight; bounds up to
 *       65536 keys take tiles of 8 keys (eight lanes per key, each key's
 *       hashing spread over its lanes, one short round per tile, at most
 *       four workgroups of 4 wavefronts per CU, for inserts bound by
 *       latency), larger bounds tiles of 64 keys with the insert's launch
 *       shape (which the tiles of 8 keys do not use). 1: tiles of 64 keys;
 *       2: tiles of 8 keys. The racing insert's guarantees hold either way.
 * Errors: EINVAL (null handle or pointer, unknown option, value out of
 * range). */
typedef enum {
    BBFC_OPT_INSERT_INFLIGHT = 1,
    BBFC_OPT_QUERY_EARLY_EXIT = 2,
    BBFC_OPT_INSERT_TILE = 3
} bbfc_option;
bbfc_status bbfc_set_option(bbfc_handle h, int32_t option, int64_t value);
bbfc_status bbfc_get_option(bbfc_handle h, int32_t option, int64_t *value);

/* What bbfc_insert of n keys would launch on this filter under its current
 * options and shape; nothing is enqueued. *tile_keys: keys per wavefront
 * tile (64 or 8); *keys_in_flight: the most keys the launch works on at
 * once (working wavefronts x tiles per wavefront x keys per tile), which
 * is the bound of BBFC_OPT_INSERT_INFLIGHT rounded down to whole
 * wavefronts (at least one), at most what the launch holds resident, and
 * at most n rounded up to whole tiles;
 * *workgroups: the grid. Outputs may be null. Errors: EINVAL (null
 * handle), EHIP. */
bbfc_status bbfc_insert_launch_info(bbfc_handle h, uint64_t n, uint32_t *tile_keys, uint64_t *keys_in_flight,
                                    uint64_t *workgroups);

/* Launch shape of the kernels for one operation (a filter and a batch plan
 * hold one per operation): lanes per key (8 or 4: 8 or 16 bytes per lane
 * per block read), 64-key tiles per wavefront (1 or 2: more reads in
 * flight per wavefront; an insert falls back to 1 where two tiles and the
 * rank table exceed a workgroup's LDS), a cap on resident workgroups per
 * CU (0 = as many as fit) and, for a batch plan's queries, the schedule:
 * units_per_grab == 0 strides units of tiles_per_wave tiles statically over
 * the wavefronts; 1..4096 hands them out in order, that many per atomic
 * grab, from eight queues (one per XCD) that deal the blocks of units in
 * turn (single filters always stride; batch inserts always grab one slot
 * at a time). Defaults {8, 1, 0, 0} (batch queries {8, 1, 0, 8}, batch
 * inserts {8, 1, 0, 1}). ms is
 * filled by the tuners. Shapes change speed only, never answers, and never
 * the deterministic insert; a racing insert's filter is schedule dependent
 * anyway. */
typedef struct {
    int32_t lanes_per_key;
    int32_t tiles_per_wave;
    int32_t wgs_per_cu;
    int32_t units_per_grab;
    float ms;
} bbfc_launch_shape;

#define BBFC_OP_INSERT 0
#define BBFC_OP_QUERY 1

/* Shape of one filter's kernels for `op` (BBFC_OP_INSERT or
 * BBFC_OP_QUERY); units_per_grab is ignored. Errors: EINVAL. */
bbfc_status bbfc_set_shape(bbfc_handle h, int32_t op, bbfc_launch_shape shape);
bbfc_status bbfc_get_shape(bbfc_handle h, int32_t op, bbfc_launch_shape *shape);

/* Number of blocks for n_keys keys at `space_bits_per_key` bits per key:
 * ceil(n_keys * space_bits_per_key / 512), at least 1 (App. C sizes a
 * filter by rounding the bit count up to a multiple of 512). */
uint64_t bbfc_blocks_for(uint64_t n_keys, double space_bits_per_key);

/* Dense integer rank of every cost value, as the device compares them:
 * out[a*513 + j] for 0 <= a <= k, 0 <= j <= 512 is the number of distinct
 * doubles cost(j', a') smaller than cost(j, a) over all pairs with
 * 1 <= a' <= min(j', k); pairs with a == 0, a > j are 0xFFFF. Host memory,
 * (k+1)*513 entries. Pure host computation (no device needed). */
bbfc_status bbfc_rank_table(bbfc_cost cost, uint32_t bits_per_key, uint16_t *out);

/* Text of a status code (a bbfc_status value, taken as a plain int so that
 * any value is valid); unknown codes give "unknown status". */
const char *bbfc_status_string(int32_t s);
const char *bbfc_last_error(void);

/* ------------------------------------------------------------------ */
/* DNA q-grams (k-mers) as keys (Section 4.3: genomes and sequenced reads  */
/* represented as sets of q-grams, usually 21 <= q <= 31).                */
/* ------------------------------------------------------------------ */

/* Sequences are 2-bit packed, A=0, C=1, G=2, T=3, 32 bases per 64-bit word,
 * base i in bits 63-2(i mod 32) .. 62-2(i mod 32) of word i/32 (the earlier
 * base in the higher bits). The sequence d_seq (device memory, at least
 * ceil(n_segments*seg_len/32) words) is cut into n_segments segments of
 * seg_len bases laid end to end (one genome: one segment; reads of one
 * length: one segment per read). Every window of q consecutive bases
 * inside a segment gives one key: its forward value (2q bits, first base
 * most significant) or that of its reverse complement (bases complemented,
 * b -> 3-b, and reversed), whichever is smaller (the canonical q-gram).
 * Key t is the window at base s*seg_len + j, s = t / w, j = t mod w, with
 * w = seg_len - q + 1 windows per segment (none if seg_len < q).
 * 1 <= q <= 32. */

/* Number of keys: n_segments * max(seg_len - q + 1, 0). */
uint64_t bbfc_kmer_count(uint64_t n_segments, uint64_t seg_len, uint32_t q);

/* Writes the bbfc_kmer_count keys to d_keys (device memory). Errors:
 * EINVAL (null pointers with keys to write, q out of range, sequence
 * longer than 2^62 bases), EHIP. */
bbfc_status bbfc_kmer_keys(const uint64_t *d_seq, uint64_t n_segments, uint64_t seg_len, uint32_t q,
                           uint64_t *d_keys, hipStream_t stream);

/* bbfc_insert of the sequence's keys, computed inside the insert kernel
 * from the packed bases (no key array is written). */
bbfc_status bbfc_insert_kmers(bbfc_handle h, const uint64_t *d_seq, uint64_t n_segments, uint64_t seg_len, uint32_t q,
                              hipStream_t stream);

/* bbfc_query of the sequence's keys, computed inside the query kernel;
 * the answer for key t is bit t mod 64 of d_out_bits[t/64]. EINVAL also
 * when the output overlaps the sequence. */
bbfc_status bbfc_query_kmers(bbfc_handle h, const uint64_t *d_seq, uint64_t n_segments, uint64_t seg_len, uint32_t q,
                             uint64_t *d_out_bits, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Batches: many filters of uneven sizes built or queried in one          */
/* persistent launch (insert and query as above, filter by filter).       */
/* ------------------------------------------------------------------ */

typedef struct bbfc_batch *bbfc_batch_handle;

/* A plan over n_filters filters (one device, one number of choices) in
 * which filter f receives n_keys[f] keys per call (host array, copied).
 * Layout of every call on the plan: filter f's keys are
 * d_keys[o_f .. o_f + n_keys[f]) with o_f = n_keys[0] + ... + n_keys[f-1];
 * its packed answers (bbfc_batch_query) start at word
 * ceil(n_keys[0]/64) + ... + ceil(n_keys[f-1]/64), in bbfc_query's layout.
 * Filters with no keys are allowed. The filters must outlive the plan and
 * every graph captured from it. Each call on a plan resets and uses the
 * plan's work counter, so calls on one plan must not overlap (enqueue them
 * on one stream). Errors: EINVAL (null pointers,
 * n_filters == 0, mixed devices or choices), EHIP. */
bbfc_status bbfc_batch_create(const bbfc_handle *filters, const uint64_t *n_keys, uint32_t n_filters,
                              bbfc_batch_handle *out);
bbfc_status bbfc_batch_destroy(bbfc_batch_handle b);

/* Total keys and answer words of the plan's layout (either may be null). */
bbfc_status bbfc_batch_layout(bbfc_batch_handle b, uint64_t *total_keys, uint64_t *total_out_words);

/* Racing insert of every filter's keys in one persistent launch. Each
 * filter keeps at most its own bound on keys in flight
 * (BBFC_OPT_INSERT_INFLIGHT of that filter), as bbfc_insert does. */
bbfc_status bbfc_batch_insert(bbfc_batch_handle b, const uint64_t *d_keys, hipStream_t stream);

/* Query of every filter's keys in one persistent launch; the answers of
 * filter f equal bbfc_query's on the same keys. The output must not overlap
 * the keys. */
bbfc_status bbfc_batch_query(bbfc_batch_handle b, const uint64_t *d_keys, uint64_t *d_out_bits, hipStream_t stream);

bbfc_status bbfc_batch_set_shape(bbfc_batch_handle b, int32_t op, bbfc_launch_shape shape);
bbfc_status bbfc_batch_get_shape(bbfc_batch_handle b, int32_t op, bbfc_launch_shape *shape);

/* Autotuner: times every candidate shape (lanes per key 8|4, tiles per
 * wavefront 1|2, workgroups per CU unbounded|2, and for queries a static
 * stride or ordered grabs of 16 units) of the plan's persistent
 * kernel for `op` on the caller's keys, `reps` timed runs each after one
 * warm-up, keeps the fastest in the plan and returns it in *best (may be
 * null). Insert trials run on a snapshot: the filters' words are copied
 * aside (device memory equal to their size is allocated for the duration)
 * and restored before every trial and at the end, so the filters are
 * unchanged on return. Synchronises `stream`. */
bbfc_status bbfc_batch_tune(bbfc_batch_handle b, int32_t op, const uint64_t *d_keys, uint64_t *d_out_bits,
                            uint32_t reps, hipStream_t stream, bbfc_launch_shape *best);

/* Autotuner of one filter's kernels: times each shape (lanes per key 8|4,
 * tiles per wavefront 1|2, workgroups per CU unbounded|2) of `op` on
 * d_keys[0..n), `reps` timed runs each after one warm-up, and makes the
 * fastest the filter's shape for `op` (returned in *best, may be null);
 * the shape and insert tile in force are kept unless another is more than
 * 2% faster. For inserts the shapes run in tiles of 64 keys and one more
 * trial runs in tiles of 8 keys; the winner's tile becomes the filter's
 * BBFC_OPT_INSERT_TILE (unchanged when the tile in force wins), under the
 * filter's bound on keys in flight.
 * Insert trials run on a snapshot (8*n_blocks words of device memory for
 * the duration), restored before every trial and at the end, so the
 * filter is unchanged on return; query trials write d_out_bits. The same
 * call sequence the tuner times is what a later bbfc_insert/bbfc_query
 * launches. Synchronises `stream`. */
bbfc_status bbfc_tune(bbfc_handle h, int32_t op, const uint64_t *d_keys, uint64_t n, uint64_t *d_out_bits,
                      uint32_t reps, hipStream_t stream, bbfc_launch_shape *best);

/* ------------------------------------------------------------------ */
/* Graphs: batch launches captured once and replayed.                    */
/* ------------------------------------------------------------------ */

typedef struct bbfc_graph *bbfc_graph_handle;

/* Captures into one executable hipGraph the launches of
 * bbfc_batch_insert(insert_plan, d_insert_keys) followed by
 * bbfc_batch_query(query_plan, d_query_keys, d_out_bits); either plan may
 * be null (not both). The graph keeps its own copy of the plans' tables as
 * of capture time (later shape changes do not affect it) and records the
 * buffer addresses, which must stay valid while the graph is used. The
 * captured kernels contain no memset nodes. */
bbfc_status bbfc_graph_create(bbfc_batch_handle insert_plan, const uint64_t *d_insert_keys,
                              bbfc_batch_handle query_plan, const uint64_t *d_query_keys, uint64_t *d_out_bits,
                              bbfc_graph_handle *out);
bbfc_status bbfc_graph_launch(bbfc_graph_handle g, hipStream_t stream);
/* Synchronises the device, then frees the graph and its tables. */
bbfc_status bbfc_graph_destroy(bbfc_graph_handle g);

/* ------------------------------------------------------------------ */
/* Serving: query requests of mixed sizes from host memory, continuously  */
/* batched against one resident filter.                                   */
/* ------------------------------------------------------------------ */

typedef struct bbfc_server *bbfc_server_handle;

/* n_slots: batches that may be in flight at once, each on its own stream
 *     (1..16); max_batch_keys: keys one batch stages (a multiple of 64,
 *     64..2^30; pinned host and device memory of 8 bytes per key plus
 *     answers is allocated per slot); max_pending_keys: admission limit on
 *     keys submitted but not yet staged (a request is still admitted when
 *     nothing is pending, whatever its size); poll_us: a slot's worker polls
 *     its batch for completion, yielding between polls for the first 1 ms
 *     and then sleeping poll_us between polls (0: yielding throughout);
 *     batch_window_us: while other batches are on the device, the worker
 *     gathering the next batch waits up to this long after the oldest
 *     pending request's arrival for more requests (or until half a batch is
 *     pending); with the device idle a batch goes at once (0: never wait).
 *     Both at most 100000. Defaults (config == NULL): 4 slots, 2^20 keys per
 *     batch, 2^28 pending keys, 20 us, 0. */
typedef struct {
    uint32_t n_slots;
    uint64_t max_batch_keys;
    uint64_t max_pending_keys;
    uint32_t poll_us;
    uint32_t batch_window_us;
} bbfc_server_config;

/* Writes the defaults that config == NULL stands for into *config.
 * Errors: EINVAL (null config). */
bbfc_status bbfc_server_default_config(bbfc_server_config *config);

/* Starts one worker thread per slot serving queries on `filter`. Requests
 * that arrive while others are in flight are admitted into the next batch
 * as slots and memory free up: the oldest pending work fills a free slot's
 * batch (each request's part starts on a 64-key boundary; a request larger
 * than the room left continues in the next batch), and every batch is one
 * key upload, one query launch (the filter's query shape) and one answer
 * download on its slot's stream. Answers are those of bbfc_query on the
 * same keys, whatever the mix. The filter must outlive the server;
 * inserting into it while serving is allowed (queries see some subset of
 * the in-flight inserts). Errors: EINVAL, EHIP. */
bbfc_status bbfc_server_create(bbfc_handle filter, const bbfc_server_config *config, bbfc_server_handle *out);

/* Waits for the admitted requests, stops the threads and frees the server. */
bbfc_status bbfc_server_destroy(bbfc_server_handle s);

/* Submits a query of h_keys[0..n) (host memory). On completion
 * ceil(n/64) words of h_out_bits (host memory) hold the packed answers, as
 * bbfc_query writes them. Both buffers must stay valid until the request
 * is waited for. Thread-safe. Errors: EINVAL, EBUSY (admission: the
 * pending keys would exceed max_pending_keys; retry later), EHIP (an
 * earlier device error stopped the server). */
bbfc_status bbfc_server_submit(bbfc_server_handle s, const uint64_t *h_keys, uint64_t n, uint64_t *h_out_bits,
                               uint64_t *ticket);

/* As bbfc_server_submit, with the keys d_keys[0..n) and the answers
 * d_out_bits[0..ceil(n/64)) in device memory on the filter's device
 * (caller-owned; they must not overlap). Nothing is staged: the request
 * joins the same queue, and a batch of such requests is one query launch
 * that reads each request's keys in place and writes its answers straight
 * into its buffer (bbfc_query's layout). A batch holds requests of one
 * kind (host or device) and at most 1024 request pieces. The buffers must
 * stay valid, and the keys unchanged, until the request is waited for;
 * after bbfc_server_wait returns, the answers are in device memory and
 * need no further synchronisation. Errors as bbfc_server_submit, and
 * EINVAL when the output overlaps the keys. */
bbfc_status bbfc_server_submit_device(bbfc_server_handle s, const uint64_t *d_keys, uint64_t n,
                                      uint64_t *d_out_bits, uint64_t *ticket);

/* Waits for a request (timeout_s < 0: no limit) and forgets its ticket
 * (wait once per ticket). *latency_us (may be null) receives the time from
 * submission to answers in the caller's buffer. Errors: EINVAL (unknown
 * ticket), EBUSY (timed out; the ticket stays valid), EHIP. */
bbfc_status bbfc_server_wait(bbfc_server_handle s, uint64_t ticket, double timeout_s, double *latency_us);

/* Batches launched, keys staged in them (with padding) and requests done. */
bbfc_status bbfc_server_stats(bbfc_server_handle s, uint64_t *batches, uint64_t *batched_keys, uint64_t *completed);

/* Measurement driver: submits request i = keys h_keys[req_offsets[i] ..
 * req_offsets[i+1]) at arrival_s[i] seconds after the call (non-decreasing;
 * busy-waits to each arrival; retries when admission is full), its answers
 * to h_out_bits + out_offsets[i], then waits for all. latency_us[i] counts
 * from the scheduled arrival, so admission waits are included. *wall_s (may
 * be null) receives the time from the start to the last answer. */
bbfc_status bbfc_server_replay(bbfc_server_handle s, const uint64_t *h_keys, const uint64_t *req_offsets,
                               uint32_t n_requests, const double *arrival_s, uint64_t *h_out_bits,
                               const uint64_t *out_offsets, double *latency_us, double *wall_s);

/* bbfc_server_replay for device-resident requests: request i reads
 * d_keys[req_offsets[i] .. req_offsets[i+1]) in place and its answers go to
 * d_out_bits + out_offsets[i] (both device memory; the offset arrays,
 * arrival times and latencies are host memory), each submitted as by
 * bbfc_server_submit_device at its arrival time. */
bbfc_status bbfc_server_replay_device(bbfc_server_handle s, const uint64_t *d_keys, const uint64_t *req_offsets,
                                      uint32_t n_requests, const double *arrival_s, uint64_t *d_out_bits,
                                      const uint64_t *out_offsets, double *latency_us, double *wall_s);

/* ------------------------------------------------------------------ */
/* Measurement hooks: the kernels that calibrate the roofline. They do   */
/* not touch any filter.                                                  */
/* ------------------------------------------------------------------ */

/* Random line gathers: n_access reads of whole lines of access_bytes (64
 * or 128) bytes at pseudo-random access_bytes-aligned positions of d_buf,
 * which holds n_lines64 64-byte lines (a power of two, >= 2), access_bytes/8
 * lanes per line, as the filter kernels read blocks (64). Writes at most
 * one word per workgroup into d_sink (>= 65536 words). */
bbfc_status bbfc_probe_gather(const uint64_t *d_buf, uint64_t n_lines64, uint32_t access_bytes, uint64_t n_access,
                              uint64_t seed, uint64_t *d_sink, hipStream_t stream);

/* Random 64-bit atomic ORs: n_access lines, eight lanes each ORing one
 * word of the line, as the insert kernel writes (n_lines a power of two). */
bbfc_status bbfc_probe_atomic64(uint64_t *d_buf, uint64_t n_lines, uint64_t n_access, uint64_t seed,
                                hipStream_t stream);

/* The insert's memory pattern with a stand-in for its arithmetic: n_keys
 * keys, each reading two random 64-byte lines of d_buf (n_lines lines, a
 * power of two; eight lanes per line). mask_bits == 0: reads only. mask_bits
 * in [1, 32]: each key also draws a mask of that many random bit positions,
 * picks the line that gains fewer new bits and ORs the mask into it with
 * 64-bit atomics on the words that gain a bit (at most one line rewritten per
 * key, after both reads, as in bbfc_insert). Writes at most one word per
 * workgroup into d_sink (>= 65536 words). Measures what the device sustains
 * for the insert's pattern (compare with bbfc_insert on a buffer of the
 * filter's size, starting from zero). BBFC_EINVAL for null buffers, a line
 * count that is not a power of two, or mask_bits outside [0, 32]. */
bbfc_status bbfc_probe_insert_pattern(uint64_t *d_buf, uint64_t n_lines, uint64_t n_keys, int32_t mask_bits,
                                      uint64_t seed, uint64_t *d_sink, hipStream_t stream);

/* The insert's pattern of bbfc_probe_insert_pattern (mask_bits in [1, 32])
 * under three schedules, to locate the insert's ceiling:
 *   0  as bbfc_probe_insert_pattern: a unit's reads, then its atomics;
 *   1  pipelined: a wavefront decides a unit's 64 keys, then issues their
 *      atomics (an OR of zero where a word gains nothing) and right after
 *      them the next unit's reads, so no wait for reads covers atomics;
 *   2  the line that receives the mask is chosen from the key alone, not
 *      from the words read, so the atomics do not wait for the reads (the
 *      reads are still made; their words are summed into d_sink's
 *      condition). Not an insert: it measures the same traffic without the
 *      dependency of the write on the reads.
 * Arguments and errors as bbfc_probe_insert_pattern, plus EINVAL for
 * another schedule. */
bbfc_status bbfc_probe_insert_schedule(uint64_t *d_buf, uint64_t n_lines, uint64_t n_keys, int32_t mask_bits,
                                       int32_t schedule, uint64_t seed, uint64_t *d_sink, hipStream_t stream);

/* Round-trip latency of one wavefront's dependent memory steps: `waves`
 * workgroups of one wavefront (1..1024) each time `iters` steps (1..2^20)
 * with the device's constant-rate clock and write the mean nanoseconds
 * per step to d_out[w] (device memory, `waves` doubles). d_buf holds
 * n_lines 64-byte lines (a power of two, >= 8); eight lanes share a line,
 * as in the filter kernels. kind 0: a random line read whose address
 * depends on the previous read; 1: a random 64-bit atomic OR and the wait
 * for it (sets bits in d_buf); 2: a random line read, then an atomic OR
 * into the line just read, and the wait for both (the racing insert's
 * round trip); 3: a coalesced 512-byte load of the next words of d_buf
 * (read as a key stream), its address depending on the previous load.
 * Errors: EINVAL for null buffers or arguments out of range; EHIP. */
bbfc_status bbfc_probe_latency(uint64_t *d_buf, uint64_t n_lines, int32_t kind, uint32_t iters, uint32_t waves,
                               double *d_out, hipStream_t stream);

/* Plain copy of n_words words, to calibrate the traffic counters. With
 * request_bytes == 128 every lane moves 16 contiguous bytes (128-byte
 * requests, a streaming copy; an odd last word is not copied). With
 * request_bytes == 64 every group of eight lanes moves one 64-byte half of a
 * 128-byte line per instruction, the low halves first, then the high halves
 * (64-byte requests, the size of a filter block read); n_words must then be
 * a multiple of 128. Errors: EINVAL for null buffers, another request size
 * or a bad n_words; EHIP. */
bbfc_status bbfc_probe_copy(const uint64_t *d_src, uint64_t *d_dst, uint64_t n_words, uint32_t request_bytes,
                            hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Host-side checks of the device hashing code (no device needed).      */
/* ------------------------------------------------------------------ */

/* Block index h(x) in [0, n_blocks) for multiplier a, through the same
 * source the kernels compile (Section 3.4). */
uint64_t bbfc_host_block_hash(uint64_t n_blocks, uint64_t a, uint64_t x);

/* Candidate block of key x for block multiplier a in a filter of n_blocks
 * blocks in `subarrays` sub-arrays with h_0 multiplier sub_mult: h_0(x) S +
 * h(x), through the same source the kernels compile. Returns 0 when
 * n_blocks is 0 or subarrays does not divide it. */
uint64_t bbfc_host_block_index(uint64_t n_blocks, uint64_t subarrays, uint64_t sub_mult, uint64_t a, uint64_t x);

/* Bit address f(x) in [0, 512) for multiplier a (Section 3.4, b = 2^9). */
uint32_t bbfc_host_bit_hash(uint64_t a, uint64_t x);

/* The key's address set F(x) (Section 3.3, eq. bitset; App. B for
 * DISTINCT) as a 512-bit mask: bit f is bit f%64 of out[f/64], out[8] host
 * memory. bit_mult[k] are the bit multipliers. Errors: EINVAL for null
 * pointers, k outside [1, 32] or an unknown bit_selection. */
bbfc_status bbfc_host_key_mask(const uint64_t *bit_mult, uint32_t k, int32_t bit_selection, uint64_t x,
                               uint64_t *out);

#ifdef __cplusplus
}
#endif

#endif /* BBFC_H */
