/*
 * Sequential CPU oracle for Blocked Bloom filters with choices
 * (Schmitz, Zentgraf, Rahmann, "Blocked Bloom Filters with Choices",
 * arXiv 2501.18977).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers. The HIP library never
 * links, loads or calls this file, and this file includes nothing of the HIP
 * library: the two sides share no code, header, table or constant.
 *
 * What it computes is the paper's definition executed one key at a time in
 * key order, with no blocking, batching or reordering:
 *
 *   filter    M blocks of 512 bits; block b is the eight 64-bit words
 *             W[8b .. 8b+7]; bit f of a block is bit (f mod 64) of word
 *             (f div 64)                         (Section 2.2; reading R2)
 *   layout    T sub-arrays of S = M/T blocks; h_0(x) in [T] picks the
 *             sub-array and h_i(x) in [S] the block inside it, so candidate
 *             i is block h_0(x) S + h_i(x); T = 1 is a single array
 *                                      (Section 3.4, "Parallelization")
 *   F(x)      { f_i(x) : i = 1..k }, f_i random-strategy bit hashes into
 *             [512]                  (Section 3.1 eq. bitset; Section 3.3),
 *             or k distinct addresses by the insertion procedure of App. B
 *   j, a      for a candidate block with bit set F':
 *             j = |F' u F(x)|, a = |F(x) \ F'|    (Section 3.2; App. A)
 *   insert    no-op if some candidate already holds all of F(x); otherwise
 *             F(x) is set in the candidate of lowest cost, the first one
 *             on equal cost                        (Sections 3.1, 3.2; R5)
 *   query     true iff F(x) is a subset of some candidate block
 *                                                           (Section 3.1)
 *
 * Readings of points the paper leaves open (each one is restated where it
 * is used):
 *   R1  keys are u = 64-bit words for every hash.
 *   R3  hash multipliers are odd, >= 2^32, coprime to the modulus; the
 *       default set comes from a SplitMix64 stream (Steele, Lea, Flood 2014)
 *       seeded by the filter seed: c block multipliers, then k bit ones,
 *       then the sub-array multiplier when there are sub-arrays.
 *   R4  a modulus of 1 hashes every key to 0.
 *   R5  on equal cost the lower choice index wins.
 *   R6  costs are IEEE-754 double, evaluated left to right as written in
 *       bbo_cost; equal doubles are ties.
 *   R7  the k in a/k and in the MIX/LA power is the parameter k.
 *
 * Pins that hold this file to the paper rather than to itself live in the
 * test suite: a set-based Python restatement on tiny inputs, the exact
 * one-choice false-positive closed form, the cost identities the paper
 * states, the M = 1 and c = 1 reductions, and zero false negatives.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BBO_COST_NONE 0
#define BBO_COST_MIX 1
#define BBO_COST_LA 2
#define BBO_COST_EXP 3

/* ------------------------------------------------------------------ */
/* Linear hash x -> ((a*x) mod 2^64) mod b, with the two modifications   */
/* for even b (Section 3.4, "Hash functions"):                           */
/*   b = 2^s      : the s most significant bits of a*x (u = 64, R1)      */
/*   b even       : (p xor (p >> 32)) mod b, q = floor(64/2) = 32        */
/*   b odd        : p mod b                                              */
/*   b = 1        : 0 (R4; avoids a shift by 64)                         */
/* ------------------------------------------------------------------ */
uint64_t bbo_hash(uint64_t a, uint64_t x, uint64_t b)
{
    uint64_t p = a * x; /* unsigned arithmetic wraps: mod 2^64 */
    if (b == 1)
        return 0;
    if ((b & (b - 1)) == 0) {
        unsigned s = 0;
        while (((uint64_t)1 << s) != b)
            s++;
        return p >> (64 - s);
    }
    if ((b & 1) == 0)
        return (p ^ (p >> 32)) % b;
    return p % b;
}

/* Where a key's candidates lie (Section 3.4, "Parallelization"): the M
 * blocks form T sub-arrays of S = M/T blocks each (T divides M); h_0, with
 * its own multiplier, picks the sub-array, and the block hashes h_i map into
 * [S]. T = 1 is the single array of Section 3.1 (h_0 = 0 by R4, S = M). */
typedef struct {
    uint64_t M;        /* blocks in the filter */
    uint64_t T;        /* sub-arrays */
    uint64_t sub_mult; /* multiplier of h_0; unused when T = 1 */
} bbo_layout;

/* Index of the block that block hash a selects for key x. */
uint64_t bbo_block(const bbo_layout *L, uint64_t a, uint64_t x)
{
    uint64_t S = L->M / L->T;
    return bbo_hash(L->sub_mult, x, L->T) * S + bbo_hash(a, x, S);
}

/* F(x) as a 512-bit mask (eq. bitset; random bit selection, Section 3.3). */
void bbo_mask(const uint64_t *bit_mult, uint32_t k, uint64_t x, uint64_t m[8])
{
    memset(m, 0, 8 * sizeof(uint64_t));
    for (uint32_t i = 0; i < k; i++) {
        uint64_t f = bbo_hash(bit_mult[i], x, 512);
        m[f / 64] |= (uint64_t)1 << (f % 64);
    }
}

/* Paper defaults for the cost parameter: sigma = 2.5 for k = 7 and 50 for
 * k = 14, mu = 3.5, beta = golden ratio (App. C, caption of the load
 * histogram figure; Section 4). For other k the MIX sigma of the nearer
 * printed k is used (R8). */
double bbo_default_param(int kind, uint32_t k)
{
    switch (kind) {
    case BBO_COST_MIX:
        return (k <= 10) ? 2.5 : 50.0;
    case BBO_COST_LA:
        return 3.5;
    case BBO_COST_EXP:
        return (1.0 + sqrt(5.0)) / 2.0;
    default:
        return 0.0;
    }
}

/* Insertion cost of a block that would hold j bits after the insertion, a
 * of them new (App. A eq. cost:mix, eq. cost:la, eq. cost:exp; Section 3.2
 * eq. cost:exp). Evaluated left to right as written (R6). */
double bbo_cost(int kind, double param, uint32_t k, uint32_t j, uint32_t a)
{
    switch (kind) {
    case BBO_COST_MIX: /* sigma * k * (j/256)^k + a */
        return param * (double)k * pow((double)j / 256.0, (double)k) + (double)a;
    case BBO_COST_LA: /* k * ((j + mu*k)/256)^k + a */
        return (double)k * pow(((double)j + param * (double)k) / 256.0, (double)k) + (double)a;
    case BBO_COST_EXP: /* beta^(j/128) + a/k */
        return pow(param, (double)j / 128.0) + (double)a / (double)k;
    default:
        return 0.0;
    }
}

/* Number of set bits of a word (the popcount of Section 3.4 / App. A). */
static unsigned popc64(uint64_t v)
{
    return (unsigned)__builtin_popcountll(v);
}

/* Distinct bit selection (Section 3.3, App. B), on raw values: raw[i] lies
 * in [512 - i] (i counted from 0); it is increased by one for every address
 * already chosen that is at or below its current value, scanning the chosen
 * addresses in increasing order, which are kept sorted. Writes the k
 * distinct addresses, sorted, to out. */
void bbo_distinct_positions(const uint32_t *raw, uint32_t k, uint32_t *out)
{
    uint32_t used = 0;
    for (uint32_t i = 0; i < k; i++) {
        uint32_t v = raw[i];
        uint32_t pos = 0;
        while (pos < used && out[pos] <= v) { /* every occupied address at or below v */
            v++;
            pos++;
        }
        for (uint32_t t = used; t > pos; t--) /* insertion keeps the addresses sorted */
            out[t] = out[t - 1];
        out[pos] = v;
        used++;
    }
}

/* F(x) under distinct bit selection: f_i hashed into [512 - i + 1]
 * (modulus 513 - i for i = 1..k, the hash of Section 3.4), then made
 * distinct as above. */
void bbo_mask_distinct(const uint64_t *bit_mult, uint32_t k, uint64_t x, uint64_t m[8])
{
    uint32_t raw[32] = {0}, pos[32] = {0};
    memset(m, 0, 8 * sizeof(uint64_t));
    for (uint32_t i = 0; i < k; i++)
        raw[i] = (uint32_t)bbo_hash(bit_mult[i], x, 512 - i);
    bbo_distinct_positions(raw, k, pos);
    for (uint32_t i = 0; i < k; i++)
        m[pos[i] / 64] |= (uint64_t)1 << (pos[i] % 64);
}

/* F(x) as a mask under either strategy: 0 random (Section 3.3), 1 distinct. */
static void bbo_mask_sel(int distinct, const uint64_t *bit_mult, uint32_t k, uint64_t x, uint64_t m[8])
{
    if (distinct)
        bbo_mask_distinct(bit_mult, k, x, m);
    else
        bbo_mask(bit_mult, k, x, m);
}

/* Insert one key (Sections 3.1, 3.2). Returns the chosen choice index, or
 * -1 when some candidate already contains F(x). */
int bbo_insert_one(uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct, int kind, double param,
                   const uint64_t *block_mult, const uint64_t *bit_mult, uint64_t x)
{
    uint64_t m[8];
    uint64_t blk[8];
    uint32_t j[8], a[8];
    bbo_mask_sel(distinct, bit_mult, k, x, m);
    for (uint32_t i = 0; i < c; i++) {
        blk[i] = bbo_block(L, block_mult[i], x);
        const uint64_t *B = W + 8 * blk[i];
        unsigned before = 0, after = 0;
        for (int w = 0; w < 8; w++) {
            before += popc64(B[w]);
            after += popc64(B[w] | m[w]);
        }
        j[i] = after;
        a[i] = after - before;
    }
    for (uint32_t i = 0; i < c; i++)
        if (a[i] == 0)
            return -1; /* already present: nothing to set */
    uint32_t best = 0;
    if (c > 1) {
        double best_cost = bbo_cost(kind, param, k, j[0], a[0]);
        for (uint32_t i = 1; i < c; i++) {
            double ci = bbo_cost(kind, param, k, j[i], a[i]);
            if (ci < best_cost) { /* strict: the first minimum wins (R5) */
                best = i;
                best_cost = ci;
            }
        }
    }
    uint64_t *B = W + 8 * blk[best];
    for (int w = 0; w < 8; w++)
        B[w] |= m[w];
    return (int)best;
}

/* Sequential insertion of keys[0..n) in order. Returns how many keys set
 * at least one bit. */
uint64_t bbo_insert(uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct, int kind, double param,
                    const uint64_t *block_mult, const uint64_t *bit_mult, const uint64_t *keys,
                    uint64_t n)
{
    uint64_t written = 0;
    for (uint64_t t = 0; t < n; t++)
        if (bbo_insert_one(W, L, c, k, distinct, kind, param, block_mult, bit_mult, keys[t]) >= 0)
            written++;
    return written;
}

/* Query one key: F(x) subset of some candidate block (Section 3.1). */
int bbo_query_one(const uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct,
                  const uint64_t *block_mult, const uint64_t *bit_mult, uint64_t x)
{
    uint64_t m[8];
    bbo_mask_sel(distinct, bit_mult, k, x, m);
    for (uint32_t i = 0; i < c; i++) {
        const uint64_t *B = W + 8 * bbo_block(L, block_mult[i], x);
        int all = 1;
        for (int w = 0; w < 8; w++)
            if ((B[w] & m[w]) != m[w])
                all = 0;
        if (all)
            return 1;
    }
    return 0;
}

/* Queries keys[0..n); bit t of out_bits[t/64] (least significant first) is
 * the answer for keys[t]; bits past n in the last word are zero. Returns the
 * number of positive answers. */
uint64_t bbo_query(const uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct,
                   const uint64_t *block_mult, const uint64_t *bit_mult, const uint64_t *keys, uint64_t n,
                   uint64_t *out_bits)
{
    uint64_t hits = 0;
    if (out_bits)
        memset(out_bits, 0, ((n + 63) / 64) * sizeof(uint64_t));
    for (uint64_t t = 0; t < n; t++) {
        int h = bbo_query_one(W, L, c, k, distinct, block_mult, bit_mult, keys[t]);
        hits += (uint64_t)h;
        if (h && out_bits)
            out_bits[t / 64] |= (uint64_t)1 << (t % 64);
    }
    return hits;
}

/* SplitMix64 (Steele, Lea, Flood 2014): state += golden gamma, then the
 * variant-13 finaliser. */
static uint64_t splitmix_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ull;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* Default hash multipliers of a filter with seed `seed` (Section 3.4's
 * "random large integer a, coprime with b"; reading R3): one SplitMix64
 * stream; each draw is made odd; draws below 2^32 or sharing a factor with
 * the modulus are skipped. Block multipliers come first (modulus S = M/T),
 * then bit multipliers (modulus 512, or 512 - i for the i-th with distinct
 * bit selection, counting from 0), then, with T > 1 sub-arrays, the
 * multiplier of h_0 (modulus T). */
void bbo_derive_multipliers(uint64_t seed, uint64_t M, uint64_t T, uint32_t c, uint32_t k, int distinct,
                            uint64_t *block_mult, uint64_t *bit_mult, uint64_t *sub_mult)
{
    uint64_t st = seed;
    uint64_t S = M / T;
    for (uint32_t i = 0; i < c;) {
        uint64_t a = splitmix_next(&st) | 1;
        if (a >= ((uint64_t)1 << 32) && gcd64(a, S) == 1)
            block_mult[i++] = a;
    }
    for (uint32_t i = 0; i < k;) {
        uint64_t a = splitmix_next(&st) | 1;
        uint64_t b = distinct ? 512 - i : 512; /* modulus of bit hash i */
        if (a >= ((uint64_t)1 << 32) && gcd64(a, b) == 1)
            bit_mult[i++] = a;
    }
    *sub_mult = 0;
    while (T > 1) {
        uint64_t a = splitmix_next(&st) | 1;
        if (a >= ((uint64_t)1 << 32) && gcd64(a, T) == 1) {
            *sub_mult = a;
            break;
        }
    }
}

/* ----------------------- test-only comparators ----------------------- */

/* Every key's mask ORed into all of its candidates. Any correct filter of
 * these keys (sequential or with racing inserts) is bitwise contained in
 * this envelope, since bits only ever come from some key's mask placed in
 * one of its candidates. */
void bbo_envelope(uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct,
                  const uint64_t *block_mult, const uint64_t *bit_mult, const uint64_t *keys, uint64_t n)
{
    uint64_t m[8];
    for (uint64_t t = 0; t < n; t++) {
        bbo_mask_sel(distinct, bit_mult, k, keys[t], m);
        for (uint32_t i = 0; i < c; i++) {
            uint64_t *B = W + 8 * bbo_block(L, block_mult[i], keys[t]);
            for (int w = 0; w < 8; w++)
                B[w] |= m[w];
        }
    }
}

/* A filter from per-key decisions (Sections 3.1, 3.2): insert(x) either
 * finds F(x) already held by a candidate and writes nothing, or sets F(x) in
 * exactly one candidate. So a build whose decisions are known is the OR,
 * over the keys that wrote, of F(x) placed in the candidate they name.
 * decision[t] = i < c names candidate i (block h_{i+1}(keys[t])); any value
 * >= c means the key wrote nothing. Only blocks b with b mod part_mod ==
 * part_rem are written (part_mod 1: every block), so a large build can be
 * checked one residue class at a time. Returns the number of keys placed. */
uint64_t bbo_place(uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct,
                   const uint64_t *block_mult, const uint64_t *bit_mult, const uint64_t *keys,
                   const uint8_t *decision, uint64_t n, uint64_t part_mod, uint64_t part_rem)
{
    uint64_t m[8];
    uint64_t placed = 0;
    for (uint64_t t = 0; t < n; t++) {
        if (decision[t] >= c)
            continue;
        uint64_t b = bbo_block(L, block_mult[decision[t]], keys[t]);
        if (b % part_mod != part_rem)
            continue;
        bbo_mask_sel(distinct, bit_mult, k, keys[t], m);
        for (int w = 0; w < 8; w++)
            W[8 * b + w] |= m[w];
        placed++;
    }
    return placed;
}

/* Histogram of set bits per block: hist[P] = number of blocks with P bits
 * set, P in [0, 512]. */
void bbo_block_loads(const uint64_t *W, uint64_t M, uint64_t *hist)
{
    memset(hist, 0, 513 * sizeof(uint64_t));
    for (uint64_t b = 0; b < M; b++) {
        unsigned P = 0;
        for (int w = 0; w < 8; w++)
            P += popc64(W[8 * b + w]);
        hist[P]++;
    }
}

/* Low-variance false-positive estimate over negative keys (the "FPR from
 * the block loads" that Section 4.1 mentions): for each key, the exact
 * probability that k independent uniform bit addresses (or, distinct, k
 * distinct uniform ones) all fall inside one of its candidate blocks, given
 * those blocks' actual contents, by
 * inclusion-exclusion over the non-empty subsets I of choices:
 *   sum_I (-1)^(|I|+1) (|intersection of S_i, i in I| / 512)^k.
 * Returns the mean over the keys. */
double bbo_conditional_fpr(const uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct,
                           const uint64_t *block_mult, const uint64_t *keys, uint64_t n)
{
    double total = 0.0;
    for (uint64_t t = 0; t < n; t++) {
        uint64_t blk[8];
        for (uint32_t i = 0; i < c; i++)
            blk[i] = bbo_block(L, block_mult[i], keys[t]);
        double p = 0.0;
        for (uint32_t sub = 1; sub < (1u << c); sub++) {
            unsigned size = 0, inter = 0;
            for (int w = 0; w < 8; w++) {
                uint64_t acc = ~(uint64_t)0;
                for (uint32_t i = 0; i < c; i++)
                    if (sub & (1u << i))
                        acc &= W[8 * blk[i] + w];
                inter += popc64(acc);
            }
            for (uint32_t i = 0; i < c; i++)
                size += (sub >> i) & 1u;
            double term;
            if (!distinct) {
                term = pow((double)inter / 512.0, (double)k);
            } else { /* k distinct uniform addresses: C(inter, k) / C(512, k) */
                term = 1.0;
                for (uint32_t i = 0; i < k; i++)
                    term *= (inter > i) ? (double)(inter - i) / (double)(512 - i) : 0.0;
            }
            p += (size & 1) ? term : -term;
        }
        total += p;
    }
    return n ? total / (double)n : 0.0;
}

/* ------------------------- DNA q-grams as keys ------------------------ */

/* Canonical q-grams of a DNA sequence given one base per byte (A=0, C=1,
 * G=2, T=3), cut into n_segments segments of seg_len bases (Section 4.3:
 * genomes and reads represented by their q-grams). For every window of q
 * bases inside a segment, in order, the forward value reads the bases as a
 * base-4 number with the first base most significant; the reverse
 * complement reads the complemented bases (b -> 3 - b) from the last to the
 * first; the key is the smaller value. Returns the number of keys written. */
uint64_t bbo_qgrams(const uint8_t *bases, uint64_t n_segments, uint64_t seg_len, uint32_t q, uint64_t *out)
{
    uint64_t t = 0;
    if (q < 1 || q > 32 || seg_len < q)
        return 0;
    for (uint64_t s = 0; s < n_segments; s++) {
        const uint8_t *seg = bases + s * seg_len;
        for (uint64_t j = 0; j + q <= seg_len; j++) {
            uint64_t fwd = 0, rc = 0;
            for (uint32_t i = 0; i < q; i++)
                fwd = fwd * 4 + seg[j + i];
            for (uint32_t i = 0; i < q; i++)
                rc = rc * 4 + (uint64_t)(3 - seg[j + q - 1 - i]);
            out[t++] = fwd < rc ? fwd : rc;
        }
    }
    return t;
}
