/*
 * A C program that drives the library through its C ABI alone (no Python,
 * no PyTorch): device buffers from hipMalloc, results checked against the
 * sequential oracle (oracle/liboracle.so), which is linked here as test
 * infrastructure. Exit status 0 when every check passes.
 *
 *  1. default multipliers of a seeded filter equal the oracle's derivation
 *     (Section 3.4, the random multipliers coprime to their modulus);
 *  2. the deterministic insert builds the oracle's filter word for word, and
 *     queries of inserted and new keys give the oracle's answer bits;
 *  3. the racing insert has no false negatives;
 *  4. argument errors return BBFC_EINVAL with a message and enqueue nothing;
 *  5. a filter with sub-arrays (Section 3.4) from bbfc_create_config, filled
 *     by the bulk insert in a caller-owned workspace, is the oracle's
 *     one-at-a-time build word for word;
 *  6. the racing insert that records its decisions, in tiles of 8 and of 64
 *     keys: every decision names a candidate or "present", and the oracle's
 *     placement of the decided keys' masks is the filter word for word
 *     (Sections 3.1, 3.2);
 *  7. the sequential insert without allocation, on an input larger than one
 *     window, equals the allocating one and the oracle, twice in a row;
 *  8. the server with device-resident requests (two slots of 8192 keys, so
 *     that large requests span several batches) answers as the oracle.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bbfc.h"

/* oracle entry points (oracle/bbfc_oracle.c) */
typedef struct {
    uint64_t M, T, sub_mult;
} bbo_layout;
uint64_t bbo_insert(uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct, int kind, double param,
                    const uint64_t *block_mult, const uint64_t *bit_mult, const uint64_t *keys, uint64_t n);
uint64_t bbo_query(const uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct,
                   const uint64_t *block_mult, const uint64_t *bit_mult, const uint64_t *keys, uint64_t n,
                   uint64_t *out_bits);
void bbo_derive_multipliers(uint64_t seed, uint64_t M, uint64_t T, uint32_t c, uint32_t k, int distinct,
                            uint64_t *block_mult, uint64_t *bit_mult, uint64_t *sub_mult);
double bbo_default_param(int kind, uint32_t k);
uint64_t bbo_place(uint64_t *W, const bbo_layout *L, uint32_t c, uint32_t k, int distinct, const uint64_t *block_mult,
                   const uint64_t *bit_mult, const uint64_t *keys, const uint8_t *decision, uint64_t n,
                   uint64_t part_mod, uint64_t part_rem);

static int failures = 0;

#define CHECK(cond, ...)                                                                                           \
    do {                                                                                                           \
        if (!(cond)) {                                                                                             \
            printf("FAIL %s:%d: ", __FILE__, __LINE__);                                                            \
            printf(__VA_ARGS__);                                                                                   \
            printf("\n");                                                                                          \
            failures++;                                                                                            \
        }                                                                                                          \
    } while (0)

#define HIP(call)                                                                                                  \
    do {                                                                                                           \
        hipError_t e_ = (call);                                                                                    \
        if (e_ != hipSuccess) {                                                                                    \
            printf("HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__);                          \
            exit(2);                                                                                               \
        }                                                                                                          \
    } while (0)

/* Counter-based SplitMix64 keys (Steele, Lea, Flood 2014): key(seed, i) is
 * the finaliser of seed + (i + 1) * golden gamma. */
static uint64_t key_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main(void)
{
    const uint64_t M = 3001; /* odd: the remainder case of the block hash */
    const uint32_t c = 3, k = 12;
    const uint64_t n = 50000, nq = 2 * n;
    bbfc_cost exp_cost = {BBFC_COST_EXP, NAN};

    /* 1. a seeded filter's parameters */
    bbfc_handle a = NULL;
    bbfc_status st = bbfc_create_seeded(M, c, k, exp_cost, 5, &a);
    CHECK(st == BBFC_OK, "create: %s", bbfc_last_error());
    if (st != BBFC_OK)
        return 1;
    uint64_t bm[4], am[32], obm[4], oam[32], osm = 0, pM = 0;
    uint32_t pc = 0, pk = 0;
    bbfc_cost pcost;
    CHECK(bbfc_get_params(a, &pM, &pc, &pk, &pcost, bm, am) == BBFC_OK, "get_params");
    bbo_derive_multipliers(5, M, 1, c, k, 0, obm, oam, &osm);
    CHECK(pM == M && pc == c && pk == k && pcost.kind == BBFC_COST_EXP, "params");
    CHECK(pcost.param == bbo_default_param(BBFC_COST_EXP, k), "EXP base %.17g", pcost.param);
    CHECK(memcmp(bm, obm, c * 8) == 0 && memcmp(am, oam, k * 8) == 0, "multipliers differ from the oracle's");

    /* 2. deterministic insert and query against the oracle */
    uint64_t *h_keys = malloc(nq * 8);
    for (uint64_t i = 0; i < nq; i++)
        h_keys[i] = key_at(7, i); /* [0, n) inserted, [n, 2n) never inserted */
    uint64_t *d_keys = NULL, *d_out = NULL;
    HIP(hipMalloc((void **)&d_keys, nq * 8));
    HIP(hipMalloc((void **)&d_out, (nq + 63) / 64 * 8));
    HIP(hipMemcpy(d_keys, h_keys, nq * 8, hipMemcpyHostToDevice));
    CHECK(bbfc_insert_deterministic(a, d_keys, n, NULL) == BBFC_OK, "insert_deterministic: %s", bbfc_last_error());
    CHECK(bbfc_query(a, d_keys, nq, d_out, NULL) == BBFC_OK, "query: %s", bbfc_last_error());
    uint64_t *got_words = malloc(M * 64), *want_words = calloc(M * 8, 8);
    uint64_t *got_bits = malloc((nq + 63) / 64 * 8), *want_bits = malloc((nq + 63) / 64 * 8);
    CHECK(bbfc_download(a, got_words, NULL) == BBFC_OK, "download");
    HIP(hipMemcpy(got_bits, d_out, (nq + 63) / 64 * 8, hipMemcpyDeviceToHost));
    const bbo_layout L = {M, 1, 0};
    bbo_insert(want_words, &L, c, k, 0, BBFC_COST_EXP, bbo_default_param(BBFC_COST_EXP, k), bm, am, h_keys, n);
    const uint64_t hits = bbo_query(want_words, &L, c, k, 0, bm, am, h_keys, nq, want_bits);
    CHECK(memcmp(got_words, want_words, M * 64) == 0, "deterministic insert differs from the oracle");
    CHECK(memcmp(got_bits, want_bits, (nq + 63) / 64 * 8) == 0, "query bits differ from the oracle");
    CHECK(hits >= n && hits < nq, "oracle hits %llu", (unsigned long long)hits);

    /* 3. racing insert: every inserted key answers true */
    bbfc_handle b = NULL;
    bbfc_cost la = {BBFC_COST_LA, NAN};
    CHECK(bbfc_create(4096, 2, 11, la, &b) == BBFC_OK, "create: %s", bbfc_last_error());
    CHECK(bbfc_insert(b, d_keys, n, NULL) == BBFC_OK, "insert: %s", bbfc_last_error());
    CHECK(bbfc_query(b, d_keys, n, d_out, NULL) == BBFC_OK, "query: %s", bbfc_last_error());
    HIP(hipMemcpy(got_bits, d_out, (n + 63) / 64 * 8, hipMemcpyDeviceToHost));
    uint64_t answered = 0;
    for (uint64_t t = 0; t < n; t++)
        answered += (got_bits[t / 64] >> (t % 64)) & 1;
    CHECK(answered == n, "racing insert: %llu of %llu keys answer true", (unsigned long long)answered,
          (unsigned long long)n);

    /* 4. argument errors */
    bbfc_handle bad = NULL;
    CHECK(bbfc_create(0, 2, 11, la, &bad) == BBFC_EINVAL && bad == NULL, "n_blocks 0 accepted");
    CHECK(strlen(bbfc_last_error()) > 0, "no error text");
    CHECK(bbfc_create(64, 2, 33, la, &bad) == BBFC_EINVAL, "k = 33 accepted");
    CHECK(bbfc_create(64, 1, 8, la, &bad) == BBFC_EINVAL, "one choice with a cost accepted");
    CHECK(bbfc_query(b, d_keys, 1024, d_keys + 8, NULL) == BBFC_EINVAL, "overlapping output accepted");
    CHECK(bbfc_insert(b, NULL, 10, NULL) == BBFC_EINVAL, "null keys accepted");
    CHECK(bbfc_insert(b, NULL, 0, NULL) == BBFC_OK, "an empty insert is not a no-op");
    CHECK(strcmp(bbfc_status_string(BBFC_EINVAL), "invalid argument") == 0, "status string");
    CHECK(bbfc_set_option(b, BBFC_OPT_INSERT_TILE, 3) == BBFC_EINVAL, "tile option 3 accepted");
    {
        /* 4096 blocks, two choices: the default bound is 4096/8 = 512 keys,
         * which takes tiles of 8 keys; forced tiles of 64 keep the bound */
        uint32_t tk = 0;
        uint64_t kif = 0, wg = 0;
        CHECK(bbfc_insert_launch_info(b, n, &tk, &kif, &wg) == BBFC_OK, "launch info: %s", bbfc_last_error());
        CHECK(tk == 8 && kif == 512 && wg == 16, "launch info: tile %u, %llu keys in flight, %llu workgroups", tk,
              (unsigned long long)kif, (unsigned long long)wg);
        CHECK(bbfc_set_option(b, BBFC_OPT_INSERT_TILE, 1) == BBFC_OK, "tile option");
        CHECK(bbfc_insert_launch_info(b, n, &tk, &kif, NULL) == BBFC_OK && tk == 64 && kif == 512,
              "launch info with tiles of 64: tile %u, %llu keys in flight", tk, (unsigned long long)kif);
        CHECK(bbfc_set_option(b, BBFC_OPT_INSERT_TILE, 0) == BBFC_OK, "tile option");
        CHECK(bbfc_insert_launch_info(NULL, n, &tk, &kif, &wg) == BBFC_EINVAL, "null handle accepted");
    }

    /* 5. sub-arrays and the bulk insert */
    {
        const uint64_t M5 = 1u << 14, T5 = 64; /* 256 blocks per sub-array */
        const uint32_t c5 = 2, k5 = 11;
        bbfc_config cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.n_blocks = M5;
        cfg.choices = c5;
        cfg.bits_per_key = k5;
        cfg.cost = la;
        cfg.bit_selection = BBFC_BITS_RANDOM;
        cfg.seed = 11;
        cfg.subarrays = T5;
        bbfc_handle s5 = NULL;
        CHECK(bbfc_create_config(&cfg, &s5) == BBFC_OK, "create_config: %s", bbfc_last_error());
        uint64_t ws_bytes = 0, T_got = 0, sm5 = 0, bm5[4], am5[32];
        bbfc_cost cost5;
        CHECK(bbfc_bulk_insert_workspace(s5, nq, &ws_bytes) == BBFC_OK && ws_bytes > 0, "workspace size");
        void *d_ws = NULL;
        HIP(hipMalloc(&d_ws, ws_bytes));
        CHECK(bbfc_bulk_insert(s5, d_keys, nq, d_ws, ws_bytes, NULL) == BBFC_OK, "bulk_insert: %s",
              bbfc_last_error());
        CHECK(bbfc_get_params(s5, NULL, NULL, NULL, &cost5, bm5, am5) == BBFC_OK, "get_params");
        CHECK(bbfc_get_subarrays(s5, &T_got, &sm5) == BBFC_OK && T_got == T5, "get_subarrays");
        uint64_t *got5 = malloc(M5 * 64), *want5 = calloc(M5 * 8, 8);
        CHECK(bbfc_download(s5, got5, NULL) == BBFC_OK, "download");
        const bbo_layout L5 = {M5, T5, sm5};
        bbo_insert(want5, &L5, c5, k5, 0, BBFC_COST_LA, cost5.param, bm5, am5, h_keys, nq);
        CHECK(memcmp(got5, want5, M5 * 64) == 0, "bulk insert with sub-arrays differs from the oracle");
        CHECK(bbfc_bulk_insert(s5, d_keys, nq, d_ws, ws_bytes - 1, NULL) == BBFC_EINVAL, "small workspace accepted");
        HIP(hipFree(d_ws));
        free(got5);
        free(want5);
        CHECK(bbfc_destroy(s5) == BBFC_OK, "destroy");
    }

    /* 6. the racing insert with recorded decisions, in tiles of 8 keys (the
     * default at this size) and of 64 keys */
    for (int tile = 2; tile >= 1; tile--) {
        const uint64_t M6 = 4096;
        bbfc_handle r6 = NULL;
        CHECK(bbfc_create_seeded(M6, 2, 11, la, 6, &r6) == BBFC_OK, "create: %s", bbfc_last_error());
        CHECK(bbfc_set_option(r6, BBFC_OPT_INSERT_TILE, tile) == BBFC_OK, "tile option");
        uint8_t *d_dec = NULL;
        HIP(hipMalloc((void **)&d_dec, n));
        CHECK(bbfc_insert_recorded(r6, d_keys, n, d_dec, NULL) == BBFC_OK, "insert_recorded: %s", bbfc_last_error());
        CHECK(bbfc_insert_recorded(r6, d_keys, 10, (uint8_t *)d_keys + 8, NULL) == BBFC_EINVAL,
              "decisions overlapping the keys accepted");
        uint8_t *dec = malloc(n);
        HIP(hipMemcpy(dec, d_dec, n, hipMemcpyDeviceToHost));
        uint64_t bm6[4], am6[32];
        CHECK(bbfc_get_params(r6, NULL, NULL, NULL, NULL, bm6, am6) == BBFC_OK, "get_params");
        uint64_t bad_dec = 0;
        for (uint64_t t = 0; t < n; t++)
            bad_dec += dec[t] >= 2 && dec[t] != BBFC_DECISION_PRESENT;
        CHECK(bad_dec == 0, "%llu decisions name no candidate", (unsigned long long)bad_dec);
        uint64_t *got6 = malloc(M6 * 64), *want6 = calloc(M6 * 8, 8);
        CHECK(bbfc_download(r6, got6, NULL) == BBFC_OK, "download");
        const bbo_layout L6 = {M6, 1, 0};
        bbo_place(want6, &L6, 2, 11, 0, bm6, am6, h_keys, dec, n, 1, 0);
        CHECK(memcmp(got6, want6, M6 * 64) == 0, "tile option %d: the recorded decisions do not rebuild the filter",
              tile);
        HIP(hipFree(d_dec));
        free(dec);
        free(got6);
        free(want6);
        CHECK(bbfc_destroy(r6) == BBFC_OK, "destroy");
    }

    /* 7. the sequential insert without allocation (inputs above one window use
     * the static scratch), twice in a row, against the allocating insert and
     * the oracle */
    for (int call = 0; call < 2; call++) {
        const uint64_t n7 = call == 0 ? nq : nq - 20000; /* both above 2^16 keys */
        bbfc_handle x = NULL, y = NULL;
        CHECK(bbfc_create_seeded(M, c, k, exp_cost, 5, &x) == BBFC_OK, "create");
        CHECK(bbfc_create_seeded(M, c, k, exp_cost, 5, &y) == BBFC_OK, "create");
        CHECK(bbfc_insert_deterministic_noalloc(x, d_keys, n7, NULL) == BBFC_OK, "noalloc: %s", bbfc_last_error());
        CHECK(bbfc_insert_deterministic(y, d_keys, n7, NULL) == BBFC_OK, "deterministic: %s", bbfc_last_error());
        uint64_t *wx = malloc(M * 64), *wy = malloc(M * 64), *wo = calloc(M * 8, 8);
        CHECK(bbfc_download(x, wx, NULL) == BBFC_OK && bbfc_download(y, wy, NULL) == BBFC_OK, "download");
        bbo_insert(wo, &L, c, k, 0, BBFC_COST_EXP, bbo_default_param(BBFC_COST_EXP, k), bm, am, h_keys, n7);
        CHECK(memcmp(wx, wy, M * 64) == 0, "call %d: the no-allocation insert differs from the allocating one", call);
        CHECK(memcmp(wx, wo, M * 64) == 0, "call %d: the no-allocation insert differs from the oracle", call);
        free(wx);
        free(wy);
        free(wo);
        CHECK(bbfc_destroy(x) == BBFC_OK && bbfc_destroy(y) == BBFC_OK, "destroy");
    }

    /* 8. device-resident requests against the deterministic filter `a`: each
     * request starts on a 64-key boundary, so its answer words are the
     * oracle's words from there, the last one cut at its length */
    {
        bbfc_server_handle srv = NULL;
        bbfc_server_config scfg;
        CHECK(bbfc_server_default_config(&scfg) == BBFC_OK && scfg.n_slots >= 1 && scfg.max_batch_keys % 64 == 0,
              "server defaults");
        CHECK(bbfc_server_default_config(NULL) == BBFC_EINVAL, "null config accepted");
        scfg.n_slots = 2;
        scfg.max_batch_keys = 8192; /* the 30000- and 49000-key requests span several batches */
        CHECK(bbfc_server_create(a, &scfg, &srv) == BBFC_OK, "server_create: %s", bbfc_last_error());
        const uint64_t starts[4] = {0, 640, 6400, 50048}, lens[4] = {1, 4097, 30000, 49000};
        uint64_t *d_ans = NULL;
        HIP(hipMalloc((void **)&d_ans, 4 * 1024 * 8));
        uint64_t tickets[4];
        for (int i = 0; i < 4; i++)
            CHECK(bbfc_server_submit_device(srv, d_keys + starts[i], lens[i], d_ans + i * 1024, &tickets[i]) == BBFC_OK,
                  "submit_device: %s", bbfc_last_error());
        for (int i = 0; i < 4; i++)
            CHECK(bbfc_server_wait(srv, tickets[i], -1.0, NULL) == BBFC_OK, "wait: %s", bbfc_last_error());
        uint64_t *ans = malloc(4 * 1024 * 8);
        HIP(hipMemcpy(ans, d_ans, 4 * 1024 * 8, hipMemcpyDeviceToHost));
        for (int i = 0; i < 4; i++) {
            const uint64_t words = (lens[i] + 63) / 64;
            for (uint64_t w = 0; w < words; w++) {
                uint64_t want = want_bits[starts[i] / 64 + w];
                if (w == words - 1 && lens[i] % 64)
                    want &= (1ull << (lens[i] % 64)) - 1;
                CHECK(ans[i * 1024 + w] == want, "request %d word %llu differs from the oracle", i,
                      (unsigned long long)w);
            }
        }
        CHECK(bbfc_server_destroy(srv) == BBFC_OK, "server_destroy");
        HIP(hipFree(d_ans));
        free(ans);
    }

    CHECK(bbfc_destroy(a) == BBFC_OK, "destroy");
    CHECK(bbfc_destroy(b) == BBFC_OK, "destroy");
    HIP(hipFree(d_keys));
    HIP(hipFree(d_out));
    free(h_keys);
    free(got_words);
    free(want_words);
    free(got_bits);
    free(want_bits);
    if (failures) {
        printf("%d check(s) failed\n", failures);
        return 1;
    }
    printf("c abi check ok: M=%llu c=%u k=%u n=%llu; oracle hits %llu of %llu\n", (unsigned long long)M, c, k,
           (unsigned long long)n, (unsigned long long)hits, (unsigned long long)nq);
    return 0;
}
