// Library-internal state and kernel launchers (not part of the ABI).
#pragma once

#include <stdint.h>

#include <vector>

#include "bbfc_common.hpp"

struct bbfc_filter {
    uint64_t M = 0;
    uint32_t c = 0;
    uint32_t k = 0;
    int32_t cost_kind = BBFC_COST_NONE;
    double cost_param = 0.0;
    uint64_t block_mult[BBFC_MAX_CHOICES] = {};
    uint64_t bit_mult[BBFC_MAX_BITS_PER_KEY] = {};
    int32_t bit_selection = BBFC_BITS_RANDOM;
    uint64_t T = 1;               // sub-arrays (Section 3.4, Parallelization)
    uint64_t S = 0;               // blocks per sub-array, M / T
    uint64_t sub_mult = 0;        // multiplier of h_0 (T > 1)
    bbfc::HashMod blk{};          // modulus S
    bbfc::HashMod sub{};          // modulus T
    uint64_t *d_words = nullptr;  // 8*M words
    uint16_t *d_rank = nullptr;   // (k+1)*513 ranks, null for one choice
    std::vector<uint16_t> h_rank;
    int device = 0;
    int num_cus = 0;
    uint64_t max_inflight = 0;    // 0: n_blocks/(8(c-1)), no bound for c = 1
    int query_early_exit = 1;     // load choice i+1 only for keys still unanswered
    int insert_tile = 0;          // racing insert kernel: 0 by keys in flight, 1 tiles of 64 keys, 2 of 8 keys
    // launch shape per operation, [BBFC_OP_INSERT] and [BBFC_OP_QUERY]
    bbfc_launch_shape shape[2] = {{8, 1, 0, 0, 0.0f}, {8, 1, 0, 0, 0.0f}};
    size_t max_lds = 65536;       // LDS bytes a workgroup may use on this device
    // scratch of the sequential insert on large inputs, allocated on first use
    uint64_t *d_ord_claims = nullptr; // claim table
    uint8_t *d_ord_pend = nullptr;    // pending flags of a window
    uint64_t *d_ord_tail = nullptr;   // a window's remaining keys, their count, the count the last step saw
    uint64_t ord_tag = 0;             // last step tag used on this filter
};

namespace bbfc {

// Records a message for bbfc_last_error() and returns s.
bbfc_status fail(bbfc_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
bbfc_status hip_fail(hipError_t e, const char *what);
const char *last_error();

// Makes a device current for the scope of a call.
class DeviceGuard {
  public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;

  private:
    int prev_ = -1;
    bool switched_ = false;
};

KParams make_kparams(const bbfc_filter &f);

// Dynamic LDS of the insert kernels: the cost rank table (none for c = 1).
size_t rank_lds_bytes(uint32_t c, uint32_t k);

// Keys in flight for a racing insert on this filter.
uint64_t insert_inflight(const bbfc_filter &f);
// Keys per wavefront tile of the racing insert the filter launches (64 or 8).
uint32_t insert_tile_keys(const bbfc_filter &f);
// What a racing insert of n keys launches: keys per tile, tiles per
// wavefront, working wavefronts and workgroups (nothing is launched).
struct InsertGeom {
    uint32_t tile_keys;
    uint32_t tiles_per_wave;
    uint64_t waves;
    uint64_t workgroups;
};
hipError_t insert_geometry(const bbfc_filter &f, uint64_t n, InsertGeom *geom);

hipError_t launch_insert(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s);
// The racing insert that also writes each key's decision (bbfc_insert_recorded).
hipError_t launch_insert_recorded(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint8_t *decisions,
                                  hipStream_t s);
hipError_t launch_insert_det(bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s);
// The same insert with its scratch in a static device array (no allocation).
hipError_t launch_insert_det_noalloc(const bbfc_filter &f, const uint64_t *keys, uint64_t n, hipStream_t s);
hipError_t launch_query(const bbfc_filter &f, const uint64_t *keys, uint64_t n, uint64_t *out,
                        hipStream_t s);
hipError_t launch_fill_zero(uint64_t *p, uint64_t n_words, hipStream_t s);

// One piece of a query over several key arrays of one filter: keys[0..n)
// answered into out (bbfc_query's layout). unit_off is filled by the
// launcher: the piece's first unit of T 64-key tiles in the launch.
struct QueryPiece {
    const uint64_t *keys;
    uint64_t *out;
    uint64_t n;
    uint64_t unit_off;
};
constexpr uint32_t kMaxQueryPieces = 1024; // pieces per launch

// Enqueues one query launch over h_pieces[0..n_pieces) (n_pieces <=
// kMaxQueryPieces; pinned host memory,
// keys/out/n filled by the caller; unit offsets are written here), whose
// table is copied to d_pieces on the stream first. The host table must stay
// untouched until the stream has passed the copy.
hipError_t launch_query_pieces(const bbfc_filter &f, QueryPiece *h_pieces, QueryPiece *d_pieces, uint32_t n_pieces,
                               hipStream_t s);
hipError_t launch_load_histogram(const bbfc_filter &f, uint64_t *hist, hipStream_t s);

// Bulk insert through a stable partition by sub-array (bbfc_bulk.hip).
// n < 2^32 keys per launch; the workspace holds bulk_workspace_bytes(f, n).
bool bulk_supported(const bbfc_filter &f);
uint64_t bulk_workspace_bytes(const bbfc_filter &f, uint64_t n);
hipError_t launch_bulk_insert(const bbfc_filter &f, const uint64_t *keys, uint64_t n, void *workspace,
                              hipStream_t s);

// Canonical q-grams of a 2-bit packed sequence cut into segments (see
// bbfc_kmer_keys): fused insert and query, and the keys written out.
hipError_t launch_insert_kmers(const bbfc_filter &f, const uint64_t *seq, uint64_t n_segments, uint64_t seg_len, uint32_t q, hipStream_t s);
hipError_t launch_query_kmers(const bbfc_filter &f, const uint64_t *seq, uint64_t n_segments, uint64_t seg_len, uint32_t q, uint64_t *out, hipStream_t s);
hipError_t launch_kmer_keys(const uint64_t *seq, uint64_t n_segments, uint64_t seg_len, uint32_t q, uint64_t *out,
                            hipStream_t s);

hipError_t launch_probe_gather(const uint64_t *buf, uint64_t n_lines64, uint32_t access_bytes, uint64_t n_access,
                               uint64_t seed, uint64_t *sink, hipStream_t s);
hipError_t launch_probe_atomic64(uint64_t *buf, uint64_t n_lines, uint64_t n_access, uint64_t seed,
                                 hipStream_t s);
hipError_t launch_probe_insert_pattern(uint64_t *buf, uint64_t n_lines, uint64_t n_keys, int mask_bits, uint64_t seed,
                                       uint64_t *sink, hipStream_t s);
hipError_t launch_probe_insert_schedule(uint64_t *buf, uint64_t n_lines, uint64_t n_keys, int mask_bits,
                                        int schedule, uint64_t seed, uint64_t *sink, hipStream_t s);
hipError_t launch_probe_latency(uint64_t *buf, uint64_t n_lines, int kind, uint32_t iters, uint32_t waves,
                                double *out, hipStream_t s);
hipError_t launch_probe_copy(const uint64_t *src, uint64_t *dst, uint64_t n_words, uint32_t request_bytes,
                             hipStream_t s);

} // namespace bbfc
