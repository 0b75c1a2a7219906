// Query serving with continuous batching over one resident filter.
//
// Clients submit requests (host keys, host answer buffer) into one FIFO of
// admitted requests. The server has a fixed set of slots, each with its own
// stream, pinned and device staging of max_batch_keys keys, and its own
// worker thread. A worker whose slot is free takes the oldest pending work
// into one fused batch (each request's piece starts on a 64-key boundary, so
// its answer words can be copied out whole; a request larger than what is
// left of the slot continues in the next batch), copies the keys into its
// pinned staging, enqueues key upload, one query launch and answer download
// on the slot's stream, waits for the batch by polling its event, and hands
// the answer words back to their requests; a request is done when all its
// pieces are. Slots work in parallel, so host staging copies run on several
// cores at once and batches of different slots overlap on the device.
// Admission is by memory: at most max_pending_keys keys are queued (submit
// answers BBFC_EBUSY beyond that), and a batch never holds more than a
// slot's staging. One worker at a time gathers the next batch, and a
// submission wakes a worker only when one waits and none is gathering, so a
// stream of single submissions does not pay a wake-up each. With
// batch_window_us > 0, while other batches are on the device the gatherer
// waits up to that long from the oldest request's arrival for more requests
// (or half a batch): larger batches for submitters that cannot hand over
// their requests together, at the price of latency.
//
// Requests whose keys and answers are in device memory join the same queue.
// A batch holds requests of one kind: a device batch stages nothing; its
// pieces (at most kMaxDevicePieces) become a small descriptor table, copied
// to the device, and one query launch reads every piece's keys where they
// are and writes its answers straight into the request's buffer.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "bbfc_common.hpp"
#include "bbfc_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint32_t kMaxDevicePieces = bbfc::kMaxQueryPieces;

// slots, keys per batch, pending keys, poll interval (us), gathering window (us)
constexpr bbfc_server_config kDefaultConfig{4, 1u << 20, 1ull << 28, 20, 0};

struct Request {
    uint64_t ticket = 0;
    const uint64_t *keys = nullptr;
    uint64_t n = 0;
    uint64_t *out = nullptr;
    bool device = false;      // keys and answers in device memory
    uint64_t next = 0;        // first key not yet placed in a batch
    uint64_t answered = 0;    // keys whose answers are back
    Clock::time_point t_submit;
    Clock::time_point t_done;
    bool done = false;
};

struct Piece {
    std::shared_ptr<Request> req;
    uint64_t key_off; // first key of the piece within the request (multiple of 64)
    uint64_t n;
    uint64_t word_off; // first answer word of the piece in the slot's staging
};

struct Slot {
    hipStream_t stream = nullptr;
    uint64_t *h_keys = nullptr; // pinned
    uint64_t *h_out = nullptr;  // pinned
    uint64_t *d_keys = nullptr;
    uint64_t *d_out = nullptr;
    hipEvent_t done = nullptr;
    bbfc::QueryPiece *h_table = nullptr; // pinned: a device batch's pieces
    bbfc::QueryPiece *d_table = nullptr;
    bool device = false; // the planned batch is of device requests
    std::vector<Piece> pieces;
    std::thread worker;
};

} // namespace

struct bbfc_server {
    bbfc_handle filter = nullptr;
    bbfc_server_config cfg{};
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work; // workers: new requests or stop
    std::condition_variable cv_done; // waiters: a request finished
    std::deque<std::shared_ptr<Request>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> by_ticket;
    uint64_t next_ticket = 1;
    uint64_t pending_keys = 0;
    uint32_t idle = 0;       // workers waiting for work
    uint32_t in_flight = 0;  // batches on the device
    bool collecting = false; // a worker is gathering the next batch
    bool stop = false;
    hipError_t error = hipSuccess;
    // statistics
    uint64_t batches = 0;
    uint64_t batched_keys = 0;
    uint64_t completed = 0;
};

namespace {

// Takes the oldest pending work for a free slot (bookkeeping only). Called
// with the lock held; returns the number of staged keys (0: nothing to do).
uint64_t plan_slot(bbfc_server &s, Slot &slot)
{
    uint64_t used = 0;
    const uint64_t cap = s.cfg.max_batch_keys;
    slot.pieces.clear();
    slot.device = !s.pending.empty() && s.pending.front()->device;
    while (!s.pending.empty() && used < cap) {
        std::shared_ptr<Request> r = s.pending.front();
        if (r->device != slot.device || (slot.device && slot.pieces.size() >= kMaxDevicePieces))
            break; // one kind per batch; a device batch's table is bounded
        const uint64_t room = cap - used;
        const uint64_t left = r->n - r->next;
        uint64_t take = std::min(left, room);
        if (take < left)
            take -= take % 64; // a continued request resumes on a 64-key boundary
        if (take == 0)
            break;
        slot.pieces.push_back(Piece{r, r->next, take, used / 64});
        r->next += take;
        used += (take + 63) / 64 * 64;
        if (r->next == r->n) {
            s.pending.pop_front();
            s.pending_keys -= r->n;
        }
    }
    return used;
}

// Stages a planned slot's keys and enqueues upload, query and download.
// Runs without the lock: only the slot's worker touches the slot, and the
// clients keep their key buffers valid until their requests are done.
hipError_t launch_slot(bbfc_server &s, Slot &slot, uint64_t used)
{
    if (slot.device) {
        uint32_t i = 0;
        for (const Piece &p : slot.pieces)
            slot.h_table[i++] = bbfc::QueryPiece{p.req->keys + p.key_off, p.req->out + p.key_off / 64, p.n, 0};
        hipError_t e = bbfc::launch_query_pieces(*s.filter, slot.h_table, slot.d_table, i, slot.stream);
        return e == hipSuccess ? hipEventRecord(slot.done, slot.stream) : e;
    }
    for (const Piece &p : slot.pieces) {
        memcpy(slot.h_keys + p.word_off * 64, p.req->keys + p.key_off, p.n * sizeof(uint64_t));
        const uint64_t padded = (p.n + 63) / 64 * 64;
        if (padded > p.n)
            memset(slot.h_keys + p.word_off * 64 + p.n, 0, (padded - p.n) * sizeof(uint64_t));
    }
    hipError_t e = hipMemcpyAsync(slot.d_keys, slot.h_keys, used * sizeof(uint64_t), hipMemcpyHostToDevice,
                                  slot.stream);
    if (e == hipSuccess)
        e = bbfc::launch_query(*s.filter, slot.d_keys, used, slot.d_out, slot.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(slot.h_out, slot.d_out, used / 64 * sizeof(uint64_t), hipMemcpyDeviceToHost, slot.stream);
    if (e == hipSuccess)
        e = hipEventRecord(slot.done, slot.stream);
    return e;
}

// Copies a finished slot's answers into its requests' buffers (no lock); a
// device batch wrote them in place.
void copy_answers(Slot &slot)
{
    if (slot.device)
        return;
    for (const Piece &p : slot.pieces) {
        const uint64_t words = (p.n + 63) / 64;
        memcpy(p.req->out + p.key_off / 64, slot.h_out + p.word_off, words * sizeof(uint64_t));
        if (p.n % 64) // the request's last word: keep only its own answers
            p.req->out[p.key_off / 64 + words - 1] &= (1ull << (p.n % 64)) - 1;
    }
}

// Marks answered pieces and finished requests. Called with the lock held.
void finish_slot(bbfc_server &s, Slot &slot, Clock::time_point now)
{
    for (Piece &p : slot.pieces) {
        p.req->answered += p.n;
        if (p.req->answered == p.req->n) {
            p.req->done = true;
            p.req->t_done = now;
            s.completed++;
        }
    }
    slot.pieces.clear();
}

// Waits for a launched batch by polling its event: yielding between polls
// for the first kSpinUs (a batch of up to 2^20 keys is back within a few
// hundred microseconds, and a sleep would add its timer slack to the
// latency), then sleeping poll_us between polls (0: yielding throughout).
constexpr int kSpinUs = 1000;

hipError_t wait_slot(const bbfc_server &s, const Slot &slot)
{
    const Clock::time_point spin_until = Clock::now() + std::chrono::microseconds(kSpinUs);
    for (;;) {
        const hipError_t q = hipEventQuery(slot.done);
        if (q != hipErrorNotReady)
            return q;
        if (s.cfg.poll_us && Clock::now() >= spin_until)
            std::this_thread::sleep_for(std::chrono::microseconds(s.cfg.poll_us));
        else
            std::this_thread::yield();
    }
}

void slot_worker(bbfc_server *sp, Slot *slot_p)
{
    bbfc_server &s = *sp;
    Slot &slot = *slot_p;
    bbfc::DeviceGuard guard(s.filter->device);
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
        // one worker at a time gathers the next batch; the others wait
        ++s.idle;
        s.cv_work.wait(lk, [&] { return s.stop || (!s.pending.empty() && !s.collecting); });
        --s.idle;
        if (s.pending.empty())
            break; // stopping, and nothing left to serve
        s.collecting = true;
        // Batching window: while another batch is on the device, wait up to
        // batch_window_us after the oldest pending request's arrival for more
        // requests, unless half a batch is pending already. With the device
        // idle the batch goes at once.
        if (s.cfg.batch_window_us > 0 && s.in_flight > 0) {
            const Clock::time_point until =
                s.pending.front()->t_submit + std::chrono::microseconds(s.cfg.batch_window_us);
            while (!s.stop && s.pending_keys < s.cfg.max_batch_keys / 2 && Clock::now() < until) {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        }
        const uint64_t used = plan_slot(s, slot);
        s.collecting = false;
        if (!s.pending.empty() && s.idle > 0)
            s.cv_work.notify_one(); // more work than this slot holds: wake another worker
        if (used == 0)
            continue;
        s.batches++;
        s.batched_keys += used;
        s.in_flight++;
        lk.unlock();
        hipError_t e = launch_slot(s, slot, used);
        if (e == hipSuccess)
            e = wait_slot(s, slot);
        if (e == hipSuccess)
            copy_answers(slot);
        else
            (void)hipStreamSynchronize(slot.stream); // nothing of this batch may still read the staging
        const Clock::time_point now = Clock::now();
        lk.lock();
        s.in_flight--;
        if (e != hipSuccess && s.error == hipSuccess)
            s.error = e;
        finish_slot(s, slot, now);
        s.cv_done.notify_all();
    }
}

// Checks a request's arguments (no lock) and makes its record.
bbfc_status make_request(const uint64_t *keys, uint64_t n, uint64_t *out, Clock::time_point t_arrival, bool device,
                         std::shared_ptr<Request> &r)
{
    if (n > 0 && (keys == nullptr || out == nullptr))
        return bbfc::fail(BBFC_EINVAL, "null keys or output");
    if (device && n > 0) {
        const uintptr_t k0 = (uintptr_t)keys, k1 = k0 + n * 8;
        const uintptr_t o0 = (uintptr_t)out, o1 = o0 + ((n + 63) / 64) * 8;
        if (k0 < o1 && o0 < k1)
            return bbfc::fail(BBFC_EINVAL, "output overlaps the keys");
    }
    r = std::make_shared<Request>();
    r->keys = keys;
    r->n = n;
    r->out = out;
    r->device = device;
    r->t_submit = t_arrival;
    return BBFC_OK;
}

// Admits reqs[0 .. count) in order under one lock acquisition, as far as
// admission allows (the first one always fits when nothing is pending);
// tickets[i] receives each admitted request's ticket. *admitted receives how
// many were; BBFC_EBUSY when admission stopped short.
bbfc_status admit(bbfc_server_handle s, const std::shared_ptr<Request> *reqs, size_t count, uint64_t *tickets,
                  size_t *admitted)
{
    size_t i = 0;
    bool wake = false;
    bbfc_status st = BBFC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop)
            return bbfc::fail(BBFC_EINVAL, "server is stopping");
        if (s->error != hipSuccess)
            return bbfc::hip_fail(s->error, "server failed earlier");
        for (; i < count; ++i) {
            const std::shared_ptr<Request> &r = reqs[i];
            if (r->n > 0 && s->pending_keys + r->n > s->cfg.max_pending_keys && !s->pending.empty()) {
                st = bbfc::fail(BBFC_EBUSY, "admission: %llu keys already pending",
                                (unsigned long long)s->pending_keys);
                break;
            }
            r->ticket = s->next_ticket++;
            s->by_ticket[r->ticket] = r;
            if (r->n == 0) {
                r->done = true;
                r->t_done = r->t_submit;
                s->completed++;
            } else {
                s->pending.push_back(r);
                s->pending_keys += r->n;
                // wake a worker only if one is waiting and none is gathering
                // a batch already (that one sees the new requests under the lock)
                wake = wake || (s->idle > 0 && !s->collecting);
            }
            tickets[i] = r->ticket;
        }
    }
    if (wake)
        s->cv_work.notify_one();
    *admitted = i;
    return st;
}

bbfc_status submit_at(bbfc_server_handle s, const uint64_t *h_keys, uint64_t n, uint64_t *h_out_bits,
                      uint64_t *ticket, Clock::time_point t_arrival, bool device)
{
    if (s == nullptr || ticket == nullptr)
        return bbfc::fail(BBFC_EINVAL, "null server or ticket");
    std::shared_ptr<Request> r;
    const bbfc_status st = make_request(h_keys, n, h_out_bits, t_arrival, device, r);
    if (st != BBFC_OK)
        return st;
    size_t admitted = 0;
    return admit(s, &r, 1, ticket, &admitted);
}

} // namespace

using bbfc::fail;
using bbfc::hip_fail;

extern "C" {

bbfc_status bbfc_server_default_config(bbfc_server_config *config)
{
    if (config == nullptr)
        return fail(BBFC_EINVAL, "null config");
    *config = kDefaultConfig;
    return BBFC_OK;
}

bbfc_status bbfc_server_create(bbfc_handle filter, const bbfc_server_config *config, bbfc_server_handle *out)
{
    if (filter == nullptr || out == nullptr)
        return fail(BBFC_EINVAL, "null filter or output handle");
    bbfc_server_config cfg = config ? *config : kDefaultConfig;
    if (cfg.n_slots < 1 || cfg.n_slots > 16)
        return fail(BBFC_EINVAL, "n_slots must be in [1, 16]");
    if (cfg.max_batch_keys < 64 || cfg.max_batch_keys % 64 || cfg.max_batch_keys > (1ull << 30))
        return fail(BBFC_EINVAL, "max_batch_keys must be a multiple of 64 in [64, 2^30]");
    if (cfg.max_pending_keys < 1)
        return fail(BBFC_EINVAL, "max_pending_keys must be >= 1");
    if (cfg.poll_us > 100000)
        return fail(BBFC_EINVAL, "poll_us must be <= 100000");
    if (cfg.batch_window_us > 100000)
        return fail(BBFC_EINVAL, "batch_window_us must be <= 100000");
    auto *s = new bbfc_server();
    s->filter = filter;
    s->cfg = cfg;
    s->slots.resize(cfg.n_slots);
    bbfc::DeviceGuard guard(filter->device);
    hipError_t e = hipSuccess;
    for (Slot &slot : s->slots) {
        const size_t kb = cfg.max_batch_keys * sizeof(uint64_t);
        const size_t ob = cfg.max_batch_keys / 64 * sizeof(uint64_t);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&slot.h_keys, kb, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&slot.h_out, ob, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc(&slot.d_keys, kb);
        if (e == hipSuccess)
            e = hipMalloc(&slot.d_out, ob);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&slot.h_table, kMaxDevicePieces * sizeof(bbfc::QueryPiece),
                              hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc((void **)&slot.d_table, kMaxDevicePieces * sizeof(bbfc::QueryPiece));
    }
    if (e != hipSuccess) {
        bbfc_server_destroy(s);
        return hip_fail(e, "allocating server slots");
    }
    for (Slot &slot : s->slots)
        slot.worker = std::thread(slot_worker, s, &slot);
    *out = s;
    return BBFC_OK;
}

bbfc_status bbfc_server_destroy(bbfc_server_handle s)
{
    if (s == nullptr)
        return fail(BBFC_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (Slot &slot : s->slots)
        if (slot.worker.joinable())
            slot.worker.join();
    bbfc::DeviceGuard guard(s->filter->device);
    for (Slot &slot : s->slots) {
        if (slot.stream)
            (void)hipStreamSynchronize(slot.stream);
        if (slot.done)
            (void)hipEventDestroy(slot.done);
        if (slot.d_keys)
            (void)hipFree(slot.d_keys);
        if (slot.d_out)
            (void)hipFree(slot.d_out);
        if (slot.h_keys)
            (void)hipHostFree(slot.h_keys);
        if (slot.h_out)
            (void)hipHostFree(slot.h_out);
        if (slot.d_table)
            (void)hipFree(slot.d_table);
        if (slot.h_table)
            (void)hipHostFree(slot.h_table);
        if (slot.stream)
            (void)hipStreamDestroy(slot.stream);
    }
    delete s;
    return BBFC_OK;
}

bbfc_status bbfc_server_submit(bbfc_server_handle s, const uint64_t *h_keys, uint64_t n, uint64_t *h_out_bits,
                               uint64_t *ticket)
{
    return submit_at(s, h_keys, n, h_out_bits, ticket, Clock::now(), false);
}

bbfc_status bbfc_server_submit_device(bbfc_server_handle s, const uint64_t *d_keys, uint64_t n,
                                      uint64_t *d_out_bits, uint64_t *ticket)
{
    return submit_at(s, d_keys, n, d_out_bits, ticket, Clock::now(), true);
}

bbfc_status bbfc_server_wait(bbfc_server_handle s, uint64_t ticket, double timeout_s, double *latency_us)
{
    if (s == nullptr)
        return fail(BBFC_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end())
        return fail(BBFC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Request> r = it->second;
    const auto pred = [&] { return r->done || s->error != hipSuccess; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        return fail(BBFC_EBUSY, "request %llu not done yet", (unsigned long long)ticket);
    }
    if (!r->done)
        return hip_fail(s->error, "serving");
    if (latency_us)
        *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    s->by_ticket.erase(it);
    return s->error == hipSuccess ? BBFC_OK : hip_fail(s->error, "serving");
}

bbfc_status bbfc_server_stats(bbfc_server_handle s, uint64_t *batches, uint64_t *batched_keys, uint64_t *completed)
{
    if (s == nullptr)
        return fail(BBFC_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (batches)
        *batches = s->batches;
    if (batched_keys)
        *batched_keys = s->batched_keys;
    if (completed)
        *completed = s->completed;
    return BBFC_OK;
}

} // extern "C"

namespace {

bbfc_status replay(bbfc_server_handle s, const uint64_t *h_keys, const uint64_t *req_offsets, uint32_t n_requests,
                   const double *arrival_s, uint64_t *h_out_bits, const uint64_t *out_offsets, double *latency_us,
                   double *wall_s, bool device)
{
    if (s == nullptr || h_keys == nullptr || req_offsets == nullptr || arrival_s == nullptr ||
        h_out_bits == nullptr || out_offsets == nullptr || latency_us == nullptr)
        return fail(BBFC_EINVAL, "null argument");
    for (uint32_t i = 0; i + 1 < n_requests; ++i)
        if (arrival_s[i + 1] < arrival_s[i])
            return fail(BBFC_EINVAL, "arrival times must be non-decreasing");
    std::vector<std::shared_ptr<Request>> reqs(n_requests);
    std::vector<uint64_t> tickets(n_requests, 0);
    const Clock::time_point t0 = Clock::now();
    auto due_at = [&](uint32_t i) {
        return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
    };
    uint32_t next = 0; // first request not admitted yet
    while (next < n_requests) {
        const Clock::time_point due = due_at(next);
        while (Clock::now() < due) {
        }
        // every request whose arrival has passed is admitted together, with
        // one lock acquisition: a submitter behind its schedule catches up
        // instead of falling further behind
        const Clock::time_point now = Clock::now();
        uint32_t end = next + 1;
        while (end < n_requests && due_at(end) <= now)
            ++end;
        for (uint32_t i = next; i < end; ++i) {
            if (!reqs[i]) {
                // latency counts from the scheduled arrival, also while admission waits
                const bbfc_status st = make_request(h_keys + req_offsets[i], req_offsets[i + 1] - req_offsets[i],
                                                    h_out_bits + out_offsets[i], due_at(i), device, reqs[i]);
                if (st != BBFC_OK)
                    return st;
            }
        }
        size_t admitted = 0;
        const bbfc_status st = admit(s, reqs.data() + next, end - next, tickets.data() + next, &admitted);
        next += (uint32_t)admitted;
        if (st == BBFC_EBUSY)
            std::this_thread::sleep_for(std::chrono::microseconds(10)); // admission: retry when memory frees
        else if (st != BBFC_OK)
            return st;
    }
    for (uint32_t i = 0; i < n_requests; ++i) {
        const bbfc_status st = bbfc_server_wait(s, tickets[i], -1.0, &latency_us[i]);
        if (st != BBFC_OK)
            return st;
    }
    if (wall_s)
        *wall_s = std::chrono::duration<double>(Clock::now() - t0).count();
    return BBFC_OK;
}

} // namespace

extern "C" {

bbfc_status bbfc_server_replay(bbfc_server_handle s, const uint64_t *h_keys, const uint64_t *req_offsets,
                               uint32_t n_requests, const double *arrival_s, uint64_t *h_out_bits,
                               const uint64_t *out_offsets, double *latency_us, double *wall_s)
{
    return replay(s, h_keys, req_offsets, n_requests, arrival_s, h_out_bits, out_offsets, latency_us, wall_s, false);
}

bbfc_status bbfc_server_replay_device(bbfc_server_handle s, const uint64_t *d_keys, const uint64_t *req_offsets,
                                      uint32_t n_requests, const double *arrival_s, uint64_t *d_out_bits,
                                      const uint64_t *out_offsets, double *latency_us, double *wall_s)
{
    return replay(s, d_keys, req_offsets, n_requests, arrival_s, d_out_bits, out_offsets, latency_us, wall_s, true);
}

} // extern "C"
