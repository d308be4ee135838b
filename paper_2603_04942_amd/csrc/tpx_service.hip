// Continuous batching over one tpx_stream: chunks are admitted into a device
// ring buffer as they arrive (tpx_service_submit) and every run processes all
// whole chunks admitted so far, up to a batch limit, as one call of the
// stream path (tpx_service_run).  The stream path gives the same hits for any
// split of the stream into chunks, so batching changes when results appear,
// never what they are.
//
// Admission overlaps processing: a submit may come from another host thread
// while a run is on the GPU.  It reserves free ring space under a lock (the
// words of the batch in flight stay reserved until its run returns), copies
// the chunk on the service's own stream and records an event; a run makes its
// stream wait for the events of the chunks it takes, on the device.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "tpx_kernels.h"

namespace {

struct Chunk {
    uint64_t end;        // ring position after the chunk
    hipEvent_t ready;    // recorded after its copy
    bool issued;         // copy enqueued and event recorded
};

}  // namespace

struct tpx_service {
    tpx_stream* st = nullptr;
    uint64_t* ring = nullptr;     // device u64[ring_cap]
    uint64_t* stage = nullptr;    // device u64[max_batch]: a batch that wraps the ring
    uint64_t ring_cap = 0, max_batch = 0;
    hipStream_t copy = nullptr;   // admission copies
    hipEvent_t prod = nullptr;    // orders a device chunk's copy after the caller's stream
    std::mutex mu;                // guards everything below
    uint64_t wpos = 0, rpos = 0;  // words reserved / processed since creation
    uint64_t n_sub = 0, n_done = 0;
    std::deque<Chunk> q;          // admitted, unprocessed chunks in order
    std::vector<hipEvent_t> spare;
};

namespace {

void free_service(tpx_service* sv) {
    if (sv->copy) (void)hipStreamSynchronize(sv->copy);
    if (sv->st) tpx_stream_destroy(sv->st);
    if (sv->ring) (void)hipFree(sv->ring);
    if (sv->stage) (void)hipFree(sv->stage);
    for (auto& c : sv->q) (void)hipEventDestroy(c.ready);
    for (auto e : sv->spare) (void)hipEventDestroy(e);
    if (sv->prod) (void)hipEventDestroy(sv->prod);
    if (sv->copy) (void)hipStreamDestroy(sv->copy);
    delete sv;
}

// copy n words into the ring at logical position pos (two pieces when it wraps)
tpx_status ring_copy(tpx_service* sv, uint64_t pos, const uint64_t* src, uint64_t n,
                     hipMemcpyKind kind, hipStream_t hs) {
    const uint64_t at = pos % sv->ring_cap;
    const uint64_t first = n < sv->ring_cap - at ? n : sv->ring_cap - at;
    if (first && hipMemcpyAsync(sv->ring + at, src, first * 8, kind, hs) != hipSuccess)
        return TPX_EHIP;
    if (n > first && hipMemcpyAsync(sv->ring, src + first, (n - first) * 8, kind, hs) != hipSuccess)
        return TPX_EHIP;
    return TPX_OK;
}

}  // namespace

extern "C" {

tpx_status tpx_service_create(const tpx_params* p_h, size_t max_batch_pkts, size_t ring_pkts,
                              tpx_service** out_h) {
    if (!out_h || !p_h) return tpx::report(TPX_EINVAL, "NULL argument");
    if (max_batch_pkts == 0 || ring_pkts < max_batch_pkts)
        return tpx::report(TPX_EINVAL, "need 0 < max_batch_pkts <= ring_pkts");
    tpx_service* sv = new tpx_service();
    tpx_status rc = tpx_stream_create(p_h, max_batch_pkts, &sv->st);
    if (rc != TPX_OK) {
        sv->st = nullptr;
        free_service(sv);
        return rc;
    }
    sv->ring_cap = ring_pkts;
    sv->max_batch = max_batch_pkts;
    if (hipMalloc((void**)&sv->ring, ring_pkts * 8) != hipSuccess ||
        hipMalloc((void**)&sv->stage, max_batch_pkts * 8) != hipSuccess) {
        (void)hipGetLastError();
        free_service(sv);
        return tpx::report(TPX_ENOMEM, "ring allocation failed");
    }
    if (hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        sv->copy = nullptr;
        free_service(sv);
        return tpx::report(TPX_EHIP, "copy stream creation failed");
    }
    if (hipEventCreateWithFlags(&sv->prod, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        sv->prod = nullptr;
        free_service(sv);
        return tpx::report(TPX_EHIP, "event creation failed");
    }
    *out_h = sv;
    return TPX_OK;
}

tpx_status tpx_service_submit(tpx_service* sv, const uint64_t* chunk, size_t n_pkts,
                              int chunk_on_device, uint64_t* seq_h, void* stream) {
    if (!sv || (n_pkts && !chunk)) return tpx::report(TPX_EINVAL, "NULL argument");
    if (n_pkts > sv->max_batch) return tpx::report(TPX_EINVAL, "chunk larger than the batch limit");
    uint64_t pos, seq;
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->wpos + n_pkts - sv->rpos > sv->ring_cap)
            return tpx::report(TPX_ECAPACITY, "ring full: run the service first");
        if (!sv->spare.empty()) {
            ev = sv->spare.back();
            sv->spare.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            return tpx::report(TPX_EHIP, "event creation failed");
        }
        pos = sv->wpos;
        seq = sv->n_sub;
        sv->wpos += n_pkts;
        sv->n_sub++;
        sv->q.push_back(Chunk{sv->wpos, ev, false});
    }
    // a device chunk may still be written by work on the caller's stream
    tpx_status rc = TPX_OK;
    if (chunk_on_device && (hipEventRecord(sv->prod, (hipStream_t)stream) != hipSuccess ||
                            hipStreamWaitEvent(sv->copy, sv->prod, 0) != hipSuccess))
        rc = TPX_EHIP;
    if (rc == TPX_OK)
        rc = ring_copy(sv, pos, chunk, n_pkts,
                       chunk_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, sv->copy);
    if (rc == TPX_OK && hipEventRecord(ev, sv->copy) != hipSuccess) rc = TPX_EHIP;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto& c : sv->q)
            if (c.ready == ev) c.issued = true;
    }
    if (rc != TPX_OK) {
        // the reservation stays (later chunks are already behind it); the
        // stream's data for this chunk is unspecified from here on
        (void)hipGetLastError();
        return tpx::report(rc, "chunk copy into the ring failed");
    }
    if (seq_h) *seq_h = seq;
    return TPX_OK;
}

tpx_status tpx_service_run(tpx_service* sv, int flush, tpx_hit* hits, size_t hit_cap,
                           size_t* n_hits_h, uint64_t* n_done_h, tpx_stats* stats_h,
                           void* stream) {
    if (!sv || !n_hits_h || !n_done_h) return tpx::report(TPX_EINVAL, "NULL argument");
    hipStream_t hs = (hipStream_t)stream;
    // whole chunks from the front whose copies are enqueued, up to the limit
    uint64_t start, end;
    size_t take = 0;
    bool last;
    std::vector<hipEvent_t> evs;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        start = end = sv->rpos;
        while (take < sv->q.size() && sv->q[take].issued &&
               sv->q[take].end - sv->rpos <= sv->max_batch) {
            end = sv->q[take].end;
            evs.push_back(sv->q[take].ready);
            ++take;
        }
        last = take == sv->q.size();
    }
    if (take == 0 && !(flush && last)) {
        // nothing ready and no end of stream: a call on no words closes nothing
        *n_hits_h = 0;
        if (stats_h) *stats_h = tpx_stats{};
        std::lock_guard<std::mutex> lk(sv->mu);
        *n_done_h = sv->n_done;
        return TPX_OK;
    }
    for (hipEvent_t e : evs)
        if (hipStreamWaitEvent(hs, e, 0) != hipSuccess) return tpx::report(TPX_EHIP, "wait failed");
    const uint64_t n = end - start;
    const uint64_t* src = sv->ring + start % sv->ring_cap;
    if (n && start % sv->ring_cap + n > sv->ring_cap) {
        const uint64_t first = sv->ring_cap - start % sv->ring_cap;
        if (hipMemcpyAsync(sv->stage, src, first * 8, hipMemcpyDeviceToDevice, hs) != hipSuccess ||
            hipMemcpyAsync(sv->stage + first, sv->ring, (n - first) * 8, hipMemcpyDeviceToDevice,
                           hs) != hipSuccess)
            return tpx::report(TPX_EHIP, "staging copy failed");
        src = sv->stage;
    }
    // end of stream only once every admitted chunk is in this batch
    const tpx_status rc = tpx_process_stream(sv->st, src, n, flush && last, hits, hit_cap, n_hits_h,
                                             stats_h, stream);
    if (rc != TPX_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->rpos = end;
        for (size_t i = 0; i < take; ++i) {
            sv->spare.push_back(sv->q.front().ready);
            sv->q.pop_front();
        }
        sv->n_done += take;
        *n_done_h = sv->n_done;
    }
    return TPX_OK;
}

void tpx_service_destroy(tpx_service* sv) {
    if (sv) free_service(sv);
}

tpx_status tpx_service_set_segment(tpx_service* sv, uint32_t q) {
    if (!sv) return tpx::report(TPX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    return tpx_stream_set_segment(sv->st, q);
}

size_t tpx_service_device_bytes(const tpx_service* sv) {
    return sv ? tpx_stream_device_bytes(sv->st) + (sv->ring_cap + sv->max_batch) * 8 : 0;
}

// Paced replay with a native producer: a producer thread submits chunk k of
// the device-resident stream when its last word would have been acquired
// (release time t0 + end_k / rate) while the calling thread runs the service
// whenever chunks are admitted; the latency of a chunk is the completion of
// the run that processed it minus its release.
tpx_status tpx_service_replay(tpx_service* sv, const uint64_t* pk, size_t n, size_t chunk,
                              double pkts_per_s, tpx_hit* hits, size_t hit_cap, float* lat_ms_h,
                              size_t lat_cap, size_t* n_chunks_h, uint64_t* n_runs_h,
                              void* stream) {
    if (!sv || (n && !pk) || !n_chunks_h || !n_runs_h || chunk == 0 || !(pkts_per_s > 0))
        return tpx::report(TPX_EINVAL, "NULL argument, zero chunk or rate");
    if (chunk > sv->max_batch) return tpx::report(TPX_EINVAL, "chunk larger than the batch limit");
    const size_t n_chunks = (n + chunk - 1) / chunk;
    *n_chunks_h = n_chunks;
    if (lat_ms_h && lat_cap < n_chunks) return tpx::report(TPX_EINVAL, "lat_cap too small");
    using clk = std::chrono::steady_clock;
    std::vector<clk::time_point> rel(n_chunks);
    std::mutex mu;                // guards rel, issued, prod_rc
    std::condition_variable cv;   // the producer admitted a chunk or failed
    uint64_t issued = 0;          // chunks submitted (copies enqueued), in order
    tpx_status prod_rc = TPX_OK;
    uint64_t seq0 = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        seq0 = sv->n_sub;
        if (sv->n_sub != sv->n_done) return tpx::report(TPX_EINVAL, "service has unprocessed chunks");
    }
    const clk::time_point t0 = clk::now();
    std::thread producer([&]() {
        for (size_t k = 0; k < n_chunks; ++k) {
            const size_t a = k * chunk, m = std::min(chunk, n - a);
            const clk::time_point due =
                t0 + std::chrono::duration_cast<clk::duration>(
                         std::chrono::duration<double>((double)(a + m) / pkts_per_s));
            while (clk::now() < due) {
                if (due - clk::now() > std::chrono::microseconds(200))
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
            tpx_status rc;
            clk::time_point r;
            for (;;) {  // a full ring waits for the consumer
                r = clk::now();
                rc = tpx_service_submit(sv, pk + a, m, 1, nullptr, nullptr);
                if (rc != TPX_ECAPACITY) break;
                std::this_thread::yield();
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                rel[k] = due < r ? due : r;
                if (rc != TPX_OK) prod_rc = rc;
                else issued = k + 1;
            }
            cv.notify_one();
            if (rc != TPX_OK) return;
        }
    });
    tpx_status rc = TPX_OK;
    uint64_t runs = 0, done = 0;
    while (rc == TPX_OK && done < n_chunks) {
        uint64_t admitted;  // chunks whose copies are enqueued
        {
            // sleep until the producer admits a chunk not yet processed
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return issued > done || prod_rc != TPX_OK; });
            if (prod_rc != TPX_OK) break;
            admitted = issued;
        }
        size_t nh = 0;
        uint64_t n_done = 0;
        rc = tpx_service_run(sv, admitted == n_chunks ? 1 : 0, hits, hit_cap, &nh, &n_done,
                             nullptr, stream);
        const clk::time_point now = clk::now();
        if (rc != TPX_OK) break;
        ++runs;
        const uint64_t upto = n_done - seq0;
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t k = done; k < upto && k < n_chunks; ++k)
            if (lat_ms_h)
                lat_ms_h[k] = (float)std::chrono::duration<double, std::milli>(now - rel[k]).count();
        done = upto;
    }
    producer.join();
    *n_runs_h = runs;
    if (rc != TPX_OK) return rc;
    if (prod_rc != TPX_OK) return prod_rc;
    return TPX_OK;
}

}  // extern "C"

// ====================================================================== server
// Several independent request streams served at once.  Each open slot is a
// tpx_service (its own stream state, ring and staging) admitted only while
// its device memory fits the server's free HBM budget; slot k's runs go to
// HIP stream k mod n_streams, so runs of different slots issued from
// different host threads overlap on the GPU.  A slot's hits are those it gives
// alone: slots share no state.
struct tpx_server {
    tpx_params p;
    size_t budget = 0, used = 0;
    std::vector<hipStream_t> hs;
    struct Slot {
        tpx_service* sv = nullptr;
        size_t bytes = 0;
    };
    std::mutex mu;
    std::vector<Slot> slots;
};

namespace {
tpx_service* server_slot(tpx_server* sr, uint32_t slot) {
    std::lock_guard<std::mutex> lk(sr->mu);
    return slot < sr->slots.size() ? sr->slots[slot].sv : nullptr;
}
}  // namespace

extern "C" {

tpx_status tpx_server_create(const tpx_params* p_h, size_t hbm_budget_bytes, int n_streams,
                             tpx_server** out_h) {
    if (!p_h || !out_h) return tpx::report(TPX_EINVAL, "NULL argument");
    if (n_streams < 1 || n_streams > 64) return tpx::report(TPX_EINVAL, "n_streams outside 1..64");
    tpx_server* sr = new tpx_server();
    sr->p = *p_h;
    sr->budget = hbm_budget_bytes;
    for (int i = 0; i < n_streams; ++i) {
        hipStream_t h = nullptr;
        if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (auto x : sr->hs) (void)hipStreamDestroy(x);
            delete sr;
            return tpx::report(TPX_EHIP, "stream creation failed");
        }
        sr->hs.push_back(h);
    }
    *out_h = sr;
    return TPX_OK;
}

tpx_status tpx_server_open(tpx_server* sr, const tpx_params* p_h, size_t max_batch_pkts,
                           size_t ring_pkts, uint32_t* slot_h, size_t* bytes_h) {
    if (!sr || !slot_h) return tpx::report(TPX_EINVAL, "NULL argument");
    tpx_service* sv = nullptr;
    tpx_status rc = tpx_service_create(p_h ? p_h : &sr->p, max_batch_pkts, ring_pkts, &sv);
    if (rc != TPX_OK) return rc;
    const size_t bytes = tpx_service_device_bytes(sv);
    if (bytes_h) *bytes_h = bytes;
    std::lock_guard<std::mutex> lk(sr->mu);
    if (sr->used + bytes > sr->budget) {
        tpx_service_destroy(sv);
        return tpx::report(TPX_ECAPACITY, "the slot needs more device memory than the budget has free");
    }
    uint32_t slot = 0;
    while (slot < sr->slots.size() && sr->slots[slot].sv) ++slot;
    if (slot == sr->slots.size()) sr->slots.push_back({});
    sr->slots[slot].sv = sv;
    sr->slots[slot].bytes = bytes;
    sr->used += bytes;
    *slot_h = slot;
    return TPX_OK;
}

tpx_status tpx_server_submit(tpx_server* sr, uint32_t slot, const uint64_t* chunk, size_t n_pkts,
                             int chunk_on_device, uint64_t* seq_h, void* stream) {
    if (!sr) return tpx::report(TPX_EINVAL, "NULL argument");
    tpx_service* sv = server_slot(sr, slot);
    if (!sv) return tpx::report(TPX_EINVAL, "no open slot with that number");
    return tpx_service_submit(sv, chunk, n_pkts, chunk_on_device, seq_h, stream);
}

tpx_status tpx_server_run(tpx_server* sr, uint32_t slot, int flush, tpx_hit* hits,
                          size_t hit_cap, size_t* n_hits_h, uint64_t* n_done_h,
                          tpx_stats* stats_h) {
    if (!sr) return tpx::report(TPX_EINVAL, "NULL argument");
    tpx_service* sv = server_slot(sr, slot);
    if (!sv) return tpx::report(TPX_EINVAL, "no open slot with that number");
    return tpx_service_run(sv, flush, hits, hit_cap, n_hits_h, n_done_h, stats_h,
                           sr->hs[slot % sr->hs.size()]);
}

tpx_status tpx_server_close(tpx_server* sr, uint32_t slot) {
    if (!sr) return tpx::report(TPX_EINVAL, "NULL argument");
    tpx_service* sv = nullptr;
    {
        std::lock_guard<std::mutex> lk(sr->mu);
        if (slot >= sr->slots.size() || !sr->slots[slot].sv)
            return tpx::report(TPX_EINVAL, "no open slot with that number");
        sv = sr->slots[slot].sv;
        sr->used -= sr->slots[slot].bytes;
        sr->slots[slot] = {};
    }
    (void)hipStreamSynchronize(sr->hs[slot % sr->hs.size()]);
    tpx_service_destroy(sv);
    return TPX_OK;
}

size_t tpx_server_free_bytes(tpx_server* sr) {
    if (!sr) return 0;
    std::lock_guard<std::mutex> lk(sr->mu);
    return sr->budget - sr->used;
}

void tpx_server_destroy(tpx_server* sr) {
    if (!sr) return;
    for (auto& sl : sr->slots)
        if (sl.sv) tpx_service_destroy(sl.sv);
    for (auto h : sr->hs) {
        (void)hipStreamSynchronize(h);
        (void)hipStreamDestroy(h);
    }
    delete sr;
}

}  // extern "C"
