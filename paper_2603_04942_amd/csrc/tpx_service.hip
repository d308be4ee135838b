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
#include <deque>
#include <mutex>
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

}  // extern "C"
