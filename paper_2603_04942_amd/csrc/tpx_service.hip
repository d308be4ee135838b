// Continuous batching over one tpx_stream: chunks are admitted into a device
// ring buffer as they arrive (tpx_service_submit) and every run processes all
// whole chunks admitted so far, up to a batch limit, as one call of the
// stream path (tpx_service_run).  The stream path gives the same hits for any
// split of the stream into chunks, so batching changes when results appear,
// never what they are.
#include <deque>
#include <utility>

#include "tpx_kernels.h"

struct tpx_service {
    tpx_stream* st = nullptr;
    uint64_t* ring = nullptr;     // device u64[ring_cap]
    uint64_t* stage = nullptr;    // device u64[max_batch]: a batch that wraps the ring
    uint64_t ring_cap = 0, max_batch = 0;
    uint64_t wpos = 0, rpos = 0;  // words admitted / processed since creation
    uint64_t n_sub = 0, n_done = 0;
    std::deque<uint64_t> ends;    // end position of every admitted, unprocessed chunk
};

namespace {

void free_service(tpx_service* sv) {
    if (sv->st) tpx_stream_destroy(sv->st);
    if (sv->ring) (void)hipFree(sv->ring);
    if (sv->stage) (void)hipFree(sv->stage);
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
    *out_h = sv;
    return TPX_OK;
}

tpx_status tpx_service_submit(tpx_service* sv, const uint64_t* chunk, size_t n_pkts,
                              int chunk_on_device, uint64_t* seq_h, void* stream) {
    if (!sv || (n_pkts && !chunk)) return tpx::report(TPX_EINVAL, "NULL argument");
    if (n_pkts > sv->max_batch) return tpx::report(TPX_EINVAL, "chunk larger than the batch limit");
    if (sv->wpos + n_pkts - sv->rpos > sv->ring_cap)
        return tpx::report(TPX_ECAPACITY, "ring full: run the service first");
    const tpx_status rc = ring_copy(sv, sv->wpos, chunk, n_pkts,
                                    chunk_on_device ? hipMemcpyDeviceToDevice
                                                    : hipMemcpyHostToDevice,
                                    (hipStream_t)stream);
    if (rc != TPX_OK) return tpx::report(rc, "chunk copy into the ring failed");
    sv->wpos += n_pkts;
    sv->ends.push_back(sv->wpos);
    if (seq_h) *seq_h = sv->n_sub;
    ++sv->n_sub;
    return TPX_OK;
}

tpx_status tpx_service_run(tpx_service* sv, int flush, tpx_hit* hits, size_t hit_cap,
                           size_t* n_hits_h, uint64_t* n_done_h, tpx_stats* stats_h,
                           void* stream) {
    if (!sv || !n_hits_h || !n_done_h) return tpx::report(TPX_EINVAL, "NULL argument");
    hipStream_t hs = (hipStream_t)stream;
    // whole chunks from the front, up to the batch limit
    uint64_t end = sv->rpos;
    size_t take = 0;
    while (take < sv->ends.size() && sv->ends[take] - sv->rpos <= sv->max_batch)
        end = sv->ends[take++];
    const uint64_t n = end - sv->rpos;
    const bool last = take == sv->ends.size();
    const uint64_t* src = sv->ring + sv->rpos % sv->ring_cap;
    if (n && sv->rpos % sv->ring_cap + n > sv->ring_cap) {
        const uint64_t first = sv->ring_cap - sv->rpos % sv->ring_cap;
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
    sv->rpos = end;
    sv->ends.erase(sv->ends.begin(), sv->ends.begin() + take);
    sv->n_done += take;
    *n_done_h = sv->n_done;
    return TPX_OK;
}

void tpx_service_destroy(tpx_service* sv) {
    if (sv) free_service(sv);
}

}  // extern "C"
