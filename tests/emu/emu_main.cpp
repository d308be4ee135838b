// Command-line driver of the host emulation build of libtpx (test
// infrastructure).  Runs one C-ABI call sequence on inputs from a file and
// writes the outputs and the emulator's findings to another file.
//
//   emu_tpx cluster IN OUT   IN: u64 n, u32 dxy, u32 dt, x u16[n], y u16[n],
//                                tot u16[n], shot u32[n], toa u64[n]
//                            OUT: i32 status, u64 n_clusters, labels u32[n]
//   emu_tpx stream IN OUT    IN: u64 n, u64 chunk, i64 pix_epoch0,
//                                i64 tdc_epoch0, u32 q, i32 kernel
//                                (-1 staged, >= 0 fused variant),
//                                i32 persistent (0 / 1), [chunk 0: u64 count,
//                                u64 sizes[count]], packets u64[n]
//                            OUT: i32 status, u64 n_hits, tpx_hit[n_hits]
// Both append: u64 error-text length, error text (empty = no finding).
//   emu_tpx selftest         runs kernels with planted synchronisation
//                            mistakes and prints what the emulator reports
#include <stdio.h>
#include <stdlib.h>

#include <string>
#include <vector>

#include <cstring>

#include "hip_emu.h"
#include "../../include/tpx.h"

extern "C" const char* emu_errors();
int emu_selftest(FILE* out);
extern "C" uint32_t tpx_stream_get_segment(const tpx_stream* s);

namespace tpx {
struct ClusterArgs;
// the learned patches are not part of the emulation build
void launch_stream_patches(const ClusterArgs&, uint64_t, bool, const tpx_hit*, uint64_t,
                           uint32_t*, uint16_t*, int*, hipStream_t) {
    fprintf(stderr, "emu: learned patches are not emulated\n");
    abort();
}
}  // namespace tpx

namespace {

struct In {
    std::vector<char> b;
    size_t p = 0;
    template <class T>
    T get() {
        T v;
        memcpy(&v, b.data() + p, sizeof(T));
        p += sizeof(T);
        return v;
    }
    template <class T>
    void arr(T* dst, size_t n) {
        memcpy(dst, b.data() + p, n * sizeof(T));
        p += n * sizeof(T);
    }
};

template <class T>
T* dev(size_t n) {
    void* p = nullptr;
    hipMalloc(&p, n * sizeof(T) + 1);
    return (T*)p;
}

void put(FILE* f, const void* p, size_t n) { fwrite(p, 1, n, f); }

void put_errors(FILE* f) {
    const std::string e = emu_errors();
    const uint64_t n = e.size();
    put(f, &n, 8);
    put(f, e.data(), n);
}

int run_cluster(In& in, FILE* out) {
    const uint64_t n = in.get<uint64_t>();
    const uint32_t dxy = in.get<uint32_t>(), dt = in.get<uint32_t>();
    tpx_events ev;
    ev.x = dev<uint16_t>(n);
    ev.y = dev<uint16_t>(n);
    ev.tot = dev<uint16_t>(n);
    ev.shot = dev<uint32_t>(n);
    ev.toa = dev<uint64_t>(n);
    in.arr(ev.x, n);
    in.arr(ev.y, n);
    in.arr(ev.tot, n);
    in.arr(ev.shot, n);
    in.arr(ev.toa, n);
    tpx_params p;
    tpx_params_default(&p);
    p.dxy = dxy;
    p.dt_ticks = dt;
    const size_t wsb = tpx_workspace_bytes(0, n);
    void* ws = nullptr;
    hipMalloc(&ws, wsb);
    uint32_t* lab = dev<uint32_t>(n);
    size_t nc = 0;
    const int32_t st = tpx_cluster(ev, n, &p, lab, &nc, ws, wsb, nullptr);
    if (st != TPX_OK) fprintf(stderr, "tpx_cluster: %s\n", tpx_last_error());
    const uint64_t nc64 = nc;
    put(out, &st, 4);
    put(out, &nc64, 8);
    put(out, lab, n * 4);
    put_errors(out);
    return 0;
}

int run_stream(In& in, FILE* out) {
    const uint64_t n = in.get<uint64_t>(), chunk = in.get<uint64_t>();
    const int64_t pe0 = in.get<int64_t>(), te0 = in.get<int64_t>();
    const uint32_t q = in.get<uint32_t>();
    const int32_t kern = in.get<int32_t>();
    const int32_t persist = in.get<int32_t>();
    // chunk 0: a list of chunk sizes follows (u64 count, u64 sizes)
    std::vector<uint64_t> sizes;
    if (chunk == 0) {
        sizes.resize(in.get<uint64_t>());
        for (auto& z : sizes) z = in.get<uint64_t>();
    }
    uint64_t* pk = dev<uint64_t>(n);
    in.arr(pk, n);
    uint64_t max_chunk = chunk;
    for (uint64_t z : sizes) max_chunk = std::max(max_chunk, z);
    tpx_params p;
    tpx_params_default(&p);
    p.pix_epoch0 = pe0;
    p.tdc_epoch0 = te0;
    tpx_stream* s = nullptr;
    int32_t st = tpx_stream_create(&p, max_chunk ? max_chunk : 1, &s);
    std::vector<tpx_hit> all;
    if (st == TPX_OK && q) st = tpx_stream_set_segment(s, q);
    if (st == TPX_OK) st = tpx_stream_set_kernel(s, kern);
    if (st == TPX_OK) st = tpx_stream_set_persistent(s, persist ? 512 : 0);
    const size_t cap = n + 16;
    tpx_hit* hits = dev<tpx_hit>(cap);
    for (uint64_t off = 0, k = 0; st == TPX_OK; ++k) {
        const uint64_t want = chunk ? chunk : (k < sizes.size() ? sizes[k] : n - off);
        const uint64_t m = std::min<uint64_t>(want, n - off);
        // with a size list, the last entry flushes (it may be empty)
        const int flush = chunk ? off + m >= n : k + 1 >= sizes.size();
        size_t nh = 0;
        st = tpx_process_stream(s, pk + off, m, flush, hits, cap, &nh, nullptr, nullptr);
        if (st != TPX_OK) {
            fprintf(stderr, "tpx_process_stream: %s\n", tpx_last_error());
            break;
        }
        all.insert(all.end(), hits, hits + nh);
        off += m;
        if (flush) break;
    }
    if (s) tpx_stream_destroy(s);
    const uint64_t nh = all.size();
    put(out, &st, 4);
    put(out, &nh, 8);
    put(out, all.data(), nh * sizeof(tpx_hit));
    put_errors(out);
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc == 2 && std::string(argv[1]) == "selftest") return emu_selftest(stdout);
    if (argc != 4) {
        fprintf(stderr, "usage: emu_tpx cluster|stream IN OUT\n");
        return 2;
    }
    In in;
    FILE* f = fopen(argv[2], "rb");
    if (!f) return 2;
    fseek(f, 0, SEEK_END);
    in.b.resize((size_t)ftell(f));
    fseek(f, 0, SEEK_SET);
    if (fread(in.b.data(), 1, in.b.size(), f) != in.b.size()) return 2;
    fclose(f);
    FILE* out = fopen(argv[3], "wb");
    if (!out) return 2;
    const std::string mode = argv[1];
    int rc = 2;
    if (mode == "cluster") rc = run_cluster(in, out);
    else if (mode == "stream") rc = run_stream(in, out);
    fclose(out);
    return rc;
}
