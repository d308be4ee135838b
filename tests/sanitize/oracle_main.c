/* Test driver (test infrastructure): runs the oracle's whole path and its
 * local-maximum hits on a packet file, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer so that every access of the oracle is checked.
 *
 *   oracle_sanitized <packets.bin> <hits.bin> <maxima.bin> [walk.bin]
 *
 * packets.bin: little-endian u64 words; walk.bin: 1024 doubles (optional).
 * Writes the orc_hit records of orc_run, then those of orc_local_maxima over
 * the decoded events.  Exit status 0 on success; a sanitizer finding aborts.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/tpx_oracle.c"

static void* read_all(const char* path, size_t* bytes)
{
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    void* buf = malloc(n > 0 ? (size_t)n : 1);
    if (buf && n > 0 && fread(buf, 1, (size_t)n, f) != (size_t)n) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    *bytes = n > 0 ? (size_t)n : 0;
    return buf;
}

static int write_all(const char* path, const void* p, size_t bytes)
{
    FILE* f = fopen(path, "wb");
    if (!f) return -1;
    size_t w = bytes ? fwrite(p, 1, bytes, f) : 0;
    fclose(f);
    return w == bytes ? 0 : -1;
}

int main(int argc, char** argv)
{
    if (argc < 4) {
        fprintf(stderr, "usage: %s packets.bin hits.bin maxima.bin [walk.bin]\n", argv[0]);
        return 2;
    }
    size_t bytes = 0, wbytes = 0;
    uint64_t* pk = (uint64_t*)read_all(argv[1], &bytes);
    if (!pk) return 3;
    const size_t n = bytes / 8;
    double* walk = NULL;
    if (argc > 4) {
        walk = (double*)read_all(argv[4], &wbytes);
        if (!walk || wbytes != 1024 * sizeof(double)) return 3;
    }
    orc_params p = {1, 128, 64000, 0xF, 12800000000ull, 0, 0, walk};
    const size_t cap = n ? n : 1;
    orc_hit* hits = (orc_hit*)malloc(cap * sizeof(orc_hit));
    orc_stats st;
    size_t nh = 0;
    int rc = orc_run(pk, n, &p, hits, cap, &nh, &st);
    if (rc != ORC_OK) return 10 - rc;
    if (write_all(argv[2], hits, nh * sizeof(orc_hit))) return 4;

    uint16_t* ex = (uint16_t*)malloc(cap * sizeof(uint16_t));
    uint16_t* ey = (uint16_t*)malloc(cap * sizeof(uint16_t));
    uint16_t* et = (uint16_t*)malloc(cap * sizeof(uint16_t));
    uint32_t* es = (uint32_t*)malloc(cap * sizeof(uint32_t));
    uint64_t* ea = (uint64_t*)malloc(cap * sizeof(uint64_t));
    uint64_t* tr = (uint64_t*)malloc(cap * sizeof(uint64_t));
    size_t ne = 0, nt = 0, nm = 0;
    rc = orc_decode(pk, n, &p, ex, ey, et, es, ea, cap, &ne, tr, cap, &nt, NULL, &st);
    if (rc != ORC_OK) return 20 - rc;
    orc_hit* mx = (orc_hit*)malloc((ne ? ne : 1) * sizeof(orc_hit));
    rc = orc_local_maxima(ne, ex, ey, et, es, ea, 1, 128, tr, nt, walk, mx, ne, &nm);
    if (rc != ORC_OK) return 30 - rc;
    if (write_all(argv[3], mx, nm * sizeof(orc_hit))) return 4;
    free(pk); free(walk); free(hits); free(ex); free(ey); free(et); free(es); free(ea);
    free(tr); free(mx);
    return 0;
}
