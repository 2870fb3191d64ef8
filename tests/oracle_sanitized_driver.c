/*
 * Host driver for the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (TEST INFRASTRUCTURE ONLY; built and run by
 * tests/test_oracle_sanitized.py).  It reads raw pairs, builds the canonical
 * CSR with oracle_canonical_csr, evaluates every vertex with oracle_net, and
 * writes both, so the test can compare them with the regular build.
 *
 * input:  int64 n, int64 m, int32 src[m], int32 dst[m]
 * output: int64 nnz, int64 off[n + 1], int32 idx[nnz], int64 net[n][16]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_canonical_csr(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t* off, int32_t* idx,
                         int nthreads);
int oracle_net(int64_t n, const int64_t* off, const int32_t* idx, int64_t nsel, const int64_t* sel, int64_t* net,
               int nthreads);

static int read_all(FILE* f, void* p, size_t size, size_t count) { return fread(p, size, count, f) == count; }

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 3;
    int64_t n = 0, m = 0;
    if (!read_all(in, &n, sizeof n, 1) || !read_all(in, &m, sizeof m, 1)) return 4;
    int32_t* src = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* dst = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!src || !dst) return 5;
    if (m > 0 && (!read_all(in, src, sizeof(int32_t), (size_t)m) || !read_all(in, dst, sizeof(int32_t), (size_t)m)))
        return 6;
    fclose(in);
    int64_t* off = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* idx = malloc(sizeof(int32_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
    if (!off || !idx) return 7;
    int st = oracle_canonical_csr(n, m, src, dst, off, idx, 2);
    if (st != 0) return 10 - st;
    const int64_t nnz = off[n];
    int64_t* net = calloc((size_t)(n > 0 ? n : 1) * 16, sizeof(int64_t));
    if (!net) return 8;
    st = oracle_net(n, off, idx, n, NULL, net, 2);
    if (st != 0) return 20 - st;
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 9;
    fwrite(&nnz, sizeof nnz, 1, out);
    fwrite(off, sizeof(int64_t), (size_t)n + 1, out);
    fwrite(idx, sizeof(int32_t), (size_t)nnz, out);
    fwrite(net, sizeof(int64_t), (size_t)n * 16, out);
    fclose(out);
    free(src);
    free(dst);
    free(off);
    free(idx);
    free(net);
    return 0;
}
