/*
 * Drives the FP64 oracle (degrid, grid, table gradients) under
 * AddressSanitizer and UndefinedBehaviorSanitizer on small seeded problems,
 * including coordinates at and beyond the edges of the valid box, NaN and
 * infinities, empty subgrids, oversampling factors that are not powers of two
 * and subgrids deeper than the w support.
 *
 * Usage: oracle_sanitize OUT_FILE
 * Writes, per case, the inputs and outputs as raw little-endian arrays, so
 * that the test can recompute the case with the ordinary build of the oracle
 * and compare.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_degrid(int64_t n_sub, int32_t n_v, int32_t n_u, int32_t n_w, int32_t support_uv,
                      int32_t support_w, int32_t os_uv, int32_t os_w, const double* subgrids,
                      const double* g_uv, const double* g_w, const double* uvw, const int64_t* offsets,
                      double* vis);
int64_t oracle_grid(int64_t n_sub, int32_t n_v, int32_t n_u, int32_t n_w, int32_t support_uv,
                    int32_t support_w, int32_t os_uv, int32_t os_w, const double* vis, const double* g_uv,
                    const double* g_w, const double* uvw, const int64_t* offsets, double* subgrids);
int64_t oracle_table_grad(int64_t n_sub, int32_t n_v, int32_t n_u, int32_t n_w, int32_t support_uv,
                          int32_t support_w, int32_t os_uv, int32_t os_w, const double* subgrids,
                          const double* g_uv, const double* g_w, const double* uvw, const int64_t* offsets,
                          const double* grad_vis, double* grad_uv, double* grad_w);

static uint64_t rng_state;

static double uniform01(void)
{
    /* 64-bit LCG (Knuth's MMIX constants), top 53 bits */
    rng_state = rng_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void put(FILE* f, const void* p, size_t bytes)
{
    if (bytes > 0 && fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short write\n");
        exit(2);
    }
}

static void* take(size_t bytes)
{
    void* p = calloc(bytes > 0 ? bytes : 1, 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* One case: S subgrids of n_v x n_u x n_w, the given counts per subgrid. */
static void run_case(FILE* f, uint64_t seed, int32_t n_v, int32_t n_u, int32_t n_w, int32_t os_uv, int32_t os_w,
                     int64_t n_sub, const int64_t* counts)
{
    const int32_t su = 8, sw = 4;
    rng_state = seed;
    int64_t* off = take(sizeof(int64_t) * (size_t)(n_sub + 1));
    for (int64_t s = 0; s < n_sub; ++s) off[s + 1] = off[s] + counts[s];
    const int64_t n = off[n_sub];
    const size_t cells = (size_t)n_sub * n_v * n_u * n_w;
    double* sub = take(sizeof(double) * 2 * cells);
    double* g_uv = take(sizeof(double) * (size_t)os_uv * os_uv * su * su);
    double* g_w = take(sizeof(double) * (size_t)os_w * sw);
    double* uvw = take(sizeof(double) * 3 * (size_t)n);
    double* gv = take(sizeof(double) * 2 * (size_t)n);
    for (size_t i = 0; i < 2 * cells; ++i) sub[i] = uniform01() - 0.5;
    for (size_t i = 0; i < (size_t)os_uv * os_uv * su * su; ++i) g_uv[i] = uniform01();
    for (size_t i = 0; i < (size_t)os_w * sw; ++i) g_w[i] = uniform01();
    for (int64_t i = 0; i < n; ++i) {
        uvw[3 * i] = 2.0 + uniform01() * (n_u - 3.0);
        uvw[3 * i + 1] = 2.0 + uniform01() * (n_v - 3.0);
        uvw[3 * i + 2] = uniform01() * (n_w - 1.0);
        gv[2 * i] = uniform01() - 0.5;
        gv[2 * i + 1] = uniform01() - 0.5;
    }
    /* edge and non-finite coordinates on the first visibilities */
    const double special[] = {3.0, nextafter(3.0, 0.0), (double)n_u - 4.0, nextafter((double)n_u - 4.0, 0.0),
                              NAN, INFINITY, -INFINITY, -1e300, 1e300, -0.0};
    const int n_special = (int)(sizeof(special) / sizeof(special[0]));
    for (int64_t i = 0; i < n && i < 3 * n_special; ++i) uvw[3 * i + (i % 3)] = special[(i / 3) % n_special];

    double* vis = take(sizeof(double) * 2 * (size_t)n);
    double* grid = take(sizeof(double) * 2 * cells);
    double* d_uv = take(sizeof(double) * (size_t)os_uv * os_uv * su * su);
    double* d_w = take(sizeof(double) * (size_t)os_w * sw);
    const int64_t oob_d = oracle_degrid(n_sub, n_v, n_u, n_w, su, sw, os_uv, os_w, sub, g_uv, g_w, uvw, off, vis);
    const int64_t oob_g = oracle_grid(n_sub, n_v, n_u, n_w, su, sw, os_uv, os_w, gv, g_uv, g_w, uvw, off, grid);
    const int64_t oob_t = oracle_table_grad(n_sub, n_v, n_u, n_w, su, sw, os_uv, os_w, sub, g_uv, g_w, uvw, off,
                                            gv, d_uv, d_w);

    const int64_t head[8] = {n_sub, n_v, n_u, n_w, os_uv, os_w, n, 0};
    put(f, head, sizeof(head));
    put(f, off, sizeof(int64_t) * (size_t)(n_sub + 1));
    put(f, sub, sizeof(double) * 2 * cells);
    put(f, g_uv, sizeof(double) * (size_t)os_uv * os_uv * su * su);
    put(f, g_w, sizeof(double) * (size_t)os_w * sw);
    put(f, uvw, sizeof(double) * 3 * (size_t)n);
    put(f, gv, sizeof(double) * 2 * (size_t)n);
    const int64_t oob[3] = {oob_d, oob_g, oob_t};
    put(f, oob, sizeof(oob));
    put(f, vis, sizeof(double) * 2 * (size_t)n);
    put(f, grid, sizeof(double) * 2 * cells);
    put(f, d_uv, sizeof(double) * (size_t)os_uv * os_uv * su * su);
    put(f, d_w, sizeof(double) * (size_t)os_w * sw);
    free(off); free(sub); free(g_uv); free(g_w); free(uvw); free(gv);
    free(vis); free(grid); free(d_uv); free(d_w);
}

int main(int argc, char** argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: %s OUT_FILE\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "wb");
    if (!f) return 2;
    const int64_t c0[] = {300, 0, 41, 1};
    const int64_t c1[] = {0, 0};
    const int64_t c2[] = {257, 120};
    const int64_t c3[] = {90};
    run_case(f, 1, 24, 32, 4, 16, 16, 4, c0);     /* power-of-two oversampling */
    run_case(f, 2, 16, 16, 4, 16, 16, 2, c1);     /* no visibilities */
    run_case(f, 3, 20, 28, 4, 5, 7, 2, c2);       /* oversampling not a power of two */
    run_case(f, 4, 16, 24, 9, 8, 12, 1, c3);      /* w planes beyond the support */
    fclose(f);
    puts("ok");
    return 0;
}
