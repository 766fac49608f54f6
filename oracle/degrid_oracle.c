/*
 * FP64 reference ("oracle") for 3D degridding and its adjoint (gridding).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The product library never
 * calls it, links it or shares code with it: the two are written separately
 * so that one can check the other.
 *
 * What it computes (Section 2 of the paper, "Implementation"): degridding is
 * a weighted sum of regularly sampled values. The inputs are an oversampled
 * GCF for the uv plane G_uv with 8x8 support, an oversampled GCF for w G_w
 * with support 4, a stack of S subgrids of 512x512x4 and, for each subgrid,
 * its list of visibility coordinates [u,v,w]. For every visibility two sets
 * of coordinates are formed: the subgrid point g = [x,y,z] where the sum
 * starts, and the position of the weights inside the oversampled tables.
 * The visibility is then the sum over the support of
 *     G_w[o_w][t_w] * G_uv[o_v][o_u][t_v][t_u] * A[y+t_v][x+t_u][z+t_w].
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes of the repository):
 *   - subgrid memory order [S][v][u][w], w fastest, complex interleaved;
 *   - coordinates in subgrid cells with the origin at cell 0;
 *   - per axis, k = floor(c * os) of the FP64 product (exact for os = 2^m;
 *     for other factors the rounding of the product is part of the
 *     definition), the cell n = floor(k / os), the oversample index
 *     o = k - n * os, and the first tap n - (W/2 - 1);
 *   - G_uv indexed [o_v][o_u][t_v][t_u], G_w indexed [o_w][t_w];
 *   - a neighbourhood that would leave the subgrid is not wrapped or
 *     clamped: the visibility is 0 and is counted as out of range;
 *   - weights are real; values are complex.
 * The adjoint (gridding) is the transpose of the same real linear map:
 *     grid(V)[s][y+t_v][x+t_u][z+t_w] += G_w * G_uv * V_i.
 *
 * Plain loops, no blocking, no reordering beyond the definition. OpenMP only
 * splits independent visibilities (degrid) or independent subgrids (grid).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Geometry and tables shared by one call. */
typedef struct {
    int64_t n_sub;
    int32_t n_v, n_u, n_w;
    int32_t support_uv, support_w;
    int32_t os_uv, os_w;
} oracle_geom;

/*
 * Start of the support and oversample index along one axis.
 * Returns 1 if the whole support lies in [0, n_cells), else 0.
 */
static int axis_coordinates(double c, int32_t os, int32_t support, int32_t n_cells,
                            int64_t* start, int32_t* oversample)
{
    if (!isfinite(c)) return 0;
    double k = floor(c * (double)os);           /* quantised position in 1/os cells */
    double n = floor(k / (double)os);           /* cell holding the coordinate      */
    double o = k - n * (double)os;              /* offset inside the cell, [0, os)  */
    double first = n - (double)(support / 2 - 1);
    if (!(first >= 0.0) || !(first <= (double)(n_cells - support))) return 0;
    *start = (int64_t)first;
    *oversample = (int32_t)o;
    return 1;
}

/* Index of subgrid s that owns visibility i (offsets non-decreasing). */
static int64_t owner(const int64_t* offsets, int64_t n_sub, int64_t i)
{
    int64_t lo = 0, hi = n_sub;          /* invariant: offsets[lo] <= i < offsets[hi] */
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (offsets[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

static int visibility_coordinates(const oracle_geom* g, const double* uvw_i,
                                  int64_t* x, int64_t* y, int64_t* z,
                                  int32_t* o_u, int32_t* o_v, int32_t* o_w)
{
    int ok_u = axis_coordinates(uvw_i[0], g->os_uv, g->support_uv, g->n_u, x, o_u);
    int ok_v = axis_coordinates(uvw_i[1], g->os_uv, g->support_uv, g->n_v, y, o_v);
    int ok_w = axis_coordinates(uvw_i[2], g->os_w, g->support_w, g->n_w, z, o_w);
    return ok_u && ok_v && ok_w;
}

/*
 * Degrid: vis[i] (re, im) for every visibility i in [0, offsets[n_sub]).
 * subgrids: [S][n_v][n_u][n_w][2] FP64; g_uv: [os][os][W][W]; g_w: [os_w][Ww];
 * uvw: [N][3]; offsets: [S+1]. Returns the number of out-of-range visibilities.
 */
int64_t oracle_degrid(int64_t n_sub, int32_t n_v, int32_t n_u, int32_t n_w,
                      int32_t support_uv, int32_t support_w, int32_t os_uv, int32_t os_w,
                      const double* subgrids, const double* g_uv, const double* g_w,
                      const double* uvw, const int64_t* offsets, double* vis)
{
    oracle_geom g = { n_sub, n_v, n_u, n_w, support_uv, support_w, os_uv, os_w };
    int64_t n_vis = offsets[n_sub];
    int64_t oob = 0;
    #pragma omp parallel for schedule(static) reduction(+:oob)
    for (int64_t i = 0; i < n_vis; ++i) {
        int64_t s = owner(offsets, n_sub, i);
        int64_t x, y, z;
        int32_t o_u, o_v, o_w;
        double re = 0.0, im = 0.0;
        if (visibility_coordinates(&g, uvw + 3 * i, &x, &y, &z, &o_u, &o_v, &o_w)) {
            const double* guv = g_uv + ((int64_t)o_v * os_uv + o_u) * support_uv * support_uv;
            const double* gw = g_w + (int64_t)o_w * support_w;
            for (int32_t tv = 0; tv < support_uv; ++tv)
                for (int32_t tu = 0; tu < support_uv; ++tu)
                    for (int32_t tw = 0; tw < support_w; ++tw) {
                        double weight = gw[tw] * guv[tv * support_uv + tu];
                        int64_t cell = ((s * n_v + (y + tv)) * n_u + (x + tu)) * n_w + (z + tw);
                        re += weight * subgrids[2 * cell];
                        im += weight * subgrids[2 * cell + 1];
                    }
        } else {
            oob += 1;
        }
        vis[2 * i] = re;
        vis[2 * i + 1] = im;
    }
    return oob;
}

/*
 * Grid (adjoint of degrid): subgrids_out = W^T vis, overwritten (zeroed
 * first). Same shapes as oracle_degrid. Returns the out-of-range count.
 */
int64_t oracle_grid(int64_t n_sub, int32_t n_v, int32_t n_u, int32_t n_w,
                    int32_t support_uv, int32_t support_w, int32_t os_uv, int32_t os_w,
                    const double* vis, const double* g_uv, const double* g_w,
                    const double* uvw, const int64_t* offsets, double* subgrids_out)
{
    oracle_geom g = { n_sub, n_v, n_u, n_w, support_uv, support_w, os_uv, os_w };
    int64_t cells_per_sub = (int64_t)n_v * n_u * n_w;
    int64_t oob = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(+:oob)
    for (int64_t s = 0; s < n_sub; ++s) {
        double* out = subgrids_out + 2 * s * cells_per_sub;
        memset(out, 0, sizeof(double) * 2 * (size_t)cells_per_sub);
        for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) {
            int64_t x, y, z;
            int32_t o_u, o_v, o_w;
            if (!visibility_coordinates(&g, uvw + 3 * i, &x, &y, &z, &o_u, &o_v, &o_w)) {
                oob += 1;
                continue;
            }
            const double* guv = g_uv + ((int64_t)o_v * os_uv + o_u) * support_uv * support_uv;
            const double* gw = g_w + (int64_t)o_w * support_w;
            for (int32_t tv = 0; tv < support_uv; ++tv)
                for (int32_t tu = 0; tu < support_uv; ++tu)
                    for (int32_t tw = 0; tw < support_w; ++tw) {
                        double weight = gw[tw] * guv[tv * support_uv + tu];
                        int64_t cell = (((y + tv)) * n_u + (x + tu)) * n_w + (z + tw);
                        out[2 * cell] += weight * vis[2 * i];
                        out[2 * cell + 1] += weight * vis[2 * i + 1];
                    }
        }
    }
    return oob;
}

/*
 * Gradients of a real loss L with respect to the two tables, given its
 * gradient with respect to the visibilities, grad_vis[i] = dL/dRe(V_i) +
 * i dL/dIm(V_i) (pairs re, im). Each visibility is linear in each table
 * (real weights, complex values), so by the chain rule
 *   dL/dG_uv[o_v][o_u][t_v][t_u] = sum over in-range i with offsets (o_v, o_u) of
 *       Re(conj(grad_vis[i]) * sum_tw G_w[o_w][t_w] * A[y+t_v][x+t_u][z+t_w]),
 *   dL/dG_w[o_w][t_w] = sum over in-range i with offset o_w of
 *       Re(conj(grad_vis[i]) * sum_{t_v,t_u} G_uv[o_v][o_u][t_v][t_u] * A[y+t_v][x+t_u][z+t_w]),
 * where Re(conj(g) * c) = g.re * c.re + g.im * c.im. Out-of-range
 * visibilities add nothing. grad_g_uv ([os][os][W][W]) and grad_g_w
 * ([os_w][Ww]) are overwritten; either may be NULL. One serial pass over
 * the visibilities. Returns the out-of-range count.
 */
int64_t oracle_table_grad(int64_t n_sub, int32_t n_v, int32_t n_u, int32_t n_w,
                          int32_t support_uv, int32_t support_w, int32_t os_uv, int32_t os_w,
                          const double* subgrids, const double* g_uv, const double* g_w,
                          const double* uvw, const int64_t* offsets, const double* grad_vis,
                          double* grad_g_uv, double* grad_g_w)
{
    oracle_geom g = { n_sub, n_v, n_u, n_w, support_uv, support_w, os_uv, os_w };
    if (grad_g_uv)
        memset(grad_g_uv, 0, sizeof(double) * (size_t)os_uv * os_uv * support_uv * support_uv);
    if (grad_g_w)
        memset(grad_g_w, 0, sizeof(double) * (size_t)os_w * support_w);
    int64_t oob = 0;
    for (int64_t s = 0; s < n_sub; ++s) {
        for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) {
            int64_t x, y, z;
            int32_t o_u, o_v, o_w;
            if (!visibility_coordinates(&g, uvw + 3 * i, &x, &y, &z, &o_u, &o_v, &o_w)) {
                oob += 1;
                continue;
            }
            const double gre = grad_vis[2 * i], gim = grad_vis[2 * i + 1];
            const int64_t uv_row = ((int64_t)o_v * os_uv + o_u) * support_uv * support_uv;
            const double* gw = g_w + (int64_t)o_w * support_w;
            for (int32_t tv = 0; tv < support_uv; ++tv)
                for (int32_t tu = 0; tu < support_uv; ++tu) {
                    const double guv = g_uv[uv_row + tv * support_uv + tu];
                    double c_re = 0.0, c_im = 0.0;   /* sum over t_w of G_w * A */
                    for (int32_t tw = 0; tw < support_w; ++tw) {
                        int64_t cell = ((s * n_v + (y + tv)) * n_u + (x + tu)) * n_w + (z + tw);
                        const double a_re = subgrids[2 * cell], a_im = subgrids[2 * cell + 1];
                        c_re += gw[tw] * a_re;
                        c_im += gw[tw] * a_im;
                        if (grad_g_w)
                            grad_g_w[(int64_t)o_w * support_w + tw] += guv * (gre * a_re + gim * a_im);
                    }
                    if (grad_g_uv)
                        grad_g_uv[uv_row + tv * support_uv + tu] += gre * c_re + gim * c_im;
                }
        }
    }
    return oob;
}

/* Threads an OpenMP parallel region of the oracle uses. */
int32_t oracle_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads later parallel regions of the oracle use (timing only). */
void oracle_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}
