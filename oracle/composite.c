/*
 * Float64 front-to-back alpha compositing over per-tile Gaussian lists.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle).  Built with gcc as its own
 * shared object and called through ctypes by the oracle's Python code; the GPU
 * path never links or loads it.
 *
 * Rule (3D Gaussian Splatting volume rendering, which the paper's batch
 * renderer evaluates per pixel; constants fixed by the renderer's target
 * specification): pixel p = (x + 0.5, y + 0.5) visits the Gaussians of its
 * tile's list in ascending (depth, index) order with T = 1, C = 0, D = 0:
 *     q     = d^T Conic d,  d = p - (u, v)
 *     alpha = min(0.99, o * exp(-q / 2))
 *     alpha < 1/255            -> skip this Gaussian
 *     T' = T (1 - alpha) < 1e-4 -> stop, without adding this Gaussian
 *     otherwise C += rgb alpha T, D += z alpha T, T = T'
 * Output rgb = C + T bg, depth = D / (1 - T) if anything was added else 0,
 * alpha = 1 - T.
 *
 * Threshold decisions taken within a relative distance `margin` of their
 * boundary (|alpha*255 - 1| or |T'/1e-4 - 1|) are "flagged": a float32
 * implementation may legitimately take either branch.  A variant of a pixel is
 * one run in which flip bit k inverts the k-th flagged decision met along the
 * list (counting the decisions of that run, so flipping an early one can bring
 * later ones into play).  oracle_composite evaluates, for every pixel, the
 * variants of the first `max_flags` flagged decisions (2^max_flags results,
 * the first unflipped); oracle_pixel_variants enumerates every variant of one
 * pixel, widening the flip set until no run meets more flagged decisions than
 * it covers.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    const double *u, *v, *ca, *cb, *cc, *op, *rgb, *z;
} gattr_t;

typedef struct {
    double rgb[3];
    double depth;
    double alpha;
    int64_t visited;
    int nflag;
} pix_t;

static void run_pixel(const uint32_t *list, int64_t n, double px, double py, const gattr_t *A,
                      const double *bg, double margin, unsigned flips, int max_flags, pix_t *out)
{
    const double amin = 1.0 / 255.0;
    const double tmin = 1e-4;
    double T = 1.0, c0 = 0.0, c1 = 0.0, c2 = 0.0, D = 0.0;
    int added = 0, nflag = 0;
    int64_t k;
    for (k = 0; k < n; ++k) {
        const uint32_t g = list[k];
        const double dx = px - A->u[g];
        const double dy = py - A->v[g];
        const double q = A->ca[g] * dx * dx + 2.0 * A->cb[g] * dx * dy + A->cc[g] * dy * dy;
        double a = A->op[g] * exp(-0.5 * q);
        if (a > 0.99) a = 0.99;
        int skip = a < amin;
        if (fabs(a / amin - 1.0) < margin) {
            if (nflag < max_flags && ((flips >> nflag) & 1u)) skip = !skip;
            ++nflag;
        }
        if (skip) continue;
        const double Tn = T * (1.0 - a);
        int stop = Tn < tmin;
        if (fabs(Tn / tmin - 1.0) < margin) {
            if (nflag < max_flags && ((flips >> nflag) & 1u)) stop = !stop;
            ++nflag;
        }
        if (stop) { ++k; break; }
        const double w = a * T;
        c0 += A->rgb[3 * (size_t)g + 0] * w;
        c1 += A->rgb[3 * (size_t)g + 1] * w;
        c2 += A->rgb[3 * (size_t)g + 2] * w;
        D += A->z[g] * w;
        T = Tn;
        added = 1;
    }
    out->visited = k;
    out->rgb[0] = c0 + T * bg[0];
    out->rgb[1] = c1 + T * bg[1];
    out->rgb[2] = c2 + T * bg[2];
    out->depth = added ? D / (1.0 - T) : 0.0;
    out->alpha = 1.0 - T;
    out->nflag = nflag;
}

/*
 * ranges: [tiles_x * tiles_y][2] (start, end) into `values` (Gaussian ids).
 * Per-Gaussian arrays are indexed by Gaussian id; rgb is [N][3].
 * Outputs: rgb [H][W][3], depth/alpha [H][W], variants var_rgb
 * [2^max_flags][H][W][3] and var_depth [2^max_flags][H][W] (may be NULL),
 * nflag [H][W] (primary run's flagged-decision count; +65536 when a variant
 * met more flagged decisions than max_flags), visited [H][W] (list entries
 * visited up to termination).  Returns 0.
 */
/* Threads the compositing loop runs on (OpenMP's default team size). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the team size of later compositing calls (n >= 1); returns the new size. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return oracle_threads();
}

int oracle_composite(int W, int H, int ts, int tiles_x, const int64_t *ranges, const uint32_t *values,
                     const double *u, const double *v, const double *ca, const double *cb, const double *cc,
                     const double *op, const double *rgb, const double *z, const double *bg,
                     double margin, int max_flags,
                     double *out_rgb, double *out_depth, double *out_alpha,
                     double *var_rgb, double *var_depth, double *var_alpha, int32_t *nflag_out,
                     int64_t *visited_out)
{
    gattr_t A = {u, v, ca, cb, cc, op, rgb, z};
    const int nvar = 1 << max_flags;
    const size_t npix = (size_t)W * (size_t)H;
    int y;
#pragma omp parallel for schedule(dynamic, 1)
    for (y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            const int64_t t = (int64_t)(y / ts) * tiles_x + (x / ts);
            const int64_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
            const double px = x + 0.5, py = y + 0.5;
            pix_t r0;
            run_pixel(values + s0, s1 - s0, px, py, &A, bg, margin, 0u, max_flags, &r0);
            out_rgb[3 * p + 0] = r0.rgb[0];
            out_rgb[3 * p + 1] = r0.rgb[1];
            out_rgb[3 * p + 2] = r0.rgb[2];
            out_depth[p] = r0.depth;
            out_alpha[p] = r0.alpha;
            visited_out[p] = r0.visited;
            int unresolved = r0.nflag > max_flags;
            for (int f = 0; f < nvar; ++f) {
                pix_t rf = r0;
                if (r0.nflag > 0 && f > 0) {
                    run_pixel(values + s0, s1 - s0, px, py, &A, bg, margin, (unsigned)f, max_flags, &rf);
                    if (rf.nflag > max_flags) unresolved = 1;
                }
                if (var_rgb) {
                    double *d = var_rgb + ((size_t)f * npix + p) * 3;
                    d[0] = rf.rgb[0];
                    d[1] = rf.rgb[1];
                    d[2] = rf.rgb[2];
                }
                if (var_depth) var_depth[(size_t)f * npix + p] = rf.depth;
                if (var_alpha) var_alpha[(size_t)f * npix + p] = rf.alpha;
            }
            nflag_out[p] = r0.nflag + (unresolved ? 65536 : 0);
        }
    }
    return 0;
}

/*
 * Every admissible result of pixel (x, y): all 2^m variants, where m is the
 * smallest flip-set size such that no variant run meets more than m flagged
 * decisions (m starts at the unflipped run's count).  Results go to
 * out_rgb [2^m][3], out_depth [2^m], out_alpha [2^m] (room for 2^max_m each);
 * returns 2^m, or -1 if m would exceed max_m.
 */
int oracle_pixel_variants(int x, int y, int ts, int tiles_x, const int64_t *ranges, const uint32_t *values,
                          const double *u, const double *v, const double *ca, const double *cb, const double *cc,
                          const double *op, const double *rgb, const double *z, const double *bg, double margin,
                          int max_m, double *out_rgb, double *out_depth, double *out_alpha)
{
    gattr_t A = {u, v, ca, cb, cc, op, rgb, z};
    const int64_t t = (int64_t)(y / ts) * tiles_x + (x / ts);
    const int64_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
    const double px = x + 0.5, py = y + 0.5;
    pix_t r;
    run_pixel(values + s0, s1 - s0, px, py, &A, bg, margin, 0u, 31, &r);
    int m = r.nflag;
    for (;;) {
        if (m > max_m) return -1;
        int widest = m;
        for (unsigned f = 0; f < (1u << m); ++f) {
            run_pixel(values + s0, s1 - s0, px, py, &A, bg, margin, f, m, &r);
            if (r.nflag > widest) widest = r.nflag;
            out_rgb[3 * (size_t)f + 0] = r.rgb[0];
            out_rgb[3 * (size_t)f + 1] = r.rgb[1];
            out_rgb[3 * (size_t)f + 2] = r.rgb[2];
            out_depth[f] = r.depth;
            out_alpha[f] = r.alpha;
        }
        if (widest == m) return (int)(1u << m);
        m = widest;
    }
}
