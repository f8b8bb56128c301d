/*
 * Plain FP64 CPU reference for the view-factor radiosity model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark have an independent, obviously-correct answer to
 * compare the GPU path with.  It shares no code with the GPU library.
 *
 * Every routine is a direct transcription of a definition of the paper
 * (Potter et al., "Fast hierarchical low-rank view factor matrices for thermal
 * irradiance on planetary surfaces"):
 *   - facet geometry, midpoint collocation ........ section 3
 *   - view factor entry F_ij (eq. FF-def) ......... section 3
 *   - visibility V_ij: back-face test, then a ray
 *     between centroids (eq. for V_ij) ........... section 3.2
 *   - full matrix, row by row (Algorithm 1) ....... section 3.3
 *   - insolation with a point sun (eq. insolation)  section 2
 * No blocking, no reordering, no acceleration structure: loops over all
 * pairs and all triangles.  OpenMP only splits independent rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* Segment / ray parameters accepted as an occluding hit: t in (T_LO, T_HI). */
#define ORC_T_LO 1e-9
#define ORC_T_HI (1.0 - 1e-9)

static inline double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static inline void sub3(const double *a, const double *b, double *out)
{
    out[0] = a[0] - b[0];
    out[1] = a[1] - b[1];
    out[2] = a[2] - b[2];
}

static inline void cross3(const double *a, const double *b, double *out)
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

int orc_version(void) { return 1; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Section 3: centroid x_i, unit normal n_i and area A_i of triangle i with
 * vertices (a, b, c): x = (a+b+c)/3, n = (b-a)x(c-a)/|.|, A = |(b-a)x(c-a)|/2.
 * Returns the number of degenerate (zero-area) faces; their n is left zero.
 */
int64_t orc_geometry(const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                     double *x, double *n, double *area)
{
    int64_t bad = 0;
    (void)nv;
    for (int64_t i = 0; i < nf; ++i) {
        const double *a = verts + 3 * (int64_t)faces[3 * i + 0];
        const double *b = verts + 3 * (int64_t)faces[3 * i + 1];
        const double *c = verts + 3 * (int64_t)faces[3 * i + 2];
        double e1[3], e2[3], cr[3];
        for (int k = 0; k < 3; ++k)
            x[3 * i + k] = (a[k] + b[k] + c[k]) / 3.0;
        sub3(b, a, e1);
        sub3(c, a, e2);
        cross3(e1, e2, cr);
        double len = sqrt(dot3(cr, cr));
        area[i] = 0.5 * len;
        if (len > 0.0) {
            for (int k = 0; k < 3; ++k)
                n[3 * i + k] = cr[k] / len;
        } else {
            n[3 * i] = n[3 * i + 1] = n[3 * i + 2] = 0.0;
            ++bad;
        }
    }
    return bad;
}

/*
 * Moeller-Trumbore ray/triangle test (Moeller & Trumbore, J. Graphics Tools
 * 1997) for the point o + t d.  A hit needs barycentrics u >= 0, v >= 0,
 * u + v <= 1 (edges count as hits) and t in (tlo, thi).  A ray parallel to
 * the triangle's plane never hits.
 */
static int ray_hits_triangle(const double *o, const double *d, double tlo, double thi,
                             const double *p0, const double *p1, const double *p2)
{
    double e1[3], e2[3], pv[3], tv[3], qv[3];
    sub3(p1, p0, e1);
    sub3(p2, p0, e2);
    cross3(d, e2, pv);
    double det = dot3(e1, pv);
    if (det == 0.0)
        return 0;
    double inv = 1.0 / det;
    sub3(o, p0, tv);
    double u = dot3(tv, pv) * inv;
    if (u < 0.0 || u > 1.0)
        return 0;
    cross3(tv, e1, qv);
    double v = dot3(d, qv) * inv;
    if (v < 0.0 || u + v > 1.0)
        return 0;
    double t = dot3(e2, qv) * inv;
    return t > tlo && t < thi;
}

int orc_ray_hits_triangle(const double *o, const double *d, double tlo, double thi,
                          const double *tri9)
{
    return ray_hits_triangle(o, d, tlo, thi, tri9, tri9 + 3, tri9 + 6);
}

/* Back-face part of V_ij (section 3.2): n_i.(x_j-x_i) > 0 and n_j.(x_i-x_j) > 0. */
static inline int facing(const double *xi, const double *ni, const double *xj, const double *nj)
{
    double r[3];
    sub3(xj, xi, r);
    return dot3(ni, r) > 0.0 && -dot3(nj, r) > 0.0;
}

/* Is the open segment (x_i, x_j) blocked by some triangle k not in {i, j}? */
static int segment_blocked(int64_t i, int64_t j, const double *x, int64_t ntri, const double *tri)
{
    double d[3];
    sub3(x + 3 * j, x + 3 * i, d);
    for (int64_t k = 0; k < ntri; ++k) {
        if (k == i || k == j)
            continue;
        const double *t = tri + 9 * k;
        if (ray_hits_triangle(x + 3 * i, d, ORC_T_LO, ORC_T_HI, t, t + 3, t + 6))
            return 1;
    }
    return 0;
}

/*
 * Pairwise visibility V (section 3.2), full N x N uint8 matrix, row-major.
 * mode 0: back-face test only (every facing pair counts as visible).
 * mode 1: back-face test, then the centroid-to-centroid segment is tested
 *         against every mesh triangle except i and j (brute force).
 * The segment test is evaluated once per unordered pair and mirrored, so V is
 * symmetric.  The diagonal is 0.
 */
void orc_pair_visibility(int64_t N, const double *x, const double *n, int64_t ntri,
                         const double *tri, int mode, uint8_t *vis)
{
    memset(vis, 0, (size_t)(N * N));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = i + 1; j < N; ++j) {
            int v = facing(x + 3 * i, n + 3 * i, x + 3 * j, n + 3 * j);
            if (v && mode == 1)
                v = !segment_blocked(i, j, x, ntri, tri);
            vis[i * N + j] = (uint8_t)v;
            vis[j * N + i] = (uint8_t)v;
        }
    }
}

/* eq. FF-def without the visibility factor: the kernel value for a facing pair. */
static inline double kernel_entry(const double *xi, const double *ni, const double *xj,
                                  const double *nj, double aj)
{
    double r[3];
    sub3(xj, xi, r);
    double ci = dot3(ni, r);
    double cj = -dot3(nj, r);
    if (ci <= 0.0 || cj <= 0.0)
        return 0.0;
    double rr = dot3(r, r);
    return ci * cj * aj / (ORC_PI * rr * rr);
}

/*
 * Dense F (eq. FF-def, Algorithm 1 semantics): F_ij = kernel * V_ij * A_j for
 * i != j, F_ii = 0.  vis == NULL means back-face visibility only.
 * F is N x N row-major.
 */
void orc_F_dense(int64_t N, const double *x, const double *n, const double *area,
                 const uint8_t *vis, double *F)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double v = 0.0;
            if (j != i && (vis == NULL || vis[i * N + j]))
                v = kernel_entry(x + 3 * i, n + 3 * i, x + 3 * j, n + 3 * j, area[j]);
            F[i * N + j] = v;
        }
    }
}

/*
 * Segment test cast from facet i towards facet j for every ordered facing
 * pair (not symmetrised): vis[i*N + j] = 1 when the pair faces and the open
 * segment from x_i to x_j misses every other triangle.  The two directions of
 * one pair can differ where a segment grazes an edge or a vertex; this is the
 * asymmetry that casting once per unordered pair removes.  Test use only.
 */
void orc_directed_visibility(int64_t N, const double *x, const double *n, int64_t ntri,
                             const double *tri, uint8_t *vis)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            int v = j != i && facing(x + 3 * i, n + 3 * i, x + 3 * j, n + 3 * j);
            if (v)
                v = !segment_blocked(i, j, x, ntri, tri);
            vis[i * N + j] = (uint8_t)v;
        }
    }
}

/*
 * Selected rows of F with visibility computed on the fly:
 *   mode 0: back-face only; mode 1: brute-force segment test against tri,
 *   cast from the facet with the smaller index of the pair, exactly as
 *   orc_pair_visibility does, so these rows equal rows of the dense F built
 *   from that symmetric V.
 * out is nrows x N row-major.
 */
void orc_F_rows(int64_t N, const double *x, const double *n, const double *area,
                int64_t ntri, const double *tri, int mode, int64_t nrows,
                const int64_t *rows, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        for (int64_t j = 0; j < N; ++j) {
            double v = 0.0;
            if (j != i) {
                v = kernel_entry(x + 3 * i, n + 3 * i, x + 3 * j, n + 3 * j, area[j]);
                if (v != 0.0 && mode == 1 &&
                    segment_blocked(i < j ? i : j, i < j ? j : i, x, ntri, tri))
                    v = 0.0;
            }
            out[r * N + j] = v;
        }
    }
}

/*
 * Y = F X without storing F (rows computed on the fly), X and Y column-major
 * N x R with leading dimensions ldx, ldy.  vis == NULL: back-face visibility
 * only; else vis is the full N x N uint8 matrix.
 */
void orc_matvec_free(int64_t N, const double *x, const double *n, const double *area,
                     const uint8_t *vis, int64_t R, const double *X, int64_t ldx,
                     double *Y, int64_t ldy)
{
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)(R > 0 ? R : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < N; ++i) {
            for (int64_t r = 0; r < R; ++r)
                acc[r] = 0.0;
            for (int64_t j = 0; j < N; ++j) {
                if (j == i || (vis != NULL && !vis[i * N + j]))
                    continue;
                double f = kernel_entry(x + 3 * i, n + 3 * i, x + 3 * j, n + 3 * j, area[j]);
                if (f == 0.0)
                    continue;
                for (int64_t r = 0; r < R; ++r)
                    acc[r] += f * X[j + r * ldx];
            }
            for (int64_t r = 0; r < R; ++r)
                Y[i + r * ldy] = acc[r];
        }
        free(acc);
    }
}

/*
 * Sun visibility for the insolation (eq. insolation, section 5.1): facet i
 * sees a point sun in unit direction s when the ray x_i + t s, t > 1e-9,
 * hits no mesh triangle other than i.  out is N x R column-major uint8.
 */
void orc_sun_visibility(int64_t N, const double *x, int64_t ntri, const double *tri,
                        int64_t R, const double *suns, uint8_t *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 8)
    for (int64_t r = 0; r < R; ++r) {
        for (int64_t i = 0; i < N; ++i) {
            const double *s = suns + 3 * r;
            int lit = 1;
            for (int64_t k = 0; k < ntri && lit; ++k) {
                if (k == i)
                    continue;
                const double *t = tri + 9 * k;
                if (ray_hits_triangle(x + 3 * i, s, ORC_T_LO, INFINITY, t, t + 3, t + 6))
                    lit = 0;
            }
            out[i + r * N] = (uint8_t)lit;
        }
    }
}
