/*
 * oracle.c -- plain, slow, obviously-correct FP64 CPU reference for the
 * polyhedral spatial join of "3DPipe" (arXiv 2604.19982).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * bench's CPU-baseline leg load this library.  It shares no code, header,
 * helper or table with the GPU library; the two are independent.
 *
 * What it computes (every function cites the passage it follows):
 *   - the polyhedron distance d(P1,P2): minimum Euclidean distance between
 *     points of the two surfaces (Section 2.1, definition of d);
 *   - the triangle-triangle distance as the minimum of 6 point-triangle and 9
 *     segment-segment distances (Section 2.2, "Triangle-Triangle Distance
 *     Computation"), plus an exact test for crossing triangles, which those
 *     15 candidates miss (their distance is 0 although every candidate is
 *     positive);
 *   - the facet-level bounds of Eq. (1) and Eq. (2) (Section 2.1), and
 *     reference values of the per-facet Hausdorff bound hd(f',P) and proxy
 *     Hausdorff bound ph(P,f') that make them valid (the paper defers their
 *     definitions to TDBase; the readings used here are stated at each
 *     function);
 *   - object MBBs and vertex anchors (Section 2.1, "Object and Voxel
 *     Centers"; anchors are always surface vertices here).
 *
 * Inputs are float32 coordinates; every computation promotes them to double
 * (exact).  Exact orientation signs use floating-point expansion arithmetic
 * (error-free TwoSum and FMA-based TwoProduct, after Shewchuk 1997).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* A mesh set, object-major; see meshgen for the layout. */
typedef struct {
    int32_t n_objects, n_lods;
    const float *verts;        /* [V*3] */
    const int64_t *vert_begin; /* [n] */
    const int32_t *vert_count; /* [n] */
    const int32_t *tris;       /* [T*3] local vertex indices */
    const int64_t *tri_begin;  /* [n*L] */
    const int32_t *tri_count;  /* [n*L] */
    const int32_t *parent;     /* [T] parent index at LoD-1, -1 at LoD 0 */
} om_set;

/* ------------------------------------------------------------------------
 * Exact signs by expansion arithmetic.
 * ---------------------------------------------------------------------- */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

/* Add b to the nonoverlapping expansion e[0..n) (increasing magnitude),
 * dropping zero components.  Returns the new length. */
static int grow(double *e, int n, double b)
{
    double q = b;
    int m = 0;
    for (int i = 0; i < n; i++) {
        double s, h;
        two_sum(q, e[i], &s, &h);
        if (h != 0.0) e[m++] = h;
        q = s;
    }
    if (q != 0.0) e[m++] = q;
    return m;
}

/* exact sign of sum_k terms[k] */
static int sign_of_sum(const double *terms, int n)
{
    double e[64];
    int m = 0;
    for (int k = 0; k < n; k++) m = grow(e, m, terms[k]);
    if (m == 0) return 0;
    return e[m - 1] > 0.0 ? 1 : (e[m - 1] < 0.0 ? -1 : 0);
}

/* x*y*z for float-valued doubles as an exact two-term sum. */
static void triple(double x, double y, double z, double sgn, double *hi, double *lo)
{
    double p = x * y;            /* exact: 24+24 significant bits */
    double h = p * z;
    double l = fma(p, z, -h);    /* exact error of the rounded product */
    *hi = sgn * h;
    *lo = sgn * l;
}

/* Sign of the 4x4 determinant |a 1; b 1; c 1; d 1| (rows), expanded into its
 * 24 signed triple products, each split exactly into two doubles. */
int oracle_orient3d(const double *a, const double *b, const double *c, const double *d)
{
    const double *P[4] = {a, b, c, d};
    /* cofactor expansion along the column of ones:
     * det = -det3(b,c,d) + det3(a,c,d) - det3(a,b,d) + det3(a,b,c) */
    static const int rows[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    static const double outer[4] = {-1.0, 1.0, -1.0, 1.0};
    /* det3(p,q,r) = p.(q x r): six terms p_i q_j r_k with the sign of (ijk) */
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const double psign[6] = {1.0, -1.0, -1.0, 1.0, 1.0, -1.0};
    double t[48];
    int n = 0;
    for (int m = 0; m < 4; m++) {
        const double *p = P[rows[m][0]], *q = P[rows[m][1]], *r = P[rows[m][2]];
        for (int k = 0; k < 6; k++) {
            triple(p[perm[k][0]], q[perm[k][1]], r[perm[k][2]], outer[m] * psign[k], &t[n], &t[n + 1]);
            n += 2;
        }
    }
    return sign_of_sum(t, n);
}

/* Sign of |a_i a_j 1; b_i b_j 1; c_i c_j 1| for the projection onto axes (i,j). */
int oracle_orient2d(const double *a, const double *b, const double *c, int i, int j)
{
    double t[6];
    t[0] = a[i] * b[j];
    t[1] = -a[i] * c[j];
    t[2] = -a[j] * b[i];
    t[3] = a[j] * c[i];
    t[4] = b[i] * c[j];
    t[5] = -b[j] * c[i];
    return sign_of_sum(t, 6);
}

/* ------------------------------------------------------------------------
 * Exact intersection of closed triangles (any degeneracy).
 *
 * Two closed triangles meet iff an edge of one meets the other closed
 * triangle: with non-coplanar planes the common part lies on the planes'
 * line and its end points lie on edges; with coplanar triangles either the
 * boundaries cross or one contains the other (then its edges lie inside).
 * ---------------------------------------------------------------------- */
static int in_box2(const double *p, const double *q, const double *x, int i, int j)
{
    return fmin(p[i], q[i]) <= x[i] && x[i] <= fmax(p[i], q[i]) &&
           fmin(p[j], q[j]) <= x[j] && x[j] <= fmax(p[j], q[j]);
}

/* closed segments pq and ab in the projection (i,j) */
static int seg_seg2(const double *p, const double *q, const double *a, const double *b, int i, int j)
{
    int d1 = oracle_orient2d(p, q, a, i, j), d2 = oracle_orient2d(p, q, b, i, j);
    int d3 = oracle_orient2d(a, b, p, i, j), d4 = oracle_orient2d(a, b, q, i, j);
    if (d1 * d2 < 0 && d3 * d4 < 0) return 1;
    if (d1 == 0 && in_box2(p, q, a, i, j)) return 1;
    if (d2 == 0 && in_box2(p, q, b, i, j)) return 1;
    if (d3 == 0 && in_box2(a, b, p, i, j)) return 1;
    if (d4 == 0 && in_box2(a, b, q, i, j)) return 1;
    return 0;
}

/* closed segment pq and closed triangle abc in the projection (i,j) */
static int seg_tri2(const double *p, const double *q, const double *a, const double *b, const double *c, int i, int j)
{
    int o = oracle_orient2d(a, b, c, i, j);
    if (o != 0) {
        int s1 = oracle_orient2d(a, b, p, i, j);
        int s2 = oracle_orient2d(b, c, p, i, j);
        int s3 = oracle_orient2d(c, a, p, i, j);
        if (s1 * o >= 0 && s2 * o >= 0 && s3 * o >= 0) return 1;
    }
    return seg_seg2(p, q, a, b, i, j) || seg_seg2(p, q, b, c, i, j) || seg_seg2(p, q, c, a, i, j);
}

/* Coplanar point sets: at least one coordinate projection is injective on
 * their affine hull and the others can only add false meets, so a meet in 3D
 * is a meet in all three projections. */
static int seg_seg3(const double *p, const double *q, const double *a, const double *b)
{
    if (oracle_orient3d(p, q, a, b) != 0) return 0;
    return seg_seg2(p, q, a, b, 0, 1) && seg_seg2(p, q, a, b, 1, 2) && seg_seg2(p, q, a, b, 0, 2);
}

static int collinear3(const double *a, const double *b, const double *c)
{
    return oracle_orient2d(a, b, c, 0, 1) == 0 && oracle_orient2d(a, b, c, 1, 2) == 0 &&
           oracle_orient2d(a, b, c, 0, 2) == 0;
}

static int seg_tri3(const double *p, const double *q, const double *a, const double *b, const double *c)
{
    if (collinear3(a, b, c))  /* the triangle is the union of its edges */
        return seg_seg3(p, q, a, b) || seg_seg3(p, q, b, c) || seg_seg3(p, q, c, a);
    int sp = oracle_orient3d(a, b, c, p), sq = oracle_orient3d(a, b, c, q);
    if (sp * sq > 0) return 0;
    if (sp == 0 && sq == 0)
        return seg_tri2(p, q, a, b, c, 0, 1) && seg_tri2(p, q, a, b, c, 1, 2) && seg_tri2(p, q, a, b, c, 0, 2);
    /* the segment meets the plane in one point: does the line pass through
     * the closed triangle?  (three edge orientations of one sign, or zero) */
    int s1 = oracle_orient3d(p, q, a, b), s2 = oracle_orient3d(p, q, b, c), s3 = oracle_orient3d(p, q, c, a);
    int pos = s1 > 0 || s2 > 0 || s3 > 0;
    int neg = s1 < 0 || s2 < 0 || s3 < 0;
    return !(pos && neg);
}

/* t1, t2: 3 corners x 3 coordinates (double, exact copies of float32) */
int oracle_tri_tri_intersect_d(const double *t1, const double *t2)
{
    for (int k = 0; k < 3; k++) {  /* closed boxes apart => apart */
        double lo1 = fmin(t1[k], fmin(t1[3 + k], t1[6 + k])), hi1 = fmax(t1[k], fmax(t1[3 + k], t1[6 + k]));
        double lo2 = fmin(t2[k], fmin(t2[3 + k], t2[6 + k])), hi2 = fmax(t2[k], fmax(t2[3 + k], t2[6 + k]));
        if (hi1 < lo2 || hi2 < lo1) return 0;
    }
    for (int e = 0; e < 3; e++) {
        const double *p = t1 + 3 * e, *q = t1 + 3 * ((e + 1) % 3);
        if (seg_tri3(p, q, t2, t2 + 3, t2 + 6)) return 1;
    }
    for (int e = 0; e < 3; e++) {
        const double *p = t2 + 3 * e, *q = t2 + 3 * ((e + 1) % 3);
        if (seg_tri3(p, q, t1, t1 + 3, t1 + 6)) return 1;
    }
    return 0;
}

int oracle_tri_tri_intersect(const float *t1f, const float *t2f)
{
    double t1[9], t2[9];
    for (int k = 0; k < 9; k++) { t1[k] = t1f[k]; t2[k] = t2f[k]; }
    return oracle_tri_tri_intersect_d(t1, t2);
}

/* ------------------------------------------------------------------------
 * Distances (FP64).
 * ---------------------------------------------------------------------- */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }

/* squared distance from p to the closed segment ab */
static double pt_seg_d2(const double *p, const double *a, const double *b)
{
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double L = dot3(ab, ab);
    double t = 0.0;
    if (L > 0.0) {
        t = dot3(ap, ab) / L;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double w[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
    return dot3(w, w);
}

/* Distance from p to the closed triangle abc.  The minimiser of
 * |a + s(b-a) + t(c-a) - p|^2 over the triangle is the unconstrained one
 * (normal equations) when that is feasible; otherwise the convex problem's
 * minimum is on the boundary, i.e. on one of the three edges. */
double oracle_pt_tri(const double *p, const double *a, const double *b, const double *c)
{
    double e0[3], e1[3], w[3];
    sub3(b, a, e0);
    sub3(c, a, e1);
    sub3(p, a, w);
    double A = dot3(e0, e0), B = dot3(e0, e1), C = dot3(e1, e1);
    double u = dot3(w, e0), v = dot3(w, e1);
    double det = A * C - B * B;
    if (det > 0.0) {
        double s = (C * u - B * v) / det;
        double t = (A * v - B * u) / det;
        if (s >= 0.0 && t >= 0.0 && s + t <= 1.0) {
            double r[3] = {w[0] - s * e0[0] - t * e1[0], w[1] - s * e0[1] - t * e1[1], w[2] - s * e0[2] - t * e1[2]};
            return sqrt(dot3(r, r));
        }
    }
    double d = pt_seg_d2(p, a, b);
    d = fmin(d, pt_seg_d2(p, b, c));
    d = fmin(d, pt_seg_d2(p, c, a));
    return sqrt(d);
}

/* Distance between closed segments p0p1 and q0q1: the unconstrained
 * minimiser of |p0 + s d1 - q0 - t d2|^2 if it lies in [0,1]^2, else the
 * smallest of the four end-point-to-segment distances (the minimum of the
 * convex problem over the square is then on its boundary). */
double oracle_seg_seg(const double *p0, const double *p1, const double *q0, const double *q1)
{
    double d1[3], d2[3], r[3];
    sub3(p1, p0, d1);
    sub3(q1, q0, d2);
    sub3(p0, q0, r);
    double a = dot3(d1, d1), b = dot3(d1, d2), e = dot3(d2, d2);
    double c = dot3(d1, r), f = dot3(d2, r);
    double det = a * e - b * b;
    if (det > 0.0) {
        double s = (b * f - c * e) / det;
        double t = (a * f - b * c) / det;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
            double w[3] = {r[0] + s * d1[0] - t * d2[0], r[1] + s * d1[1] - t * d2[1], r[2] + s * d1[2] - t * d2[2]};
            return sqrt(dot3(w, w));
        }
    }
    double d = pt_seg_d2(p0, q0, q1);
    d = fmin(d, pt_seg_d2(p1, q0, q1));
    d = fmin(d, pt_seg_d2(q0, p0, p1));
    d = fmin(d, pt_seg_d2(q1, p0, p1));
    return sqrt(d);
}

/* The 15-candidate minimum of Section 2.2 (6 vertex-triangle, 9 edge-edge). */
double oracle_tri_tri_d15(const double *t1, const double *t2)
{
    double d = DBL_MAX;
    for (int k = 0; k < 3; k++) {
        d = fmin(d, oracle_pt_tri(t1 + 3 * k, t2, t2 + 3, t2 + 6));
        d = fmin(d, oracle_pt_tri(t2 + 3 * k, t1, t1 + 3, t1 + 6));
    }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            d = fmin(d, oracle_seg_seg(t1 + 3 * i, t1 + 3 * ((i + 1) % 3), t2 + 3 * j, t2 + 3 * ((j + 1) % 3)));
    return d;
}

/* Triangle distance: 0 for meeting triangles, else the 15-candidate minimum. */
double oracle_tri_tri_dist(const float *t1f, const float *t2f, int *hit)
{
    double t1[9], t2[9];
    for (int k = 0; k < 9; k++) { t1[k] = t1f[k]; t2[k] = t2f[k]; }
    int h = oracle_tri_tri_intersect_d(t1, t2);
    if (hit) *hit = h;
    return h ? 0.0 : oracle_tri_tri_d15(t1, t2);
}

/* ------------------------------------------------------------------------
 * Object-level helpers.
 * ---------------------------------------------------------------------- */
static void facet_corners(const om_set *M, int obj, int lod, int f, double *out)
{
    const int64_t tb = M->tri_begin[(int64_t)obj * M->n_lods + lod];
    const int32_t *t = M->tris + 3 * (tb + f);
    const float *v = M->verts + 3 * M->vert_begin[obj];
    for (int k = 0; k < 3; k++)
        for (int c = 0; c < 3; c++) out[3 * k + c] = (double)v[3 * t[k] + c];
}

static double *load_facets(const om_set *M, int obj, int lod, int *nf)
{
    int n = M->tri_count[(int64_t)obj * M->n_lods + lod];
    double *F = (double *)malloc(sizeof(double) * 9 * (size_t)(n > 0 ? n : 1));
    for (int f = 0; f < n; f++) facet_corners(M, obj, lod, f, F + 9 * f);
    *nf = n;
    return F;
}

static void facet_boxes(const double *F, int n, double *box)
{
    for (int f = 0; f < n; f++)
        for (int k = 0; k < 3; k++) {
            const double *t = F + 9 * f;
            box[6 * f + k] = fmin(t[k], fmin(t[3 + k], t[6 + k]));
            box[6 * f + 3 + k] = fmax(t[k], fmax(t[3 + k], t[6 + k]));
        }
}

static int cmp_bp(const void *x, const void *y)
{
    const double a = *(const double *)x, b = *(const double *)y;
    if (a < b) return -1;
    if (a > b) return 1;
    const int64_t i = *(const int64_t *)((const char *)x + sizeof(double));
    const int64_t j = *(const int64_t *)((const char *)y + sizeof(double));
    return (i > j) - (i < j);
}

/* d(r,s) at the given LoDs: minimum over all facet pairs (Section 2.1).
 * mode 0 ("brute"): every facet pair.
 * mode 1 ("culled"): a facet pair whose boxes are at least the current best
 * apart cannot lower the minimum and is skipped; the first meeting pair ends
 * the scan (d = 0).  Both modes return the same minimum. */
static double object_distance_counted(const om_set *R, int r, int lod_r, const om_set *S, int s, int lod_s, int mode,
                                      int *hit, int64_t *evals);

double oracle_object_distance(const om_set *R, int r, int lod_r, const om_set *S, int s, int lod_s, int mode, int *hit)
{
    return object_distance_counted(R, r, lod_r, S, s, lod_s, mode, hit, NULL);
}

/* The same scan, also counting the facet pairs whose distance (or meet
 * test) it evaluated, when evals is not NULL (instrumentation only). */
static double object_distance_counted(const om_set *R, int r, int lod_r, const om_set *S, int s, int lod_s, int mode,
                                      int *hit, int64_t *evals)
{
    int64_t ne = 0;
    int nr, ns;
    double *FR = load_facets(R, r, lod_r, &nr);
    double *FS = load_facets(S, s, lod_s, &ns);
    double best = DBL_MAX;
    int h = 0;
    if (mode == 0) {
        for (int i = 0; i < nr && !h; i++)
            for (int j = 0; j < ns; j++) {
                ne++;
                if (oracle_tri_tri_intersect_d(FR + 9 * i, FS + 9 * j)) { h = 1; best = 0.0; break; }
                best = fmin(best, oracle_tri_tri_d15(FR + 9 * i, FS + 9 * j));
            }
    } else {
        /* Facets are visited in blocks of OB consecutive facets; a block pair
         * (and then a facet pair) whose boxes are at least the current best
         * apart is skipped.  Block pairs are taken in ascending box-gap order
         * so that small distances are found early.  Exact: a skipped pair's
         * distance is not below its box gap. */
        enum { OB = 32 };
        double *BR = (double *)malloc(sizeof(double) * 6 * (size_t)(nr > 0 ? nr : 1));
        double *BS = (double *)malloc(sizeof(double) * 6 * (size_t)(ns > 0 ? ns : 1));
        facet_boxes(FR, nr, BR);
        facet_boxes(FS, ns, BS);
        int nbr = (nr + OB - 1) / OB, nbs = (ns + OB - 1) / OB;
        double *KR = (double *)malloc(sizeof(double) * 6 * (size_t)(nbr > 0 ? nbr : 1));
        double *KS = (double *)malloc(sizeof(double) * 6 * (size_t)(nbs > 0 ? nbs : 1));
        for (int b = 0; b < nbr; b++)
            for (int k = 0; k < 3; k++) {
                KR[6 * b + k] = INFINITY;
                KR[6 * b + 3 + k] = -INFINITY;
                for (int i = b * OB; i < nr && i < (b + 1) * OB; i++) {
                    KR[6 * b + k] = fmin(KR[6 * b + k], BR[6 * i + k]);
                    KR[6 * b + 3 + k] = fmax(KR[6 * b + 3 + k], BR[6 * i + 3 + k]);
                }
            }
        for (int b = 0; b < nbs; b++)
            for (int k = 0; k < 3; k++) {
                KS[6 * b + k] = INFINITY;
                KS[6 * b + 3 + k] = -INFINITY;
                for (int j = b * OB; j < ns && j < (b + 1) * OB; j++) {
                    KS[6 * b + k] = fmin(KS[6 * b + k], BS[6 * j + k]);
                    KS[6 * b + 3 + k] = fmax(KS[6 * b + 3 + k], BS[6 * j + 3 + k]);
                }
            }
        int64_t nbp = (int64_t)nbr * nbs;
        struct bp { double g2; int64_t id; } *order = (struct bp *)malloc(sizeof(struct bp) * (size_t)(nbp > 0 ? nbp : 1));
        for (int64_t q = 0; q < nbp; q++) {
            const double *a = KR + 6 * (q / nbs), *b = KS + 6 * (q % nbs);
            double g2 = 0.0;
            for (int k = 0; k < 3; k++) {
                double g = fmax(0.0, fmax(b[k] - a[3 + k], a[k] - b[3 + k]));
                g2 += g * g;
            }
            order[q].g2 = g2;
            order[q].id = q;
        }
        qsort(order, (size_t)nbp, sizeof(struct bp), cmp_bp);
        double best2 = DBL_MAX;
        for (int64_t q = 0; q < nbp && !h; q++) {
            if (order[q].g2 >= best2) break;
            int b1 = (int)(order[q].id / nbs), b2 = (int)(order[q].id % nbs);
            for (int i = b1 * OB; i < nr && i < (b1 + 1) * OB && !h; i++) {
                const double *bi = BR + 6 * i;
                for (int j = b2 * OB; j < ns && j < (b2 + 1) * OB; j++) {
                    const double *bj = BS + 6 * j;
                    double g2 = 0.0;
                    for (int k = 0; k < 3; k++) {
                        double g = fmax(0.0, fmax(bj[k] - bi[3 + k], bi[k] - bj[3 + k]));
                        g2 += g * g;
                    }
                    if (g2 >= best2) continue;
                    ne++;
                    if (g2 == 0.0 && oracle_tri_tri_intersect_d(FR + 9 * i, FS + 9 * j)) { h = 1; best = 0.0; break; }
                    double d = oracle_tri_tri_d15(FR + 9 * i, FS + 9 * j);
                    if (d < best) { best = d; best2 = d * d; }
                }
            }
        }
        free(order);
        free(KR);
        free(KS);
        free(BR);
        free(BS);
    }
    free(FR);
    free(FS);
    if (hit) *hit = h;
    if (evals) *evals = ne;
    return (nr == 0 || ns == 0) ? INFINITY : best;
}

/* Batched finest-LoD (lod < 0) or fixed-LoD distances for a list of pairs. */
void oracle_pair_distances(const om_set *R, const om_set *S, int64_t n, const int32_t *rr, const int32_t *ss,
                           int lod, int mode, int threads, double *d, int8_t *hit)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < n; k++) {
        int lr = lod < 0 ? R->n_lods - 1 : lod;
        int ls = lod < 0 ? S->n_lods - 1 : lod;
        int h = 0;
        d[k] = oracle_object_distance(R, rr[k], lr, S, ss[k], ls, mode, &h);
        if (hit) hit[k] = (int8_t)h;
    }
}

/* oracle_pair_distances plus the facet pairs evaluated per object pair. */
void oracle_pair_distances_counted(const om_set *R, const om_set *S, int64_t n, const int32_t *rr, const int32_t *ss,
                                   int lod, int mode, int threads, double *d, int8_t *hit, int64_t *evals)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < n; k++) {
        int lr = lod < 0 ? R->n_lods - 1 : lod;
        int ls = lod < 0 ? S->n_lods - 1 : lod;
        int h = 0;
        d[k] = object_distance_counted(R, rr[k], lr, S, ss[k], ls, mode, &h, evals + k);
        if (hit) hit[k] = (int8_t)h;
    }
}

/* MBB over the vertices referenced by the finest LoD: 6 doubles lo[3], hi[3]. */
void oracle_mbb(const om_set *M, int obj, double *out)
{
    int L = M->n_lods - 1;
    int nf = M->tri_count[(int64_t)obj * M->n_lods + L];
    for (int k = 0; k < 3; k++) { out[k] = INFINITY; out[3 + k] = -INFINITY; }
    for (int f = 0; f < nf; f++) {
        double t[9];
        facet_corners(M, obj, L, f, t);
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < 3; k++) {
                out[k] = fmin(out[k], t[3 * c + k]);
                out[3 + k] = fmax(out[3 + k], t[3 * c + k]);
            }
    }
}

/* Object anchor (Section 2.1, "Object and Voxel Centers"): the surface vertex
 * closest to the MBB centre (ties: lowest vertex index).  A vertex is used
 * even when the centre lies inside the solid, because an interior point is
 * not an upper bound of the *surface* distance. */
void oracle_anchor(const om_set *M, int obj, double *out)
{
    double box[6];
    oracle_mbb(M, obj, box);
    double c[3] = {0.5 * (box[0] + box[3]), 0.5 * (box[1] + box[4]), 0.5 * (box[2] + box[5])};
    int L = M->n_lods - 1;
    int nf = M->tri_count[(int64_t)obj * M->n_lods + L];
    const int32_t *t = M->tris + 3 * M->tri_begin[(int64_t)obj * M->n_lods + L];
    const float *v = M->verts + 3 * M->vert_begin[obj];
    double best = INFINITY;
    int bi = -1;
    for (int k = 0; k < 3 * nf; k++) {
        int vi = t[k];
        double dx = v[3 * vi] - c[0], dy = v[3 * vi + 1] - c[1], dz = v[3 * vi + 2] - c[2];
        double d = dx * dx + dy * dy + dz * dz;
        if (d < best || (d == best && vi < bi)) { best = d; bi = vi; }
    }
    for (int k = 0; k < 3; k++) out[k] = bi >= 0 ? v[3 * bi + k] : NAN;
}

void oracle_mbb_all(const om_set *M, double *out6, double *anchor3)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int i = 0; i < M->n_objects; i++) {
        oracle_mbb(M, i, out6 + 6 * (int64_t)i);
        if (anchor3) oracle_anchor(M, i, anchor3 + 3 * (int64_t)i);
    }
}

/* ------------------------------------------------------------------------
 * Per-facet Hausdorff bounds (Section 2.1, "Facet-Level Hausdorff Bounds").
 *
 * Each finest facet g has one ancestor at every coarser LoD (follow the
 * parent map).  For a facet f' of LoD lod < L-1:
 *   ph(P,f') = max over finest facets g with ancestor f', over the corners v
 *              of g, of dist(v, f').  Every point y of P lies on some g, and
 *              dist(., f') is convex, so dist(y, anc(g)) <= ph(anc(g)); this
 *              is the property Eq. (2) needs.
 *   hd(f',P) = max over the barycentric grid points x of f' with m
 *              subdivisions per edge of min over those g of dist(x, g), plus
 *              the longest grid edge (|f' edge| / m).  dist(., P) is
 *              1-Lipschitz and every point of f' is within one grid edge of
 *              a grid point, so hd >= max_{x in f'} dist(x, P), which is what
 *              Eq. (1) needs.  A facet with no finest descendant takes the
 *              minimum over every finest facet of the object instead (the
 *              minimum over an empty set would be +inf, not 0).
 *   A facet with no descendant gets ph = 0: Eq. (2) needs ph only for the
 *   facets that are some surface point's ancestor, and a smaller lower bound
 *   from an extra facet pair is still a lower bound.
 * Both are 0 on the finest LoD.
 * ---------------------------------------------------------------------- */
int oracle_hd_ph(const om_set *M, int obj, int lod, int m, double *hd, double *ph)
{
    int L = M->n_lods;
    int64_t base = (int64_t)obj * L;
    int nc = M->tri_count[base + lod];
    if (lod == L - 1) {
        for (int f = 0; f < nc; f++) { hd[f] = 0.0; ph[f] = 0.0; }
        return 0;
    }
    int nfine = M->tri_count[base + L - 1];
    int *anc = (int *)malloc(sizeof(int) * (size_t)(nfine > 0 ? nfine : 1));
    for (int g = 0; g < nfine; g++) {
        int a = g;
        for (int l = L - 1; l > lod; l--) {
            a = M->parent[M->tri_begin[base + l] + a];
            if (a < 0) { free(anc); return -1; }
        }
        anc[g] = a;
    }
    for (int f = 0; f < nc; f++) { hd[f] = 0.0; ph[f] = 0.0; }
    double t[9], g9[9];
    /* ph */
    for (int g = 0; g < nfine; g++) {
        facet_corners(M, obj, lod, anc[g], t);
        facet_corners(M, obj, L - 1, g, g9);
        for (int c = 0; c < 3; c++) {
            double d = oracle_pt_tri(g9 + 3 * c, t, t + 3, t + 6);
            if (d > ph[anc[g]]) ph[anc[g]] = d;
        }
    }
    /* hd: descendants grouped by ancestor (counting sort) */
    int *cnt = (int *)calloc((size_t)nc + 1, sizeof(int));
    int *lst = (int *)malloc(sizeof(int) * (size_t)(nfine > 0 ? nfine : 1));
    for (int g = 0; g < nfine; g++) cnt[anc[g] + 1]++;
    for (int f = 0; f < nc; f++) cnt[f + 1] += cnt[f];
    int *pos = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    for (int f = 0; f < nc; f++) pos[f] = cnt[f];
    for (int g = 0; g < nfine; g++) lst[pos[anc[g]]++] = g;
    double *desc = (double *)malloc(sizeof(double) * 9 * (size_t)(nfine > 0 ? nfine : 1));
    for (int f = 0; f < nc; f++) {
        facet_corners(M, obj, lod, f, t);
        int nd = cnt[f + 1] - cnt[f];
        /* A facet that no finest facet descends from is bounded against the
         * whole finest mesh P: dist(x, P) is what Eq. (1) needs, and the
         * descendants are only a subset of P chosen to make the bound
         * tighter.  With an empty P the bound is +inf. */
        const int whole = nd == 0;
        if (whole) nd = nfine;
        for (int q = 0; q < nd; q++) facet_corners(M, obj, L - 1, whole ? q : lst[cnt[f] + q], desc + 9 * q);
        double worst = nd ? 0.0 : INFINITY;
        for (int i = 0; i <= m; i++)
            for (int j = 0; i + j <= m; j++) {
                int k = m - i - j;
                double x[3];
                for (int c = 0; c < 3; c++) x[c] = ((double)i * t[c] + (double)j * t[3 + c] + (double)k * t[6 + c]) / (double)m;
                double best = nd ? DBL_MAX : INFINITY;
                for (int q = 0; q < nd; q++) {
                    const double *gg = desc + 9 * q;
                    best = fmin(best, oracle_pt_tri(x, gg, gg + 3, gg + 6));
                }
                if (best > worst) worst = best;
            }
        double e = 0.0;
        for (int c = 0; c < 3; c++) {
            double u[3];
            sub3(t + 3 * ((c + 1) % 3), t + 3 * c, u);
            e = fmax(e, sqrt(dot3(u, u)));
        }
        hd[f] = worst + e / (double)m;
    }
    free(desc);
    free(pos);
    free(lst);
    free(cnt);
    free(anc);
    return 0;
}

/* Object bounds at one LoD from Eq. (1) and Eq. (2), every facet pair:
 *   lb = min max(0, d(f1',f2') - ph1 - ph2),  ub = min d(f1',f2') + hd1 + hd2. */
void oracle_lod_bounds(const om_set *R, int r, const om_set *S, int s, int lod, const double *hdr, const double *phr,
                       const double *hds, const double *phs, double *lb, double *ub)
{
    int nr, ns;
    double *FR = load_facets(R, r, lod, &nr);
    double *FS = load_facets(S, s, lod, &ns);
    double L = DBL_MAX, U = DBL_MAX;
    for (int i = 0; i < nr; i++)
        for (int j = 0; j < ns; j++) {
            double d = oracle_tri_tri_intersect_d(FR + 9 * i, FS + 9 * j) ? 0.0 : oracle_tri_tri_d15(FR + 9 * i, FS + 9 * j);
            L = fmin(L, fmax(0.0, d - phr[i] - phs[j]));
            U = fmin(U, d + hdr[i] + hds[j]);
        }
    free(FR);
    free(FS);
    *lb = L;
    *ub = U;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Triangle distances and exact meet flags for n pairs (float32 corners). */
void oracle_tri_tri_batch(int64_t n, const float *t1, const float *t2, double *d, int8_t *hit, int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t k = 0; k < n; k++) {
        int h = 0;
        d[k] = oracle_tri_tri_dist(t1 + 9 * k, t2 + 9 * k, &h);
        hit[k] = (int8_t)h;
    }
}
