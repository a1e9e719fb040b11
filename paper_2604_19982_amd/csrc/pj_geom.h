// pj_geom.h -- device geometry for the refinement kernels (gfx950).
//
// Facet-pair distance of two triangles (3DPipe Section 2.2, "Triangle-
// Triangle Distance Computation"): for disjoint triangles the minimum is
// attained by a vertex of one against the interior of the other, or by an
// edge pair, so it is the minimum of 6 vertex-plane distances (counted only
// where the vertex projects inside the other triangle) and 9 segment-segment
// distances.  Crossing triangles have distance 0 although all 15 candidates
// are positive, so an intersection test is added.
//
// Two arithmetic variants:
//   * FP32 (bulk): per-facet derived data ("records": corners, edges, unit
//     normal, inward edge normals, 1/|e|^2, hd, ph) are built once per facet
//     and reused against every facet of the other object; the crossing test
//     is the plane-straddle / line-interval test, and a crossing is reported
//     as *sure* only when the 15-candidate distance exceeds the guard band.
//   * FP64 (plain schedule, guard-band recheck, distances): the same reduced
//     distance formulation in double, plus an exact meet test whose
//     orientation signs are exact (floating-point filter, then an exact
//     expansion sum of the 48 partial products of the 4x4 determinant).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pj {

// --------------------------------------------------------------------------
// small vector helpers
// --------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
struct D3 {
    double x, y, z;
};

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)); }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return V3{fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x)};
}
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(a, fminf(b, c)); }
__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }

__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dotd(D3 a, D3 b) { return fma(a.z, b.z, fma(a.y, b.y, a.x * b.x)); }
__device__ __forceinline__ D3 crossd(D3 a, D3 b)
{
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// --------------------------------------------------------------------------
// FP32 facet record
// --------------------------------------------------------------------------
// 44 floats; the LDS copy is laid out as 11 float4.
struct Rec {
    V3 v0, v1, v2;     // corners (pair-local coordinates)
    V3 e0, e1, e2;     // e_i = v_{i+1} - v_i
    V3 n;              // unit normal, 0 for a (near-)degenerate facet
    float dn;          // n . v0
    V3 m0, m1, m2;     // inward in-plane edge normals n x e_i (0 if degenerate)
    float c0, c1, c2;  // m_i . v_i  (1 if degenerate so that "inside" never holds)
    float i0, i1, i2;  // 1 / |e_i|^2 (0 for a zero-length edge)
    float ee0, ee1, ee2;  // |e_i|^2
    float hd, ph;      // Hausdorff bounds of the facet (0 on the finest LoD)
    float ok;          // 1: well-shaped; 0: degenerate (no own-plane candidates, no sure crossing)
    float pad;
};
static_assert(sizeof(Rec) == 44 * 4, "record layout");

// The plane data (unit normal, inward edge normals and their offsets) are
// formed in FP64 from the float corners and rounded once, so their error does
// not grow for thin facets (long tube facets have corner angles near 1
// degree).  Only facets with (numerically) zero area are flagged degenerate;
// they still get correct distances through the segment candidates, and only
// their lower bound is dropped to 0.
__device__ __forceinline__ Rec make_rec(V3 a, V3 b, V3 c, float hd, float ph)
{
    Rec r;
    r.v0 = a;
    r.v1 = b;
    r.v2 = c;
    r.e0 = b - a;
    r.e1 = c - b;
    r.e2 = a - c;
    r.ee0 = dot(r.e0, r.e0);
    r.ee1 = dot(r.e1, r.e1);
    r.ee2 = dot(r.e2, r.e2);
    r.i0 = r.ee0 > 0.0f ? 1.0f / r.ee0 : 0.0f;
    r.i1 = r.ee1 > 0.0f ? 1.0f / r.ee1 : 0.0f;
    r.i2 = r.ee2 > 0.0f ? 1.0f / r.ee2 : 0.0f;
    D3 A{a.x, a.y, a.z}, B{b.x, b.y, b.z}, C{c.x, c.y, c.z};
    D3 E0 = B - A, E1 = C - B, E2 = A - C;
    D3 N = crossd(E0, C - A);
    double nn = dotd(N, N);
    double emax = fmax(dotd(E0, E0), fmax(dotd(E1, E1), dotd(E2, E2)));
    bool good = nn > 1e-24 * emax * emax;
    double inv = good ? 1.0 / sqrt(nn) : 0.0;
    D3 U{N.x * inv, N.y * inv, N.z * inv};
    D3 M0 = crossd(U, E0), M1 = crossd(U, E1), M2 = crossd(U, E2);
    r.n = V3{(float)U.x, (float)U.y, (float)U.z};
    r.dn = (float)dotd(U, A);
    r.m0 = V3{(float)M0.x, (float)M0.y, (float)M0.z};
    r.m1 = V3{(float)M1.x, (float)M1.y, (float)M1.z};
    r.m2 = V3{(float)M2.x, (float)M2.y, (float)M2.z};
    r.c0 = good ? (float)dotd(M0, A) : 1.0f;
    r.c1 = good ? (float)dotd(M1, B) : 1.0f;
    r.c2 = good ? (float)dotd(M2, C) : 1.0f;
    r.hd = hd;
    r.ph = ph;
    r.ok = good ? 1.0f : 0.0f;
    r.pad = 0.0f;
    return r;
}

// squared distance between segment (p, p + d1) and (q, q + d2); aa = |d1|^2,
// ia = 1/aa, ee = |d2|^2, ie = 1/ee, b = d1.d2, c = d1.(p - q),
// f = d2.(p - q).  The closest-parameter solve, then t from the clamped s,
// then s again from the clamped t; every result is a pair of points of the
// two segments, and the sequence ends at the true minimum (the last step can
// only move closer).
__device__ __forceinline__ float segseg2(V3 p, V3 d1, float aa, float ia, V3 q, V3 d2, float ee, float ie, float b,
                                         float c, float f)
{
    V3 r = p - q;
    float den = fmaf(aa, ee, -b * b);
    float num = fmaf(b, f, -c * ee);
    float s = clamp01(num * __builtin_amdgcn_rcpf(fmaxf(den, 1e-30f)));
    float t = clamp01(fmaf(b, s, f) * ie);
    s = clamp01(fmaf(b, t, -c) * ia);
    float wx = fmaf(s, d1.x, fmaf(-t, d2.x, r.x));
    float wy = fmaf(s, d1.y, fmaf(-t, d2.y, r.y));
    float wz = fmaf(s, d1.z, fmaf(-t, d2.z, r.z));
    return fmaf(wz, wz, fmaf(wy, wy, wx * wx));
}

// signed distance of p to the plane of R and whether p projects inside R
__device__ __forceinline__ float plane_cand2(const Rec &R, V3 p, float &h)
{
    h = dot(R.n, p) - R.dn;
    float s0 = dot(R.m0, p) - R.c0;
    float s1 = dot(R.m1, p) - R.c1;
    float s2 = dot(R.m2, p) - R.c2;
    return min3f(s0, s1, s2) >= 0.0f ? h * h : __builtin_inff();
}

// 1-D extent of triangle (p0,p1,p2) along direction L where it crosses the
// other plane; h_i are the corners' signed distances to that plane.
__device__ __forceinline__ void cross_interval(V3 L, V3 p0, V3 p1, V3 p2, float h0, float h1, float h2, float &lo,
                                               float &hi)
{
    float t0 = dot(L, p0), t1 = dot(L, p1), t2 = dot(L, p2);
    lo = __builtin_inff();
    hi = -__builtin_inff();
    if (h0 == 0.0f) { lo = fminf(lo, t0); hi = fmaxf(hi, t0); }
    if (h1 == 0.0f) { lo = fminf(lo, t1); hi = fmaxf(hi, t1); }
    if (h2 == 0.0f) { lo = fminf(lo, t2); hi = fmaxf(hi, t2); }
    if (h0 * h1 < 0.0f) { float x = t0 + (t1 - t0) * (h0 / (h0 - h1)); lo = fminf(lo, x); hi = fmaxf(hi, x); }
    if (h1 * h2 < 0.0f) { float x = t1 + (t2 - t1) * (h1 / (h1 - h2)); lo = fminf(lo, x); hi = fmaxf(hi, x); }
    if (h2 * h0 < 0.0f) { float x = t2 + (t0 - t2) * (h2 / (h2 - h0)); lo = fminf(lo, x); hi = fmaxf(hi, x); }
}

// Result of one FP32 facet pair.  The crossing test (both triangles straddle
// the other's plane and the crossing segments overlap on the planes' common
// line) decides d = 0 against d = the 15-candidate minimum.  Its FP32 form is
// taken twice: a loose one (plain signs) whose firing sets the lower estimate
// to 0, and a strict one (every sign and the overlap clear of their rounding
// error) that alone makes the upper estimate 0.  Between the two the pair is
// left open for the FP64 recheck (near-coplanar pairs whose plane distances
// are rounding noise land there).
struct Pair32 {
    float lo;   // lower estimate of the distance (0 if a crossing is possible)
    float hi;   // upper estimate (0 only for a certain crossing, else the 15-candidate minimum)
    bool sure;  // certain crossing, with the 15-candidate minimum above eps: the triangles meet
};

__device__ __forceinline__ Pair32 pair_f32(const Rec &A, const Rec &B, float eps)
{
    float best, ha0, ha1, ha2, hb0, hb1, hb2;
    best = plane_cand2(A, B.v0, hb0);
    best = fminf(best, plane_cand2(A, B.v1, hb1));
    best = fminf(best, plane_cand2(A, B.v2, hb2));
    best = fminf(best, plane_cand2(B, A.v0, ha0));
    best = fminf(best, plane_cand2(B, A.v1, ha1));
    best = fminf(best, plane_cand2(B, A.v2, ha2));
    // Edge pair (i, j): b = A.e_i . B.e_j, c = A.e_i . (A.v_i - B.v_j),
    // f = B.e_j . (A.v_i - B.v_j).  Walking the corners along the edges
    // (v_{k+1} = v_k + e_k) gives c(i, j+1) = c(i, j) - b(i, j) and
    // f(i+1, j) = f(i, j) + b(i, j), so only c(i, 0) and f(0, j) are dot
    // products.  A's edges are taken one at a time (few values live at once).
    float f0 = dot(B.e0, A.v0 - B.v0), f1 = dot(B.e1, A.v0 - B.v1), f2 = dot(B.e2, A.v0 - B.v2);
    {
        const float b0 = dot(A.e0, B.e0), b1 = dot(A.e0, B.e1), b2 = dot(A.e0, B.e2);
        const float c0 = dot(A.e0, A.v0 - B.v0), c1 = c0 - b0, c2 = c1 - b1;
        best = fminf(best, segseg2(A.v0, A.e0, A.ee0, A.i0, B.v0, B.e0, B.ee0, B.i0, b0, c0, f0));
        best = fminf(best, segseg2(A.v0, A.e0, A.ee0, A.i0, B.v1, B.e1, B.ee1, B.i1, b1, c1, f1));
        best = fminf(best, segseg2(A.v0, A.e0, A.ee0, A.i0, B.v2, B.e2, B.ee2, B.i2, b2, c2, f2));
        f0 += b0;
        f1 += b1;
        f2 += b2;
    }
    {
        const float b0 = dot(A.e1, B.e0), b1 = dot(A.e1, B.e1), b2 = dot(A.e1, B.e2);
        const float c0 = dot(A.e1, A.v1 - B.v0), c1 = c0 - b0, c2 = c1 - b1;
        best = fminf(best, segseg2(A.v1, A.e1, A.ee1, A.i1, B.v0, B.e0, B.ee0, B.i0, b0, c0, f0));
        best = fminf(best, segseg2(A.v1, A.e1, A.ee1, A.i1, B.v1, B.e1, B.ee1, B.i1, b1, c1, f1));
        best = fminf(best, segseg2(A.v1, A.e1, A.ee1, A.i1, B.v2, B.e2, B.ee2, B.i2, b2, c2, f2));
        f0 += b0;
        f1 += b1;
        f2 += b2;
    }
    {
        const float b0 = dot(A.e2, B.e0), b1 = dot(A.e2, B.e1), b2 = dot(A.e2, B.e2);
        const float c0 = dot(A.e2, A.v2 - B.v0), c1 = c0 - b0, c2 = c1 - b1;
        best = fminf(best, segseg2(A.v2, A.e2, A.ee2, A.i2, B.v0, B.e0, B.ee0, B.i0, b0, c0, f0));
        best = fminf(best, segseg2(A.v2, A.e2, A.ee2, A.i2, B.v1, B.e1, B.ee1, B.i1, b1, c1, f1));
        best = fminf(best, segseg2(A.v2, A.e2, A.ee2, A.i2, B.v2, B.e2, B.ee2, B.i2, b2, c2, f2));
    }
    Pair32 out;
    // hardware square root (about 1 ulp; the guard band is 2^-16 of the
    // pair's extent, far above it); a denormal square may flush to 0, which
    // only lowers the estimate of a distance far below the band
    const float d15 = __builtin_amdgcn_sqrtf(best);
    out.lo = d15;
    out.hi = d15;
    out.sure = false;
    // loose crossing test: each triangle strictly straddles the other's plane
    // by the FP32 signs
    const float ha_lo = min3f(ha0, ha1, ha2), ha_hi = max3f(ha0, ha1, ha2);
    const float hb_lo = min3f(hb0, hb1, hb2), hb_hi = max3f(hb0, hb1, hb2);
    if (ha_lo < 0.0f && ha_hi > 0.0f && hb_lo < 0.0f && hb_hi > 0.0f) {
        V3 L = cross(A.n, B.n);
        float alo, ahi, blo, bhi;
        cross_interval(L, A.v0, A.v1, A.v2, ha0, ha1, ha2, alo, ahi);
        cross_interval(L, B.v0, B.v1, B.v2, hb0, hb1, hb2, blo, bhi);
        if (fmaxf(alo, blo) <= fminf(ahi, bhi)) {
            out.lo = 0.0f;
            // Strict test.  A corner's plane distance is off the exact one by
            // less than eh: the unit normal and the offset are each rounded
            // once from FP64 (2^-24 relative) and the FP32 dot product adds a
            // few roundings of terms below sqrt(3) M, about 10 x 2^-24 M in
            // all, against eh = 2^-19 M.  Let the margin m be the smaller of
            // the largest distance on either side.  Each edge that changes
            // sign joins corners whose distances add to at least m, so with
            // m > 4 eh its crossing point moves by at most 2 eh / m of the
            // triangle's extent along L, and a middle corner that may sit on
            // either side moves the endpoint by at most 3 eh / m of it.  The
            // direction L (from two rounded normals) shifts positions by less
            // than 2^-21 M, under eh.
            const float eh = 0.125f * eps;
            const float ma = fminf(ha_hi, -ha_lo), mb = fminf(hb_hi, -hb_lo);
            if (ma > 4.0f * eh && mb > 4.0f * eh) {
                const float ta0 = dot(L, A.v0), ta1 = dot(L, A.v1), ta2 = dot(L, A.v2);
                const float tb0 = dot(L, B.v0), tb1 = dot(L, B.v1), tb2 = dot(L, B.v2);
                const float ea = 4.0f * eh * (max3f(ta0, ta1, ta2) - min3f(ta0, ta1, ta2)) / ma;
                const float eb = 4.0f * eh * (max3f(tb0, tb1, tb2) - min3f(tb0, tb1, tb2)) / mb;
                if (fmaxf(alo, blo) + (ea + eb + 2.0f * eh) < fminf(ahi, bhi)) {
                    out.hi = 0.0f;
                    out.sure = d15 > eps;
                }
            }
        }
    }
    return out;
}

// --------------------------------------------------------------------------
// Exact orientation signs (inputs: doubles holding float32 values)
// --------------------------------------------------------------------------
__device__ __forceinline__ void tsum(double a, double b, double &s, double &e)
{
    s = a + b;
    double z = s - a;
    e = (a - (s - z)) + (b - z);
}

// Exact sign of the sum of n doubles: running nonoverlapping expansion.
__device__ __noinline__ int exact_sign(double *t, int n)
{
    double ex[56];
    int len = 0;
    for (int k = 0; k < n; ++k) {
        double q = t[k];
        int w = 0;
        for (int i = 0; i < len; ++i) {
            double s, e;
            tsum(q, ex[i], s, e);
            q = s;
            if (e != 0.0) ex[w++] = e;
        }
        if (q != 0.0) ex[w++] = q;
        len = w;
    }
    if (len == 0) return 0;
    return ex[len - 1] > 0.0 ? 1 : -1;
}

// sign of det[a 1; b 1; c 1; d 1]; exact for float32-valued inputs.
__device__ __noinline__ int orient3d_slow(D3 a, D3 b, D3 c, D3 d)
{
    // det = sum over permutations (i j k l) of the rows' columns x,y,z,1:
    // expand as sum_{rows u<v<w} +-det3(u,v,w), det3 = sum_perm sgn * u_i v_j w_k.
    const D3 P[4] = {a, b, c, d};
    double t[48];
    int n = 0;
    const int tri[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int m = 0; m < 4; ++m) {
        double sg = (m & 1) ? 1.0 : -1.0;
        const D3 &u = P[tri[m][0]], &v = P[tri[m][1]], &w = P[tri[m][2]];
        double uu[3] = {u.x, u.y, u.z}, vv[3] = {v.x, v.y, v.z}, ww[3] = {w.x, w.y, w.z};
        const int pm[6][4] = {{0, 1, 2, 1}, {1, 2, 0, 1}, {2, 0, 1, 1}, {0, 2, 1, -1}, {2, 1, 0, -1}, {1, 0, 2, -1}};
        for (int q = 0; q < 6; ++q) {
            double p2 = uu[pm[q][0]] * vv[pm[q][1]];  // exact (two float32 factors)
            double h = p2 * ww[pm[q][2]];
            double l = fma(p2, ww[pm[q][2]], -h);
            double s = sg * (double)pm[q][3];
            t[n++] = s * h;
            t[n++] = s * l;
        }
    }
    return exact_sign(t, n);
}

__device__ __forceinline__ int orient3d(D3 a, D3 b, D3 c, D3 d)
{
    // error-bounded evaluation of the translated 3x3 form first
    double adx = a.x - d.x, ady = a.y - d.y, adz = a.z - d.z;
    double bdx = b.x - d.x, bdy = b.y - d.y, bdz = b.z - d.z;
    double cdx = c.x - d.x, cdy = c.y - d.y, cdz = c.z - d.z;
    double bc = bdy * cdz - bdz * cdy, ca = cdy * adz - cdz * ady, ab = ady * bdz - adz * bdy;
    double det = adx * bc + bdx * ca + cdx * ab;
    double perm = fabs(adx) * (fabs(bdy * cdz) + fabs(bdz * cdy)) + fabs(bdx) * (fabs(cdy * adz) + fabs(cdz * ady)) +
                  fabs(cdx) * (fabs(ady * bdz) + fabs(adz * bdy));
    double bound = 7.771561172376103e-16 * perm;  // (7 + 56 u) u, u = 2^-53
    // subtracting row d from rows a, b, c leaves the 4x4 determinant equal
    // to this translated 3x3 one
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient3d_slow(a, b, c, d);
}

// sign of det[a_i a_j 1; b_i b_j 1; c_i c_j 1]: six exact products.
__device__ __forceinline__ int orient2d(D3 a, D3 b, D3 c, int i, int j)
{
    const double A[3] = {a.x, a.y, a.z}, B[3] = {b.x, b.y, b.z}, C[3] = {c.x, c.y, c.z};
    double t[6] = {A[i] * B[j], -A[i] * C[j], -A[j] * B[i], A[j] * C[i], B[i] * C[j], -B[j] * C[i]};
    double quick = ((t[0] + t[1]) + (t[2] + t[3])) + (t[4] + t[5]);
    double mag = (fabs(t[0]) + fabs(t[1])) + (fabs(t[2]) + fabs(t[3])) + (fabs(t[4]) + fabs(t[5]));
    if (quick > 8.9e-16 * mag) return 1;
    if (-quick > 8.9e-16 * mag) return -1;
    return exact_sign(t, 6);
}

__device__ __forceinline__ double comp(D3 p, int i) { return i == 0 ? p.x : (i == 1 ? p.y : p.z); }

// closed segments meet in the (i, j) projection
__device__ __noinline__ bool seg_meet_2d(D3 p, D3 q, D3 a, D3 b, int i, int j)
{
    int o1 = orient2d(p, q, a, i, j), o2 = orient2d(p, q, b, i, j);
    int o3 = orient2d(a, b, p, i, j), o4 = orient2d(a, b, q, i, j);
    if (o1 * o2 < 0 && o3 * o4 < 0) return true;
    auto within = [&](D3 s, D3 t, D3 x) {
        return fmin(comp(s, i), comp(t, i)) <= comp(x, i) && comp(x, i) <= fmax(comp(s, i), comp(t, i)) &&
               fmin(comp(s, j), comp(t, j)) <= comp(x, j) && comp(x, j) <= fmax(comp(s, j), comp(t, j));
    };
    return (o1 == 0 && within(p, q, a)) || (o2 == 0 && within(p, q, b)) || (o3 == 0 && within(a, b, p)) ||
           (o4 == 0 && within(a, b, q));
}

// closed segment meets closed triangle in the (i, j) projection
__device__ __noinline__ bool seg_tri_meet_2d(D3 p, D3 q, D3 a, D3 b, D3 c, int i, int j)
{
    int o = orient2d(a, b, c, i, j);
    if (o != 0) {
        int s0 = orient2d(a, b, p, i, j) * o, s1 = orient2d(b, c, p, i, j) * o, s2 = orient2d(c, a, p, i, j) * o;
        if (s0 >= 0 && s1 >= 0 && s2 >= 0) return true;
    }
    return seg_meet_2d(p, q, a, b, i, j) || seg_meet_2d(p, q, b, c, i, j) || seg_meet_2d(p, q, c, a, i, j);
}

// coplanar point sets: some coordinate projection is one-to-one on their
// plane and the others only add meets, so require a meet in all three.
__device__ __noinline__ bool seg_meet_3d(D3 p, D3 q, D3 a, D3 b)
{
    if (orient3d(p, q, a, b) != 0) return false;
    return seg_meet_2d(p, q, a, b, 0, 1) && seg_meet_2d(p, q, a, b, 1, 2) && seg_meet_2d(p, q, a, b, 2, 0);
}

__device__ __noinline__ bool seg_tri_meet(D3 p, D3 q, D3 a, D3 b, D3 c)
{
    bool line = orient2d(a, b, c, 0, 1) == 0 && orient2d(a, b, c, 1, 2) == 0 && orient2d(a, b, c, 2, 0) == 0;
    if (line) return seg_meet_3d(p, q, a, b) || seg_meet_3d(p, q, b, c) || seg_meet_3d(p, q, c, a);
    int sp = orient3d(a, b, c, p), sq = orient3d(a, b, c, q);
    if (sp * sq > 0) return false;
    if (sp == 0 && sq == 0)
        return seg_tri_meet_2d(p, q, a, b, c, 0, 1) && seg_tri_meet_2d(p, q, a, b, c, 1, 2) &&
               seg_tri_meet_2d(p, q, a, b, c, 2, 0);
    int u = orient3d(p, q, a, b), v = orient3d(p, q, b, c), w = orient3d(p, q, c, a);
    return !((u > 0 || v > 0 || w > 0) && (u < 0 || v < 0 || w < 0));
}

// Exact meet test of closed triangles given as doubles holding float32 values.
__device__ __noinline__ bool tri_meet_exact(const D3 *A, const D3 *B)
{
    // each triangle must reach the other's plane (both sides or on it)
    int sa[3], sb[3];
    for (int k = 0; k < 3; ++k) sa[k] = orient3d(B[0], B[1], B[2], A[k]);
    if ((sa[0] > 0 && sa[1] > 0 && sa[2] > 0) || (sa[0] < 0 && sa[1] < 0 && sa[2] < 0)) return false;
    for (int k = 0; k < 3; ++k) sb[k] = orient3d(A[0], A[1], A[2], B[k]);
    if ((sb[0] > 0 && sb[1] > 0 && sb[2] > 0) || (sb[0] < 0 && sb[1] < 0 && sb[2] < 0)) return false;
    // an edge of one meets the other triangle
    for (int k = 0; k < 3; ++k)
        if (seg_tri_meet(A[k], A[(k + 1) % 3], B[0], B[1], B[2])) return true;
    for (int k = 0; k < 3; ++k)
        if (seg_tri_meet(B[k], B[(k + 1) % 3], A[0], A[1], A[2])) return true;
    return false;
}

// --------------------------------------------------------------------------
// FP64 facet distance (reduced formulation, corners only)
// --------------------------------------------------------------------------
__device__ __forceinline__ double segseg2_d(D3 p, D3 d1, D3 q, D3 d2)
{
    D3 r = p - q;
    double aa = dotd(d1, d1), ee = dotd(d2, d2), b = dotd(d1, d2), c = dotd(d1, r), f = dotd(d2, r);
    double den = aa * ee - b * b;
    double s = den > 0.0 ? fmin(fmax((b * f - c * ee) / den, 0.0), 1.0) : 0.0;
    double t = ee > 0.0 ? fmin(fmax((b * s + f) / ee, 0.0), 1.0) : 0.0;
    s = aa > 0.0 ? fmin(fmax((b * t - c) / aa, 0.0), 1.0) : 0.0;
    D3 w = D3{r.x + s * d1.x - t * d2.x, r.y + s * d1.y - t * d2.y, r.z + s * d1.z - t * d2.z};
    return dotd(w, w);
}

// squared plane distance of p to triangle T if p projects inside T, else inf
__device__ __forceinline__ double plane_cand2_d(const D3 *T, D3 n, double nn, D3 p)
{
    if (!(nn > 0.0)) return __builtin_inf();
    D3 e0 = T[1] - T[0], e1 = T[2] - T[1], e2 = T[0] - T[2];
    double s0 = dotd(crossd(e0, p - T[0]), n), s1 = dotd(crossd(e1, p - T[1]), n), s2 = dotd(crossd(e2, p - T[2]), n);
    if (s0 < 0.0 || s1 < 0.0 || s2 < 0.0) return __builtin_inf();
    double h = dotd(n, p - T[0]);
    return h * h / nn;
}

__device__ __forceinline__ double d15_f64(const D3 *A, const D3 *B)
{
    D3 nA = crossd(A[1] - A[0], A[2] - A[0]), nB = crossd(B[1] - B[0], B[2] - B[0]);
    double nnA = dotd(nA, nA), nnB = dotd(nB, nB);
    double best = __builtin_inf();
    for (int k = 0; k < 3; ++k) {
        best = fmin(best, plane_cand2_d(A, nA, nnA, B[k]));
        best = fmin(best, plane_cand2_d(B, nB, nnB, A[k]));
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            best = fmin(best, segseg2_d(A[i], A[(i + 1) % 3] - A[i], B[j], B[(j + 1) % 3] - B[j]));
    return sqrt(best);
}

// FP64 facet distance with the exact meet test; sets hit when they meet.
__device__ __forceinline__ double pair_f64(const D3 *A, const D3 *B, bool &hit)
{
    hit = false;
    bool boxes = true;
    {
        double al = fmin(A[0].x, fmin(A[1].x, A[2].x)), ah = fmax(A[0].x, fmax(A[1].x, A[2].x));
        double bl = fmin(B[0].x, fmin(B[1].x, B[2].x)), bh = fmax(B[0].x, fmax(B[1].x, B[2].x));
        boxes = boxes && !(ah < bl || bh < al);
        al = fmin(A[0].y, fmin(A[1].y, A[2].y)); ah = fmax(A[0].y, fmax(A[1].y, A[2].y));
        bl = fmin(B[0].y, fmin(B[1].y, B[2].y)); bh = fmax(B[0].y, fmax(B[1].y, B[2].y));
        boxes = boxes && !(ah < bl || bh < al);
        al = fmin(A[0].z, fmin(A[1].z, A[2].z)); ah = fmax(A[0].z, fmax(A[1].z, A[2].z));
        bl = fmin(B[0].z, fmin(B[1].z, B[2].z)); bh = fmax(B[0].z, fmax(B[1].z, B[2].z));
        boxes = boxes && !(ah < bl || bh < al);
    }
    if (boxes && tri_meet_exact(A, B)) {
        hit = true;
        return 0.0;
    }
    return d15_f64(A, B);
}

// --------------------------------------------------------------------------
// wave64 reductions (DPP/permute through the compiler's cross-lane ops)
// --------------------------------------------------------------------------
__device__ __forceinline__ float wave_min(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_or(int v)
{
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// float <-> ordered uint for atomicMin on non-negative values
__device__ __forceinline__ unsigned fbits(float x) { return __float_as_uint(x); }

}  // namespace pj
