// pj_kernels.hip -- HIP kernels for gfx950: ingest (boxes, anchors, hd/ph),
// MBB filter, FP32 persistent tile refinement, FP64 refinement (tiled and
// one-workgroup-per-pair), and a facet-pair entry used by tests.
#include <mutex>

#include "pj_geom.h"
#include "pj_internal.h"

namespace pj {

constexpr float kInf = __builtin_inff();

// A dispatch counts its grid in work-items per dimension with 32 bits: a
// larger grid would wrap and run only part of the work, so launchers check
// it, and the kernels over long lists stride over them with a grid capped at
// 2^16 workgroups (at least 8x what the 256 CUs hold at once, so the cap
// costs no parallelism and lists of ordinary size already take the stride).
inline bool grid_fits(int64_t blocks, int threads) { return blocks * (int64_t)threads <= 0xffffffffLL; }
constexpr int64_t kStrideBlocks = int64_t(1) << 16;
#define PJ_GRID_CHECK(blocks, threads) \
    do { \
        if (!grid_fits((blocks), (threads))) return hipErrorInvalidConfiguration; \
    } while (0)

__device__ __forceinline__ float block_min256(float v, float *sh)
{
    v = wave_min(v);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    float r = fminf(fminf(sh[0], sh[1]), fminf(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float block_max256(float v, float *sh)
{
    v = wave_max(v);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    float r = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ D3 ld3d(const float *v, int i)
{
    return D3{(double)v[3 * i], (double)v[3 * i + 1], (double)v[3 * i + 2]};
}
__device__ __forceinline__ V3 ld3f(const float *v, int i) { return V3{v[3 * i], v[3 * i + 1], v[3 * i + 2]}; }

// index of the last k with off[k] <= j (off ascending, off[0] = 0)
__device__ __forceinline__ int find_seg(const int64_t *off, int n, int64_t j)
{
    int lo = 0, hi = n;  // off[n] is the total
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Ingest: object MBB over the finest LoD's corners, then the anchor: the
// corner closest to the MBB centre (ties: lowest vertex index).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_boxes(MeshDev m, float *box, float *anchor)
{
    __shared__ float sh[4];
    __shared__ int shi[4];
    const int obj = blockIdx.x;
    const int64_t k = (int64_t)obj * m.L + (m.L - 1);
    const int nt = m.tcnt[k];
    const int32_t *t = m.tris + 3 * m.tbeg[k];
    const float *v = m.verts + 3 * m.vbeg[obj];
    float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    for (int q = threadIdx.x; q < 3 * nt; q += 256) {
        int vi = t[q];
        for (int c = 0; c < 3; ++c) {
            float x = v[3 * vi + c];
            lo[c] = fminf(lo[c], x);
            hi[c] = fmaxf(hi[c], x);
        }
    }
    float B[6];
    for (int c = 0; c < 3; ++c) {
        B[c] = block_min256(lo[c], sh);
        B[3 + c] = -block_min256(-hi[c], sh);
    }
    float cx = 0.5f * (B[0] + B[3]), cy = 0.5f * (B[1] + B[4]), cz = 0.5f * (B[2] + B[5]);
    float bd = kInf;
    int bi = 0x7fffffff;
    for (int q = threadIdx.x; q < 3 * nt; q += 256) {
        int vi = t[q];
        float dx = v[3 * vi] - cx, dy = v[3 * vi + 1] - cy, dz = v[3 * vi + 2] - cz;
        float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (d < bd || (d == bd && vi < bi)) {
            bd = d;
            bi = vi;
        }
    }
    float best = block_min256(bd, sh);
    int cand = (bd == best) ? bi : 0x7fffffff;
    for (int o = 32; o > 0; o >>= 1) cand = min(cand, __shfl_xor(cand, o, 64));
    if ((threadIdx.x & 63) == 0) shi[threadIdx.x >> 6] = cand;
    __syncthreads();
    if (threadIdx.x == 0) {
        int w = min(min(shi[0], shi[1]), min(shi[2], shi[3]));
        for (int c = 0; c < 6; ++c) box[6 * obj + c] = B[c];
        for (int c = 0; c < 3; ++c) anchor[3 * obj + c] = (nt > 0) ? v[3 * w + c] : __builtin_nanf("");
    }
}

hipError_t launch_boxes(const MeshDev &m, float *box, float *anchor, hipStream_t st)
{
    if (m.n == 0) return hipSuccess;
    PJ_GRID_CHECK(m.n, 256);
    hipLaunchKernelGGL(k_boxes, dim3(m.n), dim3(256), 0, st, m, box, anchor);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ingest: per-facet Hausdorff bounds (FP64, rounded up to float).
// ---------------------------------------------------------------------------
__device__ double pt_seg2_d(D3 p, D3 a, D3 b)
{
    D3 ab = b - a, ap = p - a;
    double L = dotd(ab, ab);
    double t = L > 0.0 ? fmin(fmax(dotd(ap, ab) / L, 0.0), 1.0) : 0.0;
    D3 w = D3{ap.x - t * ab.x, ap.y - t * ab.y, ap.z - t * ab.z};
    return dotd(w, w);
}

// distance from p to the closed triangle abc (projection if it falls inside,
// else the nearest of the three edges)
__device__ double pt_tri_d(D3 p, D3 a, D3 b, D3 c)
{
    D3 n = crossd(b - a, c - a);
    double nn = dotd(n, n);
    if (nn > 0.0) {
        double s0 = dotd(crossd(b - a, p - a), n), s1 = dotd(crossd(c - b, p - b), n), s2 = dotd(crossd(a - c, p - c), n);
        if (s0 >= 0.0 && s1 >= 0.0 && s2 >= 0.0) return fabs(dotd(n, p - a)) / sqrt(nn);
    }
    return sqrt(fmin(pt_seg2_d(p, a, b), fmin(pt_seg2_d(p, b, c), pt_seg2_d(p, c, a))));
}

// FP64 value -> float rounded up, after a relative and absolute safety margin
// for the FP64 evaluation error (coordinates up to magnitude M).
__device__ __forceinline__ float round_up_bound(double x, double M)
{
    double y = x * (1.0 + 1e-12) + 1e-13 * M;
    return __double2float_ru(y);
}

__device__ __forceinline__ double mag3(D3 a) { return fmax(fabs(a.x), fmax(fabs(a.y), fabs(a.z))); }

// ph(P, f'): for every finest facet g, max over its corners of the distance
// to its ancestor at each coarser LoD, max-reduced into that ancestor.
__device__ __forceinline__ void ph_job(const MeshDev &m, float2 *hdph, const int32_t *parent, const int64_t *job_off,
                                       const int64_t j)
{
    const int obj = find_seg(job_off, m.n, j);
    const int g = (int)(j - job_off[obj]);
    const int L = m.L;
    const int64_t base = (int64_t)obj * L;
    const float *v = m.verts + 3 * m.vbeg[obj];
    const int32_t *tg = m.tris + 3 * (m.tbeg[base + L - 1] + g);
    D3 G[3] = {ld3d(v, tg[0]), ld3d(v, tg[1]), ld3d(v, tg[2])};
    int a = g;
    for (int l = L - 1; l > 0; --l) {
        a = parent[m.tbeg[base + l] + a];
        const int32_t *ta = m.tris + 3 * (m.tbeg[base + l - 1] + a);
        D3 A0 = ld3d(v, ta[0]), A1 = ld3d(v, ta[1]), A2 = ld3d(v, ta[2]);
        double d = fmax(pt_tri_d(G[0], A0, A1, A2), fmax(pt_tri_d(G[1], A0, A1, A2), pt_tri_d(G[2], A0, A1, A2)));
        double M = fmax(fmax(mag3(G[0]), fmax(mag3(G[1]), mag3(G[2]))), fmax(mag3(A0), fmax(mag3(A1), mag3(A2))));
        float val = round_up_bound(d, M);
        atomicMax(reinterpret_cast<unsigned *>(&hdph[m.hpbeg[base + l - 1] + a].y), __float_as_uint(val));
    }
}

__global__ __launch_bounds__(256) void k_ph(MeshDev m, float2 *hdph, const int32_t *parent, const int64_t *job_off,
                                             int64_t n_total)
{
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n_total; j += (int64_t)gridDim.x * 256)
        ph_job(m, hdph, parent, job_off, j);
}

hipError_t launch_ph(const MeshDev &m, float2 *hdph, const int32_t *parent, const int64_t *job_off, int64_t n_total,
                     hipStream_t st)
{
    if (n_total == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n_total + 255) / 256, kStrideBlocks);
    hipLaunchKernelGGL(k_ph, dim3((unsigned)blocks), dim3(256), 0, st, m, hdph, parent, job_off, n_total);
    return hipGetLastError();
}

// hd(f', P): one wave per coarse facet; lane = barycentric grid point
// x = (i a + j b + k c) / msub; value = max_x min_g dist(x, g) over the
// facet's finest descendants g (every finest facet of the object when it has
// none), plus the longest grid edge.
__device__ __forceinline__ void hd_job(const MeshDev &m, float2 *hdph, const int64_t *job_off, const int64_t *desc_base,
                                       const int32_t *desc_off, const int32_t *desc_list, const int lod, const int msub,
                                       const int64_t j)
{
    const int obj = find_seg(job_off, m.n, j);
    const int f = (int)(j - job_off[obj]);
    const int L = m.L;
    const int64_t base = (int64_t)obj * L;
    const float *v = m.verts + 3 * m.vbeg[obj];
    const int32_t *tf = m.tris + 3 * (m.tbeg[base + lod] + f);
    D3 A = ld3d(v, tf[0]), B = ld3d(v, tf[1]), C = ld3d(v, tf[2]);
    int lane = threadIdx.x;
    int npts = (msub + 1) * (msub + 2) / 2;
    double worst = 0.0;
    if (lane < npts) {
        int i = 0, r = lane;
        while (r > msub - i) {
            r -= msub - i + 1;
            ++i;
        }
        int jj = r, kk = msub - i - jj;
        double inv = 1.0 / msub;
        D3 x{(i * A.x + jj * B.x + kk * C.x) * inv, (i * A.y + jj * B.y + kk * C.y) * inv,
             (i * A.z + jj * B.z + kk * C.z) * inv};
        const int64_t db = desc_base[base + lod];
        const int32_t d0 = desc_off[db + f], d1 = desc_off[db + f + 1];
        const int32_t *tfine = m.tris + 3 * m.tbeg[base + L - 1];
        double best = __builtin_inf();
        if (d1 > d0) {
            for (int q = d0; q < d1; ++q) {
                const int32_t *tg = tfine + 3 * desc_list[q];
                best = fmin(best, pt_tri_d(x, ld3d(v, tg[0]), ld3d(v, tg[1]), ld3d(v, tg[2])));
            }
        } else {
            // no finest facet descends from f: bound it against the whole
            // finest mesh (dist(x, P) is what Eq. (1) needs; the descendants
            // are only the subset that makes it cheap); +inf if P is empty
            const int nfine = m.tcnt[base + L - 1];
            for (int q = 0; q < nfine; ++q) {
                const int32_t *tg = tfine + 3 * q;
                best = fmin(best, pt_tri_d(x, ld3d(v, tg[0]), ld3d(v, tg[1]), ld3d(v, tg[2])));
            }
        }
        worst = best;
    }
    for (int o = 32; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o, 64));
    if (lane == 0) {
        D3 e0 = B - A, e1 = C - B, e2 = A - C;
        double emax = sqrt(fmax(dotd(e0, e0), fmax(dotd(e1, e1), dotd(e2, e2))));
        double M = fmax(mag3(A), fmax(mag3(B), mag3(C))) + worst;
        hdph[m.hpbeg[base + lod] + f].x = round_up_bound(worst + emax / msub, M);
    }
}

// one wave per facet job, striding over the jobs when they outnumber the grid
__global__ __launch_bounds__(64) void k_hd(MeshDev m, float2 *hdph, const int64_t *job_off, int64_t n_jobs,
                                           const int64_t *desc_base, const int32_t *desc_off,
                                           const int32_t *desc_list, int lod, int msub)
{
    for (int64_t j = blockIdx.x; j < n_jobs; j += gridDim.x)
        hd_job(m, hdph, job_off, desc_base, desc_off, desc_list, lod, msub, j);
}

hipError_t launch_hd(const MeshDev &m, float2 *hdph, const int64_t *job_off, int64_t n_jobs, const int64_t *desc_base,
                     const int32_t *desc_off, const int32_t *desc_list, int lod, int msub, hipStream_t st)
{
    if (n_jobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hd, dim3((unsigned)std::min<int64_t>(n_jobs, kStrideBlocks)), dim3(64), 0, st, m, hdph, job_off,
                       n_jobs, desc_base, desc_off, desc_list, lod, msub);
    return hipGetLastError();
}

// per (object, LoD): max hd and max ph (features of the LoD model)
__global__ __launch_bounds__(256) void k_lodmax(MeshDev m, float2 *lodmax)
{
    __shared__ float sh[4];
    const int64_t k = blockIdx.x;
    const int lod = (int)(k % m.L);
    float a = 0.0f, b = 0.0f;
    if (lod < m.L - 1) {
        const int64_t hb = m.hpbeg[k];
        const int n = m.tcnt[k];
        for (int q = threadIdx.x; q < n; q += 256) {
            float2 h = m.hdph[hb + q];
            a = fmaxf(a, h.x);
            b = fmaxf(b, h.y);
        }
    }
    a = block_max256(a, sh);
    b = block_max256(b, sh);
    if (threadIdx.x == 0) lodmax[k] = make_float2(a, b);
}

// Block records: for each run of 64 consecutive facets of an (object, LoD),
// the exact float box of their corners and their largest hd and ph.
__device__ __forceinline__ void block_rec(const MeshDev &m, float4 *blk, const int64_t *blk_off, const int64_t j)
{
    const int k = find_seg(blk_off, m.n * m.L, j);  // (object, LoD) index
    const int obj = k / m.L, lod = k % m.L;
    const int b = (int)(j - blk_off[k]);
    const int nf = m.tcnt[k];
    const int32_t *t = m.tris + 3 * m.tbeg[k];
    const float *v = m.verts + 3 * m.vbeg[obj];
    const int64_t hb = m.hpbeg[k];
    float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf}, hd = 0.0f, ph = 0.0f;
    for (int f = 64 * b; f < min(nf, 64 * b + 64); ++f) {
        for (int c = 0; c < 3; ++c) {
            const int vi = t[3 * f + c];
            for (int q = 0; q < 3; ++q) {
                lo[q] = fminf(lo[q], v[3 * vi + q]);
                hi[q] = fmaxf(hi[q], v[3 * vi + q]);
            }
        }
        if (hb >= 0) {
            hd = fmaxf(hd, m.hdph[hb + f].x);
            ph = fmaxf(ph, m.hdph[hb + f].y);
        }
    }
    (void)lod;
    blk[2 * j] = make_float4(lo[0], lo[1], lo[2], hd);
    blk[2 * j + 1] = make_float4(hi[0], hi[1], hi[2], ph);
}

__global__ __launch_bounds__(256) void k_blocks(MeshDev m, float4 *blk, const int64_t *blk_off, int64_t n_blocks)
{
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n_blocks; j += (int64_t)gridDim.x * 256)
        block_rec(m, blk, blk_off, j);
}

hipError_t launch_blocks(const MeshDev &m, float4 *blk, const int64_t *blk_off, int64_t n_blocks, hipStream_t st)
{
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_blocks, dim3((unsigned)std::min<int64_t>((n_blocks + 255) / 256, kStrideBlocks)), dim3(256), 0,
                       st, m, blk, blk_off, n_blocks);
    return hipGetLastError();
}

hipError_t launch_lodmax(const MeshDev &m, float2 *lodmax, hipStream_t st)
{
    if (m.n == 0) return hipSuccess;
    PJ_GRID_CHECK((int64_t)m.n * m.L, 256);
    hipLaunchKernelGGL(k_lodmax, dim3((unsigned)((int64_t)m.n * m.L)), dim3(256), 0, st, m, lodmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MBB filter (within-tau): every (r, s) whose box gap is <= tau survives.
// Count pass -> exclusive scan of block counts -> write pass (each block
// writes its survivors contiguously, in (thread, s) order).
// ---------------------------------------------------------------------------
constexpr int FILT_R = kFiltR, FILT_S = kFiltS;

__global__ __launch_bounds__(256) void k_filter(const float *boxR, const float *ancR, int nR, const float *boxS,
                                                 const float *ancS, int nS, float tau2, int32_t *blk_count,
                                                 const int64_t *blk_off, int32_t *cr, int32_t *cs, float *clb,
                                                 float *cub, int write_pass)
{
    __shared__ float sb[FILT_S * 9];
    __shared__ int scnt[256];
    const int r = blockIdx.x * FILT_R + threadIdx.x;
    const int s0 = blockIdx.y * FILT_S;
    const int ns = min(FILT_S, nS - s0);
    for (int q = threadIdx.x; q < ns; q += 256) {
        for (int c = 0; c < 6; ++c) sb[q * 9 + c] = boxS[6 * (int64_t)(s0 + q) + c];
        for (int c = 0; c < 3; ++c) sb[q * 9 + 6 + c] = ancS[3 * (int64_t)(s0 + q) + c];
    }
    __syncthreads();
    float b[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
    if (r < nR)
        for (int c = 0; c < 6; ++c) b[c] = boxR[6 * (int64_t)r + c];
    int count = 0;
    for (int q = 0; q < ns; ++q) {
        const float *x = sb + q * 9;
        float gx = fmaxf(0.0f, fmaxf(x[0] - b[3], b[0] - x[3]));
        float gy = fmaxf(0.0f, fmaxf(x[1] - b[4], b[1] - x[4]));
        float gz = fmaxf(0.0f, fmaxf(x[2] - b[5], b[2] - x[5]));
        float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
        count += (g2 <= tau2) ? 1 : 0;
    }
    const int blk = blockIdx.x * gridDim.y + blockIdx.y;
    if (!write_pass) {
        scnt[threadIdx.x] = count;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) scnt[threadIdx.x] += scnt[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) blk_count[blk] = scnt[0];
        return;
    }
    // block exclusive scan of the thread counts (Hillis-Steele in LDS)
    scnt[threadIdx.x] = count;
    __syncthreads();
    for (int st = 1; st < 256; st <<= 1) {
        int add = threadIdx.x >= st ? scnt[threadIdx.x - st] : 0;
        __syncthreads();
        scnt[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t pos = blk_off[blk] + scnt[threadIdx.x] - count;
    if (count == 0) return;
    float ax = ancR[3 * (int64_t)r], ay = ancR[3 * (int64_t)r + 1], az = ancR[3 * (int64_t)r + 2];
    for (int q = 0; q < ns; ++q) {
        const float *x = sb + q * 9;
        float gx = fmaxf(0.0f, fmaxf(x[0] - b[3], b[0] - x[3]));
        float gy = fmaxf(0.0f, fmaxf(x[1] - b[4], b[1] - x[4]));
        float gz = fmaxf(0.0f, fmaxf(x[2] - b[5], b[2] - x[5]));
        float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
        if (g2 <= tau2) {
            float dx = x[6] - ax, dy = x[7] - ay, dz = x[8] - az;
            cr[pos] = r;
            cs[pos] = s0 + q;
            clb[pos] = __builtin_sqrtf(g2) * (1.0f - 0x1p-20f);
            cub[pos] = __builtin_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) * (1.0f + 0x1p-20f);
            ++pos;
        }
    }
}

hipError_t launch_filter(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS, int nS,
                         float tau2, int32_t *blk_count, int64_t *blk_off, int64_t *total, int32_t *cr, int32_t *cs,
                         float *clb, float *cub, int write_pass, hipStream_t st)
{
    (void)total;
    if (nR == 0 || nS == 0) return hipSuccess;
    dim3 grid((nR + FILT_R - 1) / FILT_R, (nS + FILT_S - 1) / FILT_S);
    PJ_GRID_CHECK(grid.x, 256);
    hipLaunchKernelGGL(k_filter, grid, dim3(256), 0, st, boxR, ancR, nR, boxS, ancS, nS, tau2, blk_count, blk_off, cr,
                       cs, clb, cub, write_pass);
    return hipGetLastError();
}

// MBB filter by an x sweep (large sets).  S is held sorted by box xmin
// (boxes and anchors in that order, with the original ids); R is visited in
// its own x order so that neighbouring threads search overlapping windows.
// Thread t takes r = rord[t] and scans the S boxes whose xmin lies in
// [r.xmin - w_lo, r.xmax + w_hi]; the window is widened so that every s the
// all-pairs test would keep is inside it, and each s in it gets exactly that
// test.  Count pass -> block totals; write pass -> block scan + positions.
__device__ __forceinline__ int lower_bound_f(const float *xs, int n, float v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (xs[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_filter_sweep(const float *boxR, const float *ancR, const int32_t *rord,
                                                      int nR, const float *sbox, const float *sanc,
                                                      const int32_t *sid, const float *sxs, int nS, float tau2,
                                                      float w_lo, float w_hi, int32_t *blk_count,
                                                      const int64_t *blk_off, int32_t *cr, int32_t *cs, float *clb,
                                                      float *cub, int write_pass)
{
    __shared__ int scnt[256];
    const int t = blockIdx.x * 256 + threadIdx.x;
    int r = -1;
    float b[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
    int j0 = 0, j1 = 0;
    if (t < nR) {
        r = rord[t];
        for (int c = 0; c < 6; ++c) b[c] = boxR[6 * (int64_t)r + c];
        j0 = lower_bound_f(sxs, nS, b[0] - w_lo);
        j1 = lower_bound_f(sxs, nS, b[3] + w_hi);
        // xs[j1] >= b[3] + w_hi: include equal keys at the upper end
        while (j1 < nS && sxs[j1] <= b[3] + w_hi) ++j1;
    }
    int count = 0;
    for (int j = j0; j < j1; ++j) {
        const float *x = sbox + 6 * (int64_t)j;
        float gx = fmaxf(0.0f, fmaxf(x[0] - b[3], b[0] - x[3]));
        float gy = fmaxf(0.0f, fmaxf(x[1] - b[4], b[1] - x[4]));
        float gz = fmaxf(0.0f, fmaxf(x[2] - b[5], b[2] - x[5]));
        float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
        count += (g2 <= tau2) ? 1 : 0;
    }
    if (!write_pass) {
        scnt[threadIdx.x] = count;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) scnt[threadIdx.x] += scnt[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) blk_count[blockIdx.x] = scnt[0];
        return;
    }
    scnt[threadIdx.x] = count;
    __syncthreads();
    for (int st = 1; st < 256; st <<= 1) {
        int add = threadIdx.x >= st ? scnt[threadIdx.x - st] : 0;
        __syncthreads();
        scnt[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t pos = blk_off[blockIdx.x] + scnt[threadIdx.x] - count;
    if (count == 0) return;
    const float ax = ancR[3 * (int64_t)r], ay = ancR[3 * (int64_t)r + 1], az = ancR[3 * (int64_t)r + 2];
    for (int j = j0; j < j1; ++j) {
        const float *x = sbox + 6 * (int64_t)j;
        float gx = fmaxf(0.0f, fmaxf(x[0] - b[3], b[0] - x[3]));
        float gy = fmaxf(0.0f, fmaxf(x[1] - b[4], b[1] - x[4]));
        float gz = fmaxf(0.0f, fmaxf(x[2] - b[5], b[2] - x[5]));
        float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
        if (g2 <= tau2) {
            const float *y = sanc + 3 * (int64_t)j;
            float dx = y[0] - ax, dy = y[1] - ay, dz = y[2] - az;
            cr[pos] = r;
            cs[pos] = sid[j];
            clb[pos] = __builtin_sqrtf(g2) * (1.0f - 0x1p-20f);
            cub[pos] = __builtin_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) * (1.0f + 0x1p-20f);
            ++pos;
        }
    }
}

hipError_t launch_filter_sweep(const float *boxR, const float *ancR, const int32_t *rord, int nR, const float *sbox,
                               const float *sanc, const int32_t *sid, const float *sxs, int nS, float tau2,
                               float w_lo, float w_hi, int32_t *blk_count, const int64_t *blk_off, int32_t *cr,
                               int32_t *cs, float *clb, float *cub, int write_pass, hipStream_t st)
{
    if (nR == 0 || nS == 0) return hipSuccess;
    PJ_GRID_CHECK((nR + 255) / 256, 256);
    hipLaunchKernelGGL(k_filter_sweep, dim3((nR + 255) / 256), dim3(256), 0, st, boxR, ancR, rord, nR, sbox, sanc,
                       sid, sxs, nS, tau2, w_lo, w_hi, blk_count, blk_off, cr, cs, clb, cub, write_pass);
    return hipGetLastError();
}

// single-workgroup exclusive scan of int32 counts into int64 offsets
__global__ __launch_bounds__(1024) void k_scan(const int32_t *in, int64_t *out, int64_t *total, int n)
{
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int base = 0; base < n; base += 1024) {
        int i = base + threadIdx.x;
        int64_t x = i < n ? in[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int st = 1; st < 1024; st <<= 1) {
            int64_t add = threadIdx.x >= st ? sh[threadIdx.x - st] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) out[i] = carry + sh[threadIdx.x] - x;
        int64_t blk_total = sh[1023];
        __syncthreads();
        carry += blk_total;
    }
    if (threadIdx.x == 0) *total = carry;
}

hipError_t launch_scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t *total, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, in, out, total, n);
    return hipGetLastError();
}

// Exclusive scan of long int32 arrays (grid cell counts): blocks of 4096
// scanned in LDS with their totals, the totals scanned by one block, then
// the block offsets added.  out has n + 1 entries (out[n] = total).
constexpr int kScanTile = 4096;

__global__ __launch_bounds__(1024) void k_scan_tiles(const int32_t *in, int64_t *out, int64_t *tile_sum, int64_t n)
{
    __shared__ int64_t sh[1024];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
    int64_t v[4], t = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        t += v[j];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int st = 1; st < 1024; st <<= 1) {
        const int64_t add = threadIdx.x >= st ? sh[threadIdx.x - st] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = sh[threadIdx.x] - t;
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 1023) tile_sum[blockIdx.x] = sh[1023];
}

__global__ __launch_bounds__(1024) void k_scan_sums(int64_t *tile_sum, int ntiles, int64_t *total)
{
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int64_t x = i < ntiles ? tile_sum[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int st = 1; st < 1024; st <<= 1) {
            const int64_t add = threadIdx.x >= st ? sh[threadIdx.x - st] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ntiles) tile_sum[i] = carry + sh[threadIdx.x] - x;
        const int64_t bt = sh[1023];
        __syncthreads();
        carry += bt;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int64_t *out, const int64_t *tile_sum, int64_t n, const int64_t *total)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = i < n ? out[i] + tile_sum[i / kScanTile] : *total;
}

hipError_t launch_scan_large(const int32_t *in, int64_t *out, int64_t *total, int64_t n, hipStream_t st)
{
    // tile sums live after out[n] (the caller sizes out for n + 1 + n / 4096 + 1 entries)
    const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles > kStrideBlocks) return hipErrorInvalidValue;
    int64_t *tile_sum = out + n + 1;
    if (ntiles > 0) {
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(1024), 0, st, in, out, tile_sum, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, tile_sum, (int)ntiles, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)std::min<int64_t>((n + 256) / 256, kStrideBlocks)), dim3(256), 0,
                       st, out, tile_sum, n, total);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Refinement outputs
// ---------------------------------------------------------------------------
// Per-round initialisation (a plain kernel, so that a captured graph
// replays it): item results to +inf, A-block cursors to 0, workgroup slots to
// -1.  The item and tile counts are read from the round's counter block
// ([6] items, [1] tiles), so one graph serves every round size.
__global__ void k_init_round(ItemOut *out, const int32_t *ctr, int32_t *slots, int nslots, int32_t *cur)
{
    const int ni = ctr[6], nt = ctr[1];
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ni; i += stride)
        out[i] = ItemOut{0x7f800000u, 0x7f800000u, 0, 0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += stride) cur[i] = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += stride) slots[i] = -1;
}

hipError_t launch_init_round(ItemOut *out, const int32_t *ctr, int32_t *slots, int nslots, int32_t *cur,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_init_round, dim3(256), dim3(256), 0, st, out, ctr, slots, nslots, cur);
    return hipGetLastError();
}

__global__ void k_init_out64(ItemOut64 *out, int n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = ItemOut64{0x7ff0000000000000ull, 0x7ff0000000000000ull, 0, 0};
}

hipError_t launch_init_out64(ItemOut64 *out, int n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_out64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, kStrideBlocks)), dim3(256), 0, st,
                       out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 refinement: persistent single-wave workgroups pull tiles from a queue.
// A tile = the A facets of one (pair, LoD) item, taken in register blocks of
// 64*P (P per lane) that any wave may claim, x a range of facets of object B,
// streamed through LDS 64 at a time (each lane builds one record; all lanes
// then read every record by broadcast).  Per lane running minima of lb and
// ub (Eq. (2), Eq. (1)) are reduced across the wave with cross-lane min and
// merged into the item by atomicMin.
// ---------------------------------------------------------------------------
struct FacetSrc {
    const int32_t *tris;
    const float *verts;
    const float2 *hdph;  // nullptr on the finest LoD
    const float4 *blk;   // block records of this (object, LoD)
    const uint8_t *vlab;               // voxel of each facet (null without voxels)
    const unsigned long long *bmask;   // voxels of each block record
    int n;
};

__device__ __forceinline__ FacetSrc facet_src(const MeshDev &M, int obj, int lod)
{
    const int64_t k = (int64_t)obj * M.L + lod;
    FacetSrc s;
    s.tris = M.tris + 3 * M.tbeg[k];
    s.verts = M.verts + 3 * M.vbeg[obj];
    const int64_t hb = M.hpbeg[k];
    s.hdph = hb >= 0 ? M.hdph + hb : nullptr;
    s.blk = M.blk + 2 * M.bkbeg[k];
    s.vlab = M.vlab ? M.vlab + M.lbeg[k] : nullptr;
    s.bmask = M.bmask ? M.bmask + M.bkbeg[k] : nullptr;
    s.n = M.tcnt[k];
    return s;
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long v)
{
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    for (int o = 32; o > 0; o >>= 1) {
        lo |= (unsigned)__shfl_xor((int)lo, o, 64);
        hi |= (unsigned)__shfl_xor((int)hi, o, 64);
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ Rec load_rec(const FacetSrc &s, int f, V3 o)
{
    const int32_t i0 = s.tris[3 * f], i1 = s.tris[3 * f + 1], i2 = s.tris[3 * f + 2];
    V3 a = ld3f(s.verts, i0) - o, b = ld3f(s.verts, i1) - o, c = ld3f(s.verts, i2) - o;
    float2 h = s.hdph ? s.hdph[f] : make_float2(0.0f, 0.0f);
    return make_rec(a, b, c, h.x, h.y);
}

// One tile.  Every branch below depends only on wave-uniform values (tile
// and item fields loaded through a uniform index, readfirstlane'd flags), so
// the compiler emits scalar control flow and the wave never splits.
//
// Chunk culling: a chunk of 64 B facets is one precomputed block record (box
// of the corners, max hd, max ph); the A side of the tile is the union of its
// P block records.  With g the box gap (a lower bound of every pair's true
// distance, evaluated in FP64 and rounded down), every pair in the chunk has
// FP32 distance >= g - eps, hence ub >= g - eps and
// lb >= g - eps - phmax_A - phmax_B.  The chunk is skipped when neither bound
// can matter:
//   ub: g - eps > min(current item ub, tau - eps)   (within: cannot confirm)
//   lb: lbLow   > min(current item lb, tau + eps)   (within: cannot block a prune)
// (without tau only "cannot lower the current minimum" is used, which keeps
// the minima exact); in collect mode the chunk is skipped when g - eps
// exceeds the collect threshold.
__device__ __forceinline__ float wmin_u(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wave_min(v)))); }

__device__ __forceinline__ float block_gap(const float4 alo, const float4 ahi, const float4 blo, const float4 bhi)
{
    const double gx = fmax(0.0, fmax((double)blo.x - ahi.x, (double)alo.x - bhi.x));
    const double gy = fmax(0.0, fmax((double)blo.y - ahi.y, (double)alo.y - bhi.y));
    const double gz = fmax(0.0, fmax((double)blo.z - ahi.z, (double)alo.z - bhi.z));
    return (float)sqrt(gx * gx + gy * gy + gz * gz) * (1.0f - 0x1p-20f);
}

// Box gap in FP32 rounded down: each difference, square, sum and the
// hardware square root add at most a few ulps, so scaling by (1 - 2^-20)
// keeps it below the exact gap (a flushed denormal only lowers it).
__device__ __forceinline__ float box_gap32(const float4 alo, const float4 ahi, const float4 blo, const float4 bhi)
{
    const float gx = fmaxf(0.0f, fmaxf(blo.x - ahi.x, alo.x - bhi.x));
    const float gy = fmaxf(0.0f, fmaxf(blo.y - ahi.y, alo.y - bhi.y));
    const float gz = fmaxf(0.0f, fmaxf(blo.z - ahi.z, alo.z - bhi.z));
    return __builtin_amdgcn_sqrtf(fmaf(gz, gz, fmaf(gy, gy, gx * gx))) * (1.0f - 0x1p-20f);
}

// The cut of a chunk or facet whose FP32 distance to every A facet of the
// tile is >= g (box gap minus eps) and whose max ph is bph: it cannot change
// a decision (within), the exact minima (no tau), or the collected set.
// lbm/ubm may be any lane's running minima: each is >= the item's final one.
template <bool COLLECT>
__device__ __forceinline__ bool chunk_cut(float g, float bph, float aph, float cur_lb, float cur_ub, float lbm,
                                          float ubm, const Item &it, float tau, bool within)
{
    if (COLLECT) return g > fminf(it.thr, fminf(cur_ub, ubm) + 2.0f * it.eps);
    const float ub_cut = within ? fminf(fminf(cur_ub, ubm), tau - it.eps) : fminf(cur_ub, ubm);
    const float lb_cut = within ? fminf(fminf(cur_lb, lbm), tau + it.eps) : fminf(cur_lb, lbm);
    return g > ub_cut && fmaxf(g - aph - bph, 0.0f) > lb_cut;
}

// The A blocks of a tile with more than one are claimed one at a time from
// the tile's cursor, so other waves can take part in a tile once the list is
// used up; the owner (the wave that took the tile from the list) shows the
// tile in its workgroup slot until the cursor is exhausted.  A helper claims
// its first block before it comes here (`pre`, -1 for the owner), so a tile
// whose blocks are all taken costs it one atomic, not the set-up below.
template <int P, bool COLLECT>
__device__ __forceinline__ void refine_tile_f32(const RefineArgs &a, const int t, float4 *sh, bool owner, int pre,
                                                unsigned long long &pairs_acc, unsigned long long &culled_acc)
{
    const int lane = threadIdx.x;
    float4 *const qv = sh;  // the facet queue shares the record array
    const Tile tl = a.tiles[t];
    const Item it = a.items[tl.item];
    ItemOut *o = a.out + tl.item;
    if (!COLLECT && a.early &&
        __builtin_amdgcn_readfirstlane(__hip_atomic_load(&o->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
        return;
    const bool swap = it.flags & IT_SWAP;
    const FacetSrc SA = facet_src(swap ? a.S : a.R, it.a_obj, it.lod);
    const FacetSrc SB = facet_src(swap ? a.R : a.S, it.b_obj, it.lod);
    const int vrow = (a.vmask && SA.vlab && SB.vlab) ? a.vrow[it.cand] : -1;
    const unsigned long long *vrows = vrow >= 0 ? a.vmask + (size_t)vrow * kMaxVox : nullptr;
    const V3 org = V3{it.ox, it.oy, it.oz};
    const bool within = a.tau >= 0.0f;
    float lbm = kInf, ubm = kInf;
    int sure = 0;
    int culled = 0;
    unsigned long long npairs = 0;
    const bool finest = it.flags & IT_FINEST;
    bool stop = false;
    // the tile's A facets, one register block of 64P at a time
    const int nblk = (tl.a1 - tl.a0 + 64 * P - 1) / (64 * P);
    if (owner && nblk > 1 && lane == 0) __hip_atomic_store(a.wave_slot + blockIdx.x, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Dead A blocks.  Against the union of the B range's chunk records (box,
    // max ph) a block that passes the chunk cut passes it for every chunk of
    // the range, each being at least as far and no coarser; such a block
    // costs only its claim.  The union is formed on the first block the wave
    // takes, and the blocks are tested 64 at a time (one per lane, the
    // result a 64-bit mask kept for the batch of the last block taken).
    const int nbch = (tl.b1 - tl.b0 + 63) >> 6;
    float4 ulo = make_float4(kInf, kInf, kInf, 0.0f), uhi = make_float4(-kInf, -kInf, -kInf, 0.0f);
    bool have_u = false;
    int dead_bt = -1;
    unsigned long long dead_m = 0ull;
    for (int k = 0;; ++k) {
        int j = k;
        if (k == 0 && pre >= 0) {
            j = pre;
        } else if (nblk > 1) {
            int c = 0;
            if (lane == 0) c = atomicAdd(a.tile_cur + t, 1);
            j = __builtin_amdgcn_readfirstlane(c);
        }
        if (j >= nblk || stop) break;
        if (P == 1 && a.cull && nblk > 1) {
            if (!have_u) {
                for (int c0 = 0; c0 < nbch; c0 += 64) {
                    if (c0 + lane < nbch) {
                        const int c = (tl.b0 >> 6) + c0 + lane;
                        const float4 l = SB.blk[2 * c], h = SB.blk[2 * c + 1];
                        ulo = make_float4(fminf(ulo.x, l.x), fminf(ulo.y, l.y), fminf(ulo.z, l.z), 0.0f);
                        uhi = make_float4(fmaxf(uhi.x, h.x), fmaxf(uhi.y, h.y), fmaxf(uhi.z, h.z), fmaxf(uhi.w, h.w));
                    }
                }
                ulo = make_float4(wmin_u(ulo.x), wmin_u(ulo.y), wmin_u(ulo.z), 0.0f);
                uhi = make_float4(-wmin_u(-uhi.x), -wmin_u(-uhi.y), -wmin_u(-uhi.z), -wmin_u(-uhi.w));
                have_u = true;
            }
            const int bt = j >> 6;
            if (bt != dead_bt) {
                const float clb = __uint_as_float(__builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&o->lb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                const float cub = __uint_as_float(__builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&o->ub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                bool dead = false;
                const int jb = (bt << 6) + lane;
                if (jb < nblk) {
                    const int rb = (tl.a0 >> 6) + jb;
                    const float4 bl = SA.blk[2 * rb], bh = SA.blk[2 * rb + 1];
                    const float g = box_gap32(bl, bh, ulo, uhi) - it.eps;
                    dead = chunk_cut<COLLECT>(g, uhi.w, bh.w, clb, cub, lbm, ubm, it, a.tau, within);
                }
                dead_m = __ballot(dead);
                dead_bt = bt;
            }
            if ((dead_m >> (j & 63)) & 1ull) {
                culled += nbch;
                if (j == nblk - 1) break;
                continue;
            }
        }
        const int a0 = tl.a0 + j * 64 * P;
        int cols = 0;
        // the A records are built when the first chunk survives its test, so a
        // block whose chunks are all culled costs only block-record reads
        Rec ra[P];
        bool built = false;
        // union of the A block records (block starts are multiples of 64)
        float4 alo = SA.blk[2 * (a0 >> 6)], ahi = SA.blk[2 * (a0 >> 6) + 1];
#pragma unroll
        for (int p = 1; p < P; ++p) {
            if (a0 + 64 * p >= SA.n) break;
            const float4 l2 = SA.blk[2 * ((a0 >> 6) + p)], h2 = SA.blk[2 * ((a0 >> 6) + p) + 1];
            alo = make_float4(fminf(alo.x, l2.x), fminf(alo.y, l2.y), fminf(alo.z, l2.z), fmaxf(alo.w, l2.w));
            ahi = make_float4(fmaxf(ahi.x, h2.x), fmaxf(ahi.y, h2.y), fmaxf(ahi.z, h2.z), fmaxf(ahi.w, h2.w));
        }
        const float aph = ahi.w;
        // Voxel pairs: the B voxels paired (after the voxel filter) with any
        // voxel of this A block's facets; B chunks and facets outside them
        // cannot hold the pair that decides the item and are skipped.
        unsigned long long bvox = ~0ull;
        if (vrows) {
            unsigned long long la = 0ull;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int fa = a0 + lane + 64 * p;
                if (fa < SA.n) la |= 1ull << SA.vlab[fa];
            }
            la = wave_or64(la);
            const unsigned long long row = vrows[lane];
            if (!swap) bvox = wave_or64(((la >> lane) & 1ull) ? row : 0ull);  // rows are A (R) voxels
            else bvox = __ballot((row & la) != 0ull);                          // rows are B (R) voxels
            if (bvox == 0ull) {
                culled += (tl.b1 - tl.b0 + 63) >> 6;
                continue;
            }
        }
        // Surviving B facets wait in an LDS queue (qv: corners, hd, ph and
        // index, as gathered for the facet test) and are evaluated 64 at a
        // time: their records are built by all lanes at once, then every lane
        // runs its A facet against each of them.  The queue and the records
        // share one LDS array: a flush first takes its facets and the queue's
        // overflow beyond them into registers, writes the records over the
        // queue, and after the pair loop puts the overflow back at the front.
        int qn = 0;
        auto flush = [&](const int n) {
            if (!built) {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    int fa = a0 + lane + 64 * p;
                    if (fa >= SA.n) fa = a0;  // padding lanes repeat a real facet
                    ra[p] = load_rec(SA, fa, org);
                }
                built = true;
            }
            const int rest = qn - n;  // queued facets beyond this batch (fewer than 64)
            float4 q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), q1 = q0, q2 = q0, r0 = q0, r1 = q0, r2 = q0;
            if (lane < n) {
                q0 = qv[3 * lane];
                q1 = qv[3 * lane + 1];
                q2 = qv[3 * lane + 2];
            }
            if (lane < rest) {
                r0 = qv[3 * (n + lane)];
                r1 = qv[3 * (n + lane) + 1];
                r2 = qv[3 * (n + lane) + 2];
            }
            __syncthreads();
            if (lane < n) {
                const V3 w0{q0.x, q0.y, q0.z}, w1{q0.w, q1.x, q1.y}, w2{q1.z, q1.w, q2.x};
                Rec rb = make_rec(w0 - org, w1 - org, w2 - org, q2.y, q2.z);
                rb.pad = q2.w;
                float tmp[44];
                __builtin_memcpy(tmp, &rb, sizeof(tmp));
#pragma unroll
                for (int q = 0; q < 11; ++q)
                    sh[lane * 11 + q] = make_float4(tmp[4 * q], tmp[4 * q + 1], tmp[4 * q + 2], tmp[4 * q + 3]);
            }
            __syncthreads();
            // the item's done flag, read now and used after the pair loop (a
            // stale value costs at most one more flush), so the load's latency
            // is hidden behind the loop
            int done_pre = 0;
            if (!COLLECT && a.early) done_pre = __hip_atomic_load(&o->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // collect: the item's published minimum (>= its final one) also
            // bounds what is kept, so a lane's first pairs of a block are not
            // all kept against its own still-open minimum
            if (COLLECT && a.cull)
                ubm = fminf(ubm, __uint_as_float(__builtin_amdgcn_readfirstlane(
                                     __hip_atomic_load(&o->ub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))));
#pragma unroll 1
            for (int k = 0; k < n; ++k) {
                float tmp[44];
#pragma unroll
                for (int q = 0; q < 11; ++q) {
                    float4 x = sh[k * 11 + q];
                    tmp[4 * q] = x.x;
                    tmp[4 * q + 1] = x.y;
                    tmp[4 * q + 2] = x.z;
                    tmp[4 * q + 3] = x.w;
                }
                Rec rb;
                __builtin_memcpy(&rb, tmp, sizeof(rb));
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    Pair32 pr = pair_f32(ra[p], rb, it.eps);
                    float dlo = pr.lo * (ra[p].ok * rb.ok);
                    lbm = fminf(lbm, fmaxf(dlo - (ra[p].ph + rb.ph), 0.0f));
                    ubm = fminf(ubm, pr.hi + (ra[p].hd + rb.hd));
                    sure |= pr.sure ? 1 : 0;
                    if (COLLECT) {
                        const int fa = a0 + lane + 64 * p;
                        // the pair realising the minimum has dlo <= d + eps <= ubm + 2 eps
                        if (fa < SA.n && dlo <= fminf(it.thr, ubm + 2.0f * it.eps)) {
                            const unsigned long long slot = atomicAdd(a.collected_n, 1ull);
                            if (slot < (unsigned long long)a.collect_cap)
                                a.collected[slot] = PairRef{tl.item, fa, __float_as_int(rb.pad), 0};
                            else a.overflow[tl.item] = 1;
                        }
                    }
                }
            }
            cols += n;
            __syncthreads();
            if (lane < rest) {
                qv[3 * lane] = r0;
                qv[3 * lane + 1] = r1;
                qv[3 * lane + 2] = r2;
            }
            qn = rest;
            __syncthreads();
            if (a.cull) {  // publish the running minima so that other tiles can cull against them
                const float wl = wmin_u(lbm), wu = wmin_u(ubm);
                lbm = wl;
                ubm = wu;
                if (lane == 0) {
                    atomicMin(&o->lb, fbits(wl));
                    atomicMin(&o->ub, fbits(wu));
                }
            }
            if (!COLLECT && a.early) {
                const float wub = wmin_u(ubm);
                const int ws = __builtin_amdgcn_readfirstlane(wave_or(sure));
                const bool confirm = (a.tau > 0.0f && wub + it.eps <= a.tau) || (finest && ws);
                if (confirm) {
                    if (lane == 0) __hip_atomic_store(&o->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    stop = true;
                } else if (__builtin_amdgcn_readfirstlane(done_pre)) {
                    stop = true;
                }
            }
        };
        // Groups of up to 64 streamed chunks: lane j tests chunk j of the group
        // from its block record, a ballot leaves the chunks that may matter, and
        // the wave walks those nearest first (in order without culling).
        // Before a chunk is loaded its test is
        // repeated with the minima found so far (read back from the testing
        // lane).  One loop takes the surviving chunks of every group and ends
        // with the flush of what is left in the queue, so the flush and its
        // pair loop have a single call site.
        int g0 = tl.b0;  // next group to test
        int gb = tl.b0;  // group whose survivors are in cmask
        unsigned long long cmask = 0ull;
        float cur_lb = kInf, cur_ub = kInf;
        float gap_l = 0.0f, bph_l = 0.0f;
        for (;;) {
            // the next chunk that survives its tests, or -1 at the end of the range
            int cb = -1;
            while (!stop) {
                if (cmask == 0ull) {
                    if (g0 >= tl.b1) break;
                    const int nch = min(64, (tl.b1 - g0 + 63) >> 6);
                    if (a.cull) {
                        cur_lb = __uint_as_float(__builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(&o->lb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                        cur_ub = __uint_as_float(__builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(&o->ub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
                        bool live = false;
                        if (lane < nch) {
                            const int c = (g0 >> 6) + lane;
                            const float4 blo = SB.blk[2 * c], bhi = SB.blk[2 * c + 1];
                            gap_l = box_gap32(alo, ahi, blo, bhi) - it.eps;
                            bph_l = bhi.w;
                            live = !chunk_cut<COLLECT>(gap_l, bph_l, aph, cur_lb, cur_ub, lbm, ubm, it, a.tau, within);
                            if (vrows) live = live && (SB.bmask[c] & bvox) != 0ull;
                        }
                        cmask = __ballot(live);
                        culled += nch - __popcll(cmask);
                    } else {
                        cmask = nch == 64 ? ~0ull : ((1ull << nch) - 1ull);
                        if (vrows) {
                            const bool live = lane < nch && (SB.bmask[(g0 >> 6) + lane] & bvox) != 0ull;
                            cmask = __ballot(live);
                            culled += nch - __popcll(cmask);
                        }
                    }
                    gb = g0;
                    g0 += 64 * 64;
                    continue;
                }
                int j = __builtin_ctzll(cmask);
                if (a.cull) {
                    // nearest chunk first (smallest box gap among those left),
                    // so the running minima tighten early and the chunks after
                    // it are cut by the retest below
                    const float gm = ((cmask >> lane) & 1ull) ? gap_l : kInf;
                    const float mn = wmin_u(gm);
                    const unsigned long long at = __ballot(gm == mn) & cmask;
                    if (at != 0ull) j = __builtin_ctzll(at);
                }
                cmask &= ~(1ull << j);
                if (a.cull) {
                    const float gj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gap_l), j));
                    const float bj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bph_l), j));
                    const float l0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(lbm)));
                    const float u0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(ubm)));
                    if (__builtin_amdgcn_readfirstlane(
                            (int)chunk_cut<COLLECT>(gj, bj, aph, cur_lb, cur_ub, l0, u0, it, a.tau, within))) {
                        ++culled;
                        continue;
                    }
                }
                cb = gb + 64 * j;
                break;
            }
            if (cb >= 0) {
                const int nb = min(64, tl.b1 - cb);
                int f = cb + lane;
                if (f >= tl.b1) f = cb;
                // Facet culling: the same two-sided test with this facet's own
                // box and ph against the A block; survivors join the LDS queue
                // with the corners and bounds gathered here.
                bool keep = lane < nb;
                if (vrows) keep = keep && ((bvox >> SB.vlab[f]) & 1ull);
                const int32_t i0 = SB.tris[3 * f], i1 = SB.tris[3 * f + 1], i2 = SB.tris[3 * f + 2];
                const V3 w0 = ld3f(SB.verts, i0), w1 = ld3f(SB.verts, i1), w2 = ld3f(SB.verts, i2);
                const float2 bh = SB.hdph ? SB.hdph[f] : make_float2(0.0f, 0.0f);
                if (a.cull) {
                    const float bph = bh.y;
                    const float4 flo = make_float4(fminf(fminf(w0.x, w1.x), w2.x), fminf(fminf(w0.y, w1.y), w2.y),
                                                   fminf(fminf(w0.z, w1.z), w2.z), 0.0f);
                    const float4 fhi = make_float4(fmaxf(fmaxf(w0.x, w1.x), w2.x), fmaxf(fmaxf(w0.y, w1.y), w2.y),
                                                   fmaxf(fmaxf(w0.z, w1.z), w2.z), 0.0f);
                    const float g = box_gap32(alo, ahi, flo, fhi) - it.eps;
                    keep = keep && !chunk_cut<COLLECT>(g, bph, aph, cur_lb, cur_ub, lbm, ubm, it, a.tau, within);
                }
                const unsigned long long kmask = __ballot(keep);
                const int nk = __popcll(kmask);
                if (nk == 0) ++culled;
                if (keep) {
                    const int pos = qn + __builtin_amdgcn_mbcnt_hi((unsigned)(kmask >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((unsigned)kmask, 0u));
                    qv[3 * pos] = make_float4(w0.x, w0.y, w0.z, w1.x);
                    qv[3 * pos + 1] = make_float4(w1.y, w1.z, w2.x, w2.y);
                    qv[3 * pos + 2] = make_float4(w2.z, bh.x, bh.y, __int_as_float(f));
                }
                qn += nk;
                __syncthreads();
            }
            // a full batch (the facets beyond it stay queued), or what is left
            // at the end of the range
            if (qn >= 64 || (cb < 0 && qn > 0 && !stop)) flush(min(qn, 64));
            if (cb < 0) break;
        }
        npairs += (unsigned long long)min(64 * P, SA.n - a0) * (unsigned long long)cols;
        if (j == nblk - 1) break;  // this wave took the last block: no claim is left to try
    }  // A blocks
    if (owner && nblk > 1 && lane == 0) __hip_atomic_store(a.wave_slot + blockIdx.x, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float wl = wave_min(lbm), wu = wave_min(ubm);
    const int ws = wave_or(sure);
    if (lane == 0) {
        atomicMin(&o->lb, fbits(wl));
        atomicMin(&o->ub, fbits(wu));
        if (ws) atomicOr(&o->hit, 1);
    }
    pairs_acc += npairs;
    culled_acc += (unsigned long long)culled;
}

// Persistent single-wave workgroups take tiles from the list (longest items
// first) in order, each fetching the next index with one atomic on a counter
// that the host zeroes before the launch, so a wave that finishes early takes
// more tiles.  Lane 0 fetches and readfirstlane makes the index uniform: the
// loop control is scalar and every lane runs the same tiles.  The fetch for
// the next tile is issued before the current one is processed.
//
// Once the list is used up, the wave makes one pass over the workgroup slots
// (or the tiles) and joins every tile that still has unclaimed A blocks, so
// a tile whose facets meet over a large area (most of its pairs survive
// culling) is finished by many waves instead of holding one to the end of
// the launch.  Termination: every fetch raises the list counter; every claim
// raises a tile cursor; the pass visits each slot or tile at most once.
template <int P, bool COLLECT>
__device__ __forceinline__ void refine_tiles(const RefineArgs &a, float4 *sh)
{
    const int ntiles = *a.ntiles;
    const int nslot = gridDim.x;
    // launch-wide statistics, published once per wave
    unsigned long long pairs_acc = 0, culled_acc = 0;
    int nxt = 0;  // lane 0: the list index fetched for the next tile
    if (threadIdx.x == 0) nxt = atomicAdd(a.tile_next, 1);
    // phase 0 takes tiles from the list; then the helping pass over the tiles
    // still in progress.  A round with no more tiles than workgroups scans
    // the tiles themselves (phase 1: every tile has been taken by now, and a
    // multi-block tile with blocks left can be joined); a larger one scans
    // the workgroup slots (phase 2), starting at this workgroup's own so
    // that the helpers spread over the tiles in progress.  In phase 1 each
    // helper starts at its own tile (wrapping around), so that they do not
    // all queue on the cursors of the first tiles.  One call site of the
    // tile body keeps a single copy of it in the kernel.
    int phase = 0, h = 0;
    const int start = (int)(blockIdx.x % (unsigned)max(ntiles, 1));
    for (;;) {
        int t = -1;
        bool owner = false;
        if (phase == 0) {
            const int c = __builtin_amdgcn_readfirstlane(nxt);
            if (c < ntiles) {
                t = c;
                owner = true;
                // the fetch for the next tile is issued before this one is processed
                if (threadIdx.x == 0) nxt = atomicAdd(a.tile_next, 1);
            } else {
                phase = ntiles <= nslot ? 1 : 2;
            }
        }
        int pre = -1;
        if (phase == 1 || phase == 2) {
            // a tile with blocks left (lane l of a 64-wide look), then the
            // claim of one of them; on a lost race the look goes on
            const int lim = phase == 1 ? ntiles : nslot;
            while (t < 0 && h < lim) {
                const int hw = h + (int)threadIdx.x;
                int c = -1, nb = 0;
                if (hw < lim) {
                    int tt;
                    if (phase == 1) {
                        tt = hw + start;
                        if (tt >= ntiles) tt -= ntiles;
                    } else {
                        int w = hw + (int)blockIdx.x;
                        if (w >= nslot) w -= nslot;
                        tt = __hip_atomic_load(a.wave_slot + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (tt >= 0 && tt < ntiles) {
                        const Tile x = a.tiles[tt];
                        nb = (x.a1 - x.a0 + 64 * P - 1) / (64 * P);
                        if (nb > 1 && __hip_atomic_load(a.tile_cur + tt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < nb)
                            c = tt;
                    }
                }
                const unsigned long long m = __ballot(c >= 0);
                if (m == 0ull) {
                    h += 64;
                    continue;
                }
                const int l = __builtin_ctzll(m);
                const int tt = __builtin_amdgcn_readlane(c, l);
                const int nbt = __builtin_amdgcn_readlane(nb, l);
                h += l + 1;
                int got = 0;
                if (threadIdx.x == 0) got = atomicAdd(a.tile_cur + tt, 1);
                got = __builtin_amdgcn_readfirstlane(got);
                if (got < nbt) {
                    t = tt;
                    pre = got;
                }
            }
        }
        if (t < 0) break;
        refine_tile_f32<P, COLLECT>(a, t, sh, owner, pre, pairs_acc, culled_acc);
    }
    if (threadIdx.x == 0) {
        if (pairs_acc) atomicAdd(a.pairs_done, pairs_acc);
        if (culled_acc) atomicAdd(a.chunks_culled, culled_acc);
    }
}

// the facet queue (at most 127 entries of 3 float4) lives in the record array
static_assert(127 * 3 <= 64 * 11, "facet queue fits in the LDS record array");

// Waves per SIMD the refinement kernels are compiled for.  Three (at most
// 168 VGPRs) fit beside the 11 KB of LDS each single-wave workgroup holds
// (14 per CU); at that limit the pair loop still keeps every value in
// registers and only cold per-tile state spills.
#ifndef PJ_REFINE_WAVES
#define PJ_REFINE_WAVES 3
#endif

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PJ_REFINE_WAVES, PJ_REFINE_WAVES))) void
k_refine_f32(RefineArgs a)
{
    __shared__ float4 sh[64 * 11];
    refine_tiles<P, false>(a, sh);
}

// Collect pass: the same tiles, keeping every facet pair whose FP32 lower
// distance is at most the item's threshold (for the FP64 recheck).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PJ_REFINE_WAVES, PJ_REFINE_WAVES))) void
k_collect_f32(RefineArgs a)
{
    __shared__ float4 sh[64 * 11];
    refine_tiles<1, true>(a, sh);
}

hipError_t launch_collect_f32(const RefineArgs &a, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_collect_f32, dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_refine_f32(const RefineArgs &a, int grid, int P, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (P == 1) hipLaunchKernelGGL(k_refine_f32<1>, dim3(grid), dim3(64), 0, st, a);
    else if (P == 2) hipLaunchKernelGGL(k_refine_f32<2>, dim3(grid), dim3(64), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 refinement over tiles (guard-band recheck): one lane = one A facet,
// B facets through LDS; exact meet test; results merged with 64-bit atomicMin
// of non-negative doubles.
// ---------------------------------------------------------------------------
struct FacetSrc64 {
    const int32_t *tris;
    const float *verts;
    const float2 *hdph;
    int n;
};

// One tile (64 A facets x a B range) of the tiled FP64 kernel; the B facets
// are staged in LDS 64 at a time and the barrier after the last chunk leaves
// sb free for the next tile.
__device__ __forceinline__ void refine_tile_f64(const Refine64Args &a, const Tile tl, float *sb, const int lane)
{
    const Item it = a.items[tl.item];
    const bool swap = it.flags & IT_SWAP;
    const FacetSrc SA = facet_src(swap ? a.S : a.R, it.a_obj, it.lod);
    const FacetSrc SB = facet_src(swap ? a.R : a.S, it.b_obj, it.lod);
    int f = tl.a0 + lane;
    if (f >= SA.n) f = tl.a0;
    D3 A[3];
    for (int c = 0; c < 3; ++c) A[c] = ld3d(SA.verts, SA.tris[3 * f + c]);
    float2 ha = SA.hdph ? SA.hdph[f] : make_float2(0.0f, 0.0f);
    double lbm = __builtin_inf(), ubm = __builtin_inf();
    int hit = 0;
    for (int cb = tl.b0; cb < tl.b1; cb += 64) {
        const int nb = min(64, tl.b1 - cb);
        {
            int g = cb + lane;
            if (g >= tl.b1) g = cb;
            for (int c = 0; c < 3; ++c) {
                int vi = SB.tris[3 * g + c];
                sb[lane * 12 + 3 * c] = SB.verts[3 * vi];
                sb[lane * 12 + 3 * c + 1] = SB.verts[3 * vi + 1];
                sb[lane * 12 + 3 * c + 2] = SB.verts[3 * vi + 2];
            }
            float2 hb = SB.hdph ? SB.hdph[g] : make_float2(0.0f, 0.0f);
            sb[lane * 12 + 9] = hb.x;
            sb[lane * 12 + 10] = hb.y;
        }
        __syncthreads();
        for (int k = 0; k < nb; ++k) {
            const float *x = sb + k * 12;
            D3 B[3] = {D3{x[0], x[1], x[2]}, D3{x[3], x[4], x[5]}, D3{x[6], x[7], x[8]}};
            bool h;
            double d = pair_f64(A, B, h);
            hit |= h ? 1 : 0;
            lbm = fmin(lbm, fmax(d - ((double)ha.y + (double)x[10]), 0.0));
            ubm = fmin(ubm, d + ((double)ha.x + (double)x[9]));
        }
        __syncthreads();
    }
    lbm = wave_min_d(lbm);
    ubm = wave_min_d(ubm);
    hit = wave_or(hit);
    if (lane == 0) {
        ItemOut64 *o = a.out + tl.item;
        atomicMin(&o->lb, (unsigned long long)__double_as_longlong(lbm));
        atomicMin(&o->ub, (unsigned long long)__double_as_longlong(ubm));
        if (hit) atomicOr(&o->hit, 1);
    }
}

// one workgroup per tile, striding over the list when it is longer than the grid
__global__ __launch_bounds__(64) void k_refine_f64_tiles(Refine64Args a, int64_t ntiles)
{
    __shared__ float sb[64 * 12];
    const int lane = threadIdx.x;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) refine_tile_f64(a, a.tiles[t], sb, lane);
}

hipError_t launch_refine_f64_tiles(const Refine64Args &a, int64_t ntiles, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_f64_tiles, dim3((unsigned)std::min<int64_t>(ntiles, kStrideBlocks)), dim3(64), 0,
                       st, a, ntiles);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain schedule (the paper's Algorithm 4 shape): one 256-thread workgroup
// per (pair, LoD); the n_A x n_B facet pairs are flattened and dealt to the
// threads round-robin; thread-local minima are combined in LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void refine_item_f64_plain(const Refine64Args &a, const int item, double *shl, double *shu,
                                                      int *shh)
{
    const Item it = a.items[item];
    const bool swap = it.flags & IT_SWAP;
    const FacetSrc SA = facet_src(swap ? a.S : a.R, it.a_obj, it.lod);
    const FacetSrc SB = facet_src(swap ? a.R : a.S, it.b_obj, it.lod);
    const int64_t total = (int64_t)SA.n * SB.n;
    double lbm = __builtin_inf(), ubm = __builtin_inf();
    int hit = 0;
    for (int64_t t = threadIdx.x; t < total; t += 256) {
        const int i = (int)(t / SB.n), j = (int)(t - (int64_t)i * SB.n);
        D3 A[3], B[3];
        for (int c = 0; c < 3; ++c) {
            A[c] = ld3d(SA.verts, SA.tris[3 * i + c]);
            B[c] = ld3d(SB.verts, SB.tris[3 * j + c]);
        }
        float2 ha = SA.hdph ? SA.hdph[i] : make_float2(0.0f, 0.0f);
        float2 hb = SB.hdph ? SB.hdph[j] : make_float2(0.0f, 0.0f);
        bool h;
        double d = pair_f64(A, B, h);
        hit |= h ? 1 : 0;
        lbm = fmin(lbm, fmax(d - ((double)ha.y + (double)hb.y), 0.0));
        ubm = fmin(ubm, d + ((double)ha.x + (double)hb.x));
    }
    lbm = wave_min_d(lbm);
    ubm = wave_min_d(ubm);
    hit = wave_or(hit);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        shl[w] = lbm;
        shu[w] = ubm;
        shh[w] = hit;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ItemOut64 *o = a.out + item;
        double l = fmin(fmin(shl[0], shl[1]), fmin(shl[2], shl[3]));
        double u = fmin(fmin(shu[0], shu[1]), fmin(shu[2], shu[3]));
        o->lb = (unsigned long long)__double_as_longlong(l);
        o->ub = (unsigned long long)__double_as_longlong(u);
        o->hit = shh[0] | shh[1] | shh[2] | shh[3];
    }
    __syncthreads();  // the LDS partials are rewritten by the next item
}

// one workgroup per (pair, LoD), striding over the list when it is longer than the grid
__global__ __launch_bounds__(256) void k_refine_f64_plain(Refine64Args a, int nitems)
{
    __shared__ double shl[4], shu[4];
    __shared__ int shh[4];
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) refine_item_f64_plain(a, i, shl, shu, shh);
}

hipError_t launch_refine_f64_plain(const Refine64Args &a, int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_f64_plain, dim3((unsigned)std::min<int64_t>(nitems, kStrideBlocks)), dim3(256), 0, st, a,
                       nitems);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 recheck of collected facet pairs: exact meet test, FP64 distance,
// 64-bit atomicMin per item.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_f64_ref(const MeshDev &R, const MeshDev &S, const Item *items, const PairRef pr,
                                             ItemOut64 *out)
{
    const Item it = items[pr.item];
    const bool swap = it.flags & IT_SWAP;
    const FacetSrc SA = facet_src(swap ? S : R, it.a_obj, it.lod);
    const FacetSrc SB = facet_src(swap ? R : S, it.b_obj, it.lod);
    D3 A[3], B[3];
    for (int c = 0; c < 3; ++c) {
        A[c] = ld3d(SA.verts, SA.tris[3 * pr.a + c]);
        B[c] = ld3d(SB.verts, SB.tris[3 * pr.b + c]);
    }
    bool h;
    const double d = pair_f64(A, B, h);
    ItemOut64 *o = out + pr.item;
    atomicMin(&o->lb, (unsigned long long)__double_as_longlong(d));
    atomicMin(&o->ub, (unsigned long long)__double_as_longlong(d));
    if (h) atomicOr(&o->hit, 1);
}

__global__ __launch_bounds__(256) void k_pairs_f64(MeshDev R, MeshDev S, const Item *items, const PairRef *pairs,
                                                   int64_t n, ItemOut64 *out)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        pair_f64_ref(R, S, items, pairs[i], out);
}

hipError_t launch_pairs_f64(const MeshDev &R, const MeshDev &S, const Item *items, const PairRef *pairs, int64_t n,
                            ItemOut64 *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairs_f64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, kStrideBlocks)), dim3(256), 0, st, R,
                       S, items, pairs, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-NN candidates (Section 3.1, "MBB-based Object Filtering" for k-NN): the
// k-th smallest anchor upper bound theta_r over S, found by bisection on the
// float bit pattern (monotone for non-negative floats); then every s whose
// box gap does not exceed theta_r.  One wave per r.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float anchor_ub(const float *ar, const float *as)
{
    float dx = as[0] - ar[0], dy = as[1] - ar[1], dz = as[2] - ar[2];
    return __builtin_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) * (1.0f + 0x1p-20f);
}

__global__ __launch_bounds__(64) void k_knn_theta(const float *ancR, int nR, const float *ancS, int nS, int k,
                                                  float *theta)
{
    const int r = blockIdx.x;
    const float *ar = ancR + 3 * (int64_t)r;
    if (nS < k) {
        if (threadIdx.x == 0) theta[r] = __builtin_inff();
        return;
    }
    // invariant: count(ub <= hi) >= k; 32 halvings of [0, +inf bits] end with lo == hi
    unsigned lo = 0u, hi = 0x7f800000u;
    for (int step = 0; step < 32; ++step) {
        const unsigned mid = lo + ((hi - lo) >> 1);
        int cnt = 0;
        for (int s = threadIdx.x; s < nS; s += 64) cnt += __float_as_uint(anchor_ub(ar, ancS + 3 * (int64_t)s)) <= mid;
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        cnt = __builtin_amdgcn_readfirstlane(cnt);
        if (cnt >= k) hi = mid;
        else lo = mid + 1;
    }
    if (threadIdx.x == 0) theta[r] = __uint_as_float(lo);
}

hipError_t launch_knn_theta(const float *ancR, int nR, const float *ancS, int nS, int k, float *theta, hipStream_t st)
{
    if (nR == 0) return hipSuccess;
    PJ_GRID_CHECK(nR, 64);
    hipLaunchKernelGGL(k_knn_theta, dim3(nR), dim3(64), 0, st, ancR, nR, ancS, nS, k, theta);
    return hipGetLastError();
}

__device__ __forceinline__ float box_gap(const float *b, const float *x)
{
    float gx = fmaxf(0.0f, fmaxf(x[0] - b[3], b[0] - x[3]));
    float gy = fmaxf(0.0f, fmaxf(x[1] - b[4], b[1] - x[4]));
    float gz = fmaxf(0.0f, fmaxf(x[2] - b[5], b[2] - x[5]));
    return __builtin_sqrtf(fmaf(gz, gz, fmaf(gy, gy, gx * gx)));
}

// count pass: count[r]; write pass: survivors of r at off[r].. in s order
__global__ __launch_bounds__(64) void k_knn_cand(const float *boxR, const float *ancR, int nR, const float *boxS,
                                                 const float *ancS, int nS, const float *theta, int32_t *count,
                                                 const int64_t *off, int32_t *cs, float *clb, float *cub,
                                                 int write_pass)
{
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    const float *br = boxR + 6 * (int64_t)r;
    const float th = theta[r];
    int64_t pos = write_pass ? off[r] : 0;
    int total = 0;
    for (int s0 = 0; s0 < nS; s0 += 64) {
        const int s = s0 + lane;
        const float g = s < nS ? box_gap(br, boxS + 6 * (int64_t)s) * (1.0f - 0x1p-20f) : __builtin_inff();
        const bool keep = s < nS && g <= th;
        const unsigned long long m = __ballot(keep);
        if (write_pass && keep) {
            const int rank = __popcll(m & ((1ull << lane) - 1ull));
            cs[pos + rank] = s;
            clb[pos + rank] = g;
            cub[pos + rank] = anchor_ub(ancR + 3 * (int64_t)r, ancS + 3 * (int64_t)s);
        }
        pos += __popcll(m);
        total += __popcll(m);
    }
    if (!write_pass && lane == 0) count[r] = total;
}

hipError_t launch_knn_cand(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS, int nS,
                           const float *theta, int32_t *count, const int64_t *off, int32_t *cs, float *clb,
                           float *cub, int write_pass, hipStream_t st)
{
    if (nR == 0) return hipSuccess;
    PJ_GRID_CHECK(nR, 64);
    hipLaunchKernelGGL(k_knn_cand, dim3(nR), dim3(64), 0, st, boxR, ancR, nR, boxS, ancS, nS, theta, count, off, cs,
                       clb, cub, write_pass);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-NN candidates through a uniform grid over the S anchors (scales past
// all-pairs): the same theta_r (k-th smallest anchor bound) and the same
// candidate test as above, evaluated only on the grid cells that can hold a
// smaller bound or a box within theta_r.
//   build:  cell of every S anchor, counting sort of S by cell;
//   theta:  one thread per r visits cell shells of growing Chebyshev radius
//           around r's (clamped) cell, keeping its k smallest bounds in
//           registers, until the k-th is below the distance from r's anchor
//           to every cell not visited yet (shrunk by one cell and an error
//           margin, so an anchor binned one cell off is still covered);
//   cand:   one thread per r tests the S objects of the cells its box can
//           reach (box widened by theta_r and the widest anchor-to-box extent
//           of S per axis), count then write, then sorts its list by s (the
//           order of the all-pairs kernel).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int grid_coord(float x, float o, float inv_c, int g)
{
    const float f = (x - o) * inv_c;
    const int c = f < 0.0f ? 0 : (f >= (float)g ? g - 1 : (int)f);
    return c;
}

__global__ void k_grid_cell(const float *anc, int n, KnnGrid g, int32_t *cell_of, int32_t *count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float *a = anc + 3 * (int64_t)i;
        const int cx = grid_coord(a[0], g.ox, g.inv_c, g.gx), cy = grid_coord(a[1], g.oy, g.inv_c, g.gy),
                  cz = grid_coord(a[2], g.oz, g.inv_c, g.gz);
        const int cell = (cz * g.gy + cy) * g.gx + cx;
        cell_of[i] = cell;
        atomicAdd(count + cell, 1);
    }
}

__global__ void k_grid_scatter(const int32_t *cell_of, int n, const int64_t *beg, int32_t *fill, int32_t *items)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int cell = cell_of[i];
        items[beg[cell] + atomicAdd(fill + cell, 1)] = i;
    }
}

hipError_t launch_grid_build(const float *ancS, int nS, const KnnGrid &g, int32_t *cell_of, int32_t *count,
                             int64_t *beg, int64_t *total, int32_t *fill, int32_t *items, hipStream_t st)
{
    const int64_t ncell = (int64_t)g.gx * g.gy * g.gz;
    hipError_t e;
    if ((e = hipMemsetAsync(count, 0, ncell * 4, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(fill, 0, ncell * 4, st)) != hipSuccess) return e;
    if (nS > 0) {
        const unsigned blocks = (unsigned)std::min<int64_t>((nS + 255) / 256, kStrideBlocks);
        hipLaunchKernelGGL(k_grid_cell, dim3(blocks), dim3(256), 0, st, ancS, nS, g, cell_of, count);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_scan_large(count, beg, total, ncell, st)) != hipSuccess) return e;
    if (nS > 0) {
        const unsigned blocks = (unsigned)std::min<int64_t>((nS + 255) / 256, kStrideBlocks);
        hipLaunchKernelGGL(k_grid_scatter, dim3(blocks), dim3(256), 0, st, cell_of, nS, beg, fill, items);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// distance from x to the S anchors binned outside cells [c0, c1] of one
// axis (an anchor may sit one cell off its bin): +inf on a side where the
// grid ends
__device__ __forceinline__ double side_gap(double x, int c0, int c1, int g, double o, double c)
{
    double gap = INFINITY;
    if (c0 > 0) gap = fmin(gap, fmax(0.0, x - (o + (double)(c0 + 1) * c)));
    if (c1 < g - 1) gap = fmin(gap, fmax(0.0, (o + (double)c1 * c) - x));
    return gap;
}

__global__ __launch_bounds__(256) void k_knn_theta_grid(const float *ancR, int nR, const float *ancS, int nS, int k,
                                                        KnnGrid g, const int64_t *beg, const int32_t *items,
                                                        float *theta)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nR) return;
    const float *ar = ancR + 3 * (int64_t)r;
    if (nS < k) {
        theta[r] = __builtin_inff();
        return;
    }
    float top[kGridMaxK];  // ascending; the first k are the k smallest bounds seen
#pragma unroll
    for (int i = 0; i < kGridMaxK; ++i) top[i] = __builtin_inff();
    float kth = __builtin_inff();
    const int cx = grid_coord(ar[0], g.ox, g.inv_c, g.gx), cy = grid_coord(ar[1], g.oy, g.inv_c, g.gy),
              cz = grid_coord(ar[2], g.oz, g.inv_c, g.gz);
    const int maxr = max(max(max(cx, g.gx - 1 - cx), max(cy, g.gy - 1 - cy)), max(cz, g.gz - 1 - cz));
    auto visit = [&](int x, int y, int z) {
        const int cell = (z * g.gy + y) * g.gx + x;
        for (int64_t q = beg[cell]; q < beg[cell + 1]; ++q) {
            float v = anchor_ub(ar, ancS + 3 * (int64_t)items[q]);
            if (v < kth) {
#pragma unroll
                for (int i = 0; i < kGridMaxK; ++i) {
                    const float lo = fminf(top[i], v);
                    v = fmaxf(top[i], v);
                    top[i] = lo;
                }
#pragma unroll
                for (int i = 0; i < kGridMaxK; ++i)
                    if (i == k - 1) kth = top[i];
            }
        }
    };
    for (int rho = 0; rho <= maxr; ++rho) {
        const int z0 = max(cz - rho, 0), z1 = min(cz + rho, g.gz - 1);
        const int y0 = max(cy - rho, 0), y1 = min(cy + rho, g.gy - 1);
        const int x0 = max(cx - rho, 0), x1 = min(cx + rho, g.gx - 1);
        for (int z = z0; z <= z1; ++z) {
            const bool zface = z == cz - rho || z == cz + rho;
            for (int y = y0; y <= y1; ++y) {
                const bool yface = y == cy - rho || y == cy + rho;
                if (zface || yface) {
                    for (int x = x0; x <= x1; ++x) visit(x, y, z);
                } else {
                    if (cx - rho >= 0) visit(cx - rho, y, z);
                    if (rho > 0 && cx + rho < g.gx) visit(cx + rho, y, z);
                }
            }
        }
        const double c = (double)g.c;
        double dmin = side_gap(ar[0], cx - rho, cx + rho, g.gx, g.ox, c);
        dmin = fmin(dmin, side_gap(ar[1], cy - rho, cy + rho, g.gy, g.oy, c));
        dmin = fmin(dmin, side_gap(ar[2], cz - rho, cz + rho, g.gz, g.oz, c));
        if (dmin == INFINITY) break;  // every cell visited
        const double margin = 0x1p-18 * dmin + 0x1p-20 * (double)g.M;
        if ((double)kth < dmin - margin) break;
    }
    theta[r] = kth;
}

__global__ __launch_bounds__(256) void k_knn_cand_grid(const float *boxR, const float *ancR, int nR,
                                                       const float *boxS, const float *ancS, int nS,
                                                       const float *theta, KnnGrid g, const int64_t *beg,
                                                       const int32_t *items, int32_t *count, const int64_t *off,
                                                       int32_t *cs, float *clb, float *cub, int write_pass)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nR) return;
    const float *br = boxR + 6 * (int64_t)r;
    const float th = theta[r];
    int lo[3], hi[3];
    const float o[3] = {g.ox, g.oy, g.oz}, w[3] = {g.wx, g.wy, g.wz};
    const int gd[3] = {g.gx, g.gy, g.gz};
    for (int a = 0; a < 3; ++a) {
        if (!(th < __builtin_inff())) {
            lo[a] = 0;
            hi[a] = gd[a] - 1;
            continue;
        }
        // (the same monotone cell map as the binning; see k_filter_grid)
        const float reach = th + w[a] + 0x1p-18f * g.M;
        lo[a] = grid_coord(br[a] - reach, o[a], g.inv_c, gd[a]);
        hi[a] = grid_coord(br[3 + a] + reach, o[a], g.inv_c, gd[a]);
    }
    int64_t pos = write_pass ? off[r] : 0;
    int total = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y) {
            const int row = (z * g.gy + y) * g.gx;
            for (int64_t q = beg[row + lo[0]]; q < beg[row + hi[0] + 1]; ++q) {
                const int s = items[q];
                const float gp = box_gap(br, boxS + 6 * (int64_t)s) * (1.0f - 0x1p-20f);
                if (gp <= th) {
                    if (write_pass) {
                        cs[pos] = s;
                        clb[pos] = gp;
                        cub[pos] = anchor_ub(ancR + 3 * (int64_t)r, ancS + 3 * (int64_t)s);
                    }
                    ++pos;
                    ++total;
                }
            }
        }
    if (!write_pass) {
        count[r] = total;
        return;
    }
    // insertion sort of r's list by s (lists are short)
    const int64_t b = off[r], e = off[r + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int s = cs[i];
        const float l = clb[i], u = cub[i];
        int64_t j = i - 1;
        while (j >= b && cs[j] > s) {
            cs[j + 1] = cs[j];
            clb[j + 1] = clb[j];
            cub[j + 1] = cub[j];
            --j;
        }
        cs[j + 1] = s;
        clb[j + 1] = l;
        cub[j + 1] = u;
    }
}

// Within-tau MBB filter through the same grid: one thread per r visits the
// cells its box reaches (widened by tau, the widest anchor-to-box extent of S
// and one cell) and applies the all-pairs kernel's test and bounds to each S
// object there; count pass, then write pass in s order per r.  The count
// pass keeps the first kFilterSlots objects it finds for r; the write pass
// skips an r without candidates and takes an r with at most that many from
// its slots (recomputing their bounds), so only busier r revisit the cells.
__global__ __launch_bounds__(256) void k_filter_grid(const float *boxR, const float *ancR, int nR, const float *boxS,
                                                     const float *ancS, float tau, float tau2, KnnGrid g,
                                                     const int64_t *beg, const int32_t *items, int32_t *count,
                                                     int32_t *slot, const int64_t *off, int32_t *cr, int32_t *cs,
                                                     float *clb, float *cub, int write_pass)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nR) return;
    int kept = 0;  // write pass: candidates of r held in its slots (0: visit the cells)
    if (write_pass) {
        const int c = count[r];
        if (c == 0) return;
        if (c <= kFilterSlots) kept = c;
    }
    float b[6];
    for (int c = 0; c < 6; ++c) b[c] = boxR[6 * (int64_t)r + c];
    const float o[3] = {g.ox, g.oy, g.oz}, w[3] = {g.wx, g.wy, g.wz};
    const int gd[3] = {g.gx, g.gy, g.gz};
    int lo[3], hi[3];
    // binning and this range use the same monotone float map from a
    // coordinate to its cell, so an anchor inside the widened box is inside
    // the cell range; the small margin covers the rounding of the widening
    const float margin = 0x1p-18f * g.M;
    for (int a = 0; a < 3; ++a) {
        const float reach = tau + w[a] + margin;
        lo[a] = grid_coord(b[a] - reach, o[a], g.inv_c, gd[a]);
        hi[a] = grid_coord(b[3 + a] + reach, o[a], g.inv_c, gd[a]);
    }
    int64_t pos = write_pass ? off[r] : 0;
    int total = 0;
    int found[kFilterSlots];
    const float ax = ancR[3 * (int64_t)r], ay = ancR[3 * (int64_t)r + 1], az = ancR[3 * (int64_t)r + 2];
    // the box test and, in the write pass, the candidate's bounds
    auto test = [&](const int sidx) {
        const float *x = boxS + 6 * (int64_t)sidx;
        const float gx = fmaxf(0.0f, fmaxf(x[0] - b[3], b[0] - x[3]));
        const float gy = fmaxf(0.0f, fmaxf(x[1] - b[4], b[1] - x[4]));
        const float gz = fmaxf(0.0f, fmaxf(x[2] - b[5], b[2] - x[5]));
        const float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
        if (g2 <= tau2) {
            if (write_pass) {
                const float *sa = ancS + 3 * (int64_t)sidx;
                const float dx = sa[0] - ax, dy = sa[1] - ay, dz = sa[2] - az;
                cr[pos] = r;
                cs[pos] = sidx;
                clb[pos] = __builtin_sqrtf(g2) * (1.0f - 0x1p-20f);
                cub[pos] = __builtin_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) * (1.0f + 0x1p-20f);
            } else if (total < kFilterSlots) {
                found[total] = sidx;
            }
            ++pos;
            ++total;
        }
    };
    if (kept > 0) {
        for (int k = 0; k < kept; ++k) test(slot[(int64_t)kFilterSlots * r + k]);
    } else {
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y) {
                const int row = (z * g.gy + y) * g.gx;
                for (int64_t q = beg[row + lo[0]]; q < beg[row + hi[0] + 1]; ++q) test(items[q]);
            }
    }
    if (!write_pass) {
        count[r] = total;
        if (total <= kFilterSlots)
            for (int k = 0; k < total; ++k) slot[(int64_t)kFilterSlots * r + k] = found[k];
        return;
    }
    // insertion sort of r's candidates by s
    const int64_t b0 = off[r], e0 = off[r + 1];
    for (int64_t i = b0 + 1; i < e0; ++i) {
        const int sv = cs[i];
        const float l = clb[i], u = cub[i];
        int64_t j = i - 1;
        while (j >= b0 && cs[j] > sv) {
            cs[j + 1] = cs[j];
            clb[j + 1] = clb[j];
            cub[j + 1] = cub[j];
            --j;
        }
        cs[j + 1] = sv;
        clb[j + 1] = l;
        cub[j + 1] = u;
    }
}

hipError_t launch_filter_grid(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS,
                              float tau, float tau2, const KnnGrid &g, const int64_t *beg, const int32_t *items,
                              int32_t *count, int32_t *slot, const int64_t *off, int32_t *cr, int32_t *cs, float *clb,
                              float *cub, int write_pass, hipStream_t st)
{
    if (nR == 0) return hipSuccess;
    PJ_GRID_CHECK((nR + 255) / 256, 256);
    hipLaunchKernelGGL(k_filter_grid, dim3((nR + 255) / 256), dim3(256), 0, st, boxR, ancR, nR, boxS, ancS, tau, tau2,
                       g, beg, items, count, slot, off, cr, cs, clb, cub, write_pass);
    return hipGetLastError();
}

hipError_t launch_knn_theta_grid(const float *ancR, int nR, const float *ancS, int nS, int k, const KnnGrid &g,
                                 const int64_t *beg, const int32_t *items, float *theta, hipStream_t st)
{
    if (nR == 0) return hipSuccess;
    if (k < 1 || k > kGridMaxK) return hipErrorInvalidValue;
    PJ_GRID_CHECK((nR + 255) / 256, 256);
    hipLaunchKernelGGL(k_knn_theta_grid, dim3((nR + 255) / 256), dim3(256), 0, st, ancR, nR, ancS, nS, k, g, beg,
                       items, theta);
    return hipGetLastError();
}

hipError_t launch_knn_cand_grid(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS,
                                int nS, const float *theta, const KnnGrid &g, const int64_t *beg,
                                const int32_t *items, int32_t *count, const int64_t *off, int32_t *cs, float *clb,
                                float *cub, int write_pass, hipStream_t st)
{
    if (nR == 0) return hipSuccess;
    PJ_GRID_CHECK((nR + 255) / 256, 256);
    hipLaunchKernelGGL(k_knn_cand_grid, dim3((nR + 255) / 256), dim3(256), 0, st, boxR, ancR, nR, boxS, ancS, nS,
                       theta, g, beg, items, count, off, cs, clb, cub, write_pass);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Voxel-pair filtering (Section 3.2, Algorithms 1 and 2).  One workgroup per
// candidate object pair enumerates its voxel pairs (flattened over the
// workgroup): lb_v = MINDIST of the voxel boxes (FP32, rounded down), ub_v =
// distance of the voxel anchors (surface vertices, rounded up); the pair's
// bounds are the minima over its voxel pairs.  Pruning keeps the voxel pairs
// with lb_v <= ub_o (the object pair's upper bound; for within-tau also
// <= tau), in three kernels: count per pair, exclusive scan, write.  A
// within-tau pair that its own bounds decide (ub_o <= tau or lb_o > tau)
// keeps none.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void vp_bounds(const VoxSide &R, int vr, const VoxSide &S, int vs, float &lb, float &ub)
{
    const float *a = R.vbox + 6 * (int64_t)vr, *b = S.vbox + 6 * (int64_t)vs;
    if (a[0] > a[3] || b[0] > b[3]) {  // an empty voxel (no finest facet)
        lb = ub = __builtin_inff();
        return;
    }
    const float4 alo = make_float4(a[0], a[1], a[2], 0.0f), ahi = make_float4(a[3], a[4], a[5], 0.0f);
    const float4 blo = make_float4(b[0], b[1], b[2], 0.0f), bhi = make_float4(b[3], b[4], b[5], 0.0f);
    lb = box_gap32(alo, ahi, blo, bhi);
    ub = anchor_ub(R.vanc + 3 * (int64_t)vr, S.vanc + 3 * (int64_t)vs);
}

__device__ __forceinline__ bool vp_keep(float lb_v, float op_lb, float op_ub, float tau)
{
    if (tau >= 0.0f) {
        if (op_ub <= tau || op_lb > tau) return false;  // decided by the voxel bounds
        return lb_v <= fminf(op_ub, tau);
    }
    return lb_v <= op_ub;
}

__global__ __launch_bounds__(256) void k_vp_bound(const int32_t *cr, const int32_t *cs, const int64_t *vp_off,
                                                  VoxSide R, VoxSide S, float *vp_lb, float *op_lb, float *op_ub)
{
    __shared__ float sh[8];
    const int p = blockIdx.x;
    const int r = cr[p], s = cs[p];
    const int nr = R.vcount[r], ns = S.vcount[s];
    const int N = nr * ns;
    const int64_t off = vp_off[p];
    float lmin = __builtin_inff(), umin = __builtin_inff();
    for (int t = threadIdx.x; t < N; t += 256) {
        const int i = t / ns, j = t - (t / ns) * ns;
        float lb, ub;
        vp_bounds(R, kMaxVox * r + i, S, kMaxVox * s + j, lb, ub);
        vp_lb[off + t] = lb;  // ub_v is only needed as the pair's minimum
        lmin = fminf(lmin, lb);
        umin = fminf(umin, ub);
    }
    lmin = block_min256(lmin, sh);
    __syncthreads();
    umin = block_min256(umin, sh + 4);
    if (threadIdx.x == 0) {
        op_lb[p] = lmin;
        op_ub[p] = umin;
    }
}

__global__ __launch_bounds__(256) void k_vp_count(const int32_t *cr, const int32_t *cs, const int64_t *vp_off,
                                                  VoxSide R, VoxSide S, const float *vp_lb, const float *op_lb,
                                                  const float *op_ub, float tau, int32_t *count)
{
    __shared__ int sh[4];
    const int p = blockIdx.x;
    const float olb = op_lb[p], oub = op_ub[p];
    if (tau >= 0.0f && (oub <= tau || olb > tau)) {  // decided by its bounds: nothing kept
        if (threadIdx.x == 0) count[p] = 0;
        return;
    }
    const int N = R.vcount[cr[p]] * S.vcount[cs[p]];
    const int64_t off = vp_off[p];
    int c = 0;
    for (int t = threadIdx.x; t < N; t += 256) c += vp_keep(vp_lb[off + t], olb, oub, tau) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) count[p] = sh[0] + sh[1] + sh[2] + sh[3];
}

// survivors as (pair << 12) | (i << 6) | j, pair-major, (i, j) ascending
__global__ __launch_bounds__(256) void k_vp_write(const int32_t *cr, const int32_t *cs, const int64_t *vp_off,
                                                  VoxSide R, VoxSide S, const float *vp_lb, const float *op_lb,
                                                  const float *op_ub, float tau, const int64_t *blk_off,
                                                  uint32_t *vpairs)
{
    __shared__ int sh[256];
    const int p = blockIdx.x;
    const float olb = op_lb[p], oub = op_ub[p];
    if (tau >= 0.0f && (oub <= tau || olb > tau)) return;  // nothing kept (see k_vp_count)
    const int ns = S.vcount[cs[p]];
    const int N = R.vcount[cr[p]] * ns;
    const int64_t off = vp_off[p];
    // each thread owns a contiguous run of the flattened voxel pairs, so the
    // output keeps their order
    const int per = (N + 255) / 256;
    const int t0 = min(N, (int)threadIdx.x * per), t1 = min(N, t0 + per);
    int c = 0;
    for (int t = t0; t < t1; ++t) c += vp_keep(vp_lb[off + t], olb, oub, tau) ? 1 : 0;
    // block-wide exclusive scan of the per-thread counts (Hillis-Steele in LDS)
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int st = 1; st < 256; st <<= 1) {
        const int add = threadIdx.x >= st ? sh[threadIdx.x - st] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t pos = blk_off[p] + sh[threadIdx.x] - c;
    for (int t = t0; t < t1; ++t)
        if (vp_keep(vp_lb[off + t], olb, oub, tau)) {
            const int i = t / ns, j = t - (t / ns) * ns;
            vpairs[pos++] = ((uint32_t)p << 12) | ((uint32_t)i << 6) | (uint32_t)j;
        }
}

hipError_t launch_vp_bound(const int32_t *cr, const int32_t *cs, const int64_t *vp_off, int np, VoxSide R, VoxSide S,
                           float *vp_lb, float *op_lb, float *op_ub, hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    PJ_GRID_CHECK(np, 256);
    hipLaunchKernelGGL(k_vp_bound, dim3(np), dim3(256), 0, st, cr, cs, vp_off, R, S, vp_lb, op_lb, op_ub);
    return hipGetLastError();
}

// The survivors of each pair of a chunk as 64 rows of 64 bits (row i: the S
// voxels paired with R voxel i), built in LDS and written over the
// candidate's rows; a pair without survivors keeps its rows (all pairs).
__global__ __launch_bounds__(256) void k_vp_rows(int row0, const int64_t *blk_off, const uint32_t *vpairs,
                                                 unsigned long long *rows)
{
    __shared__ unsigned long long sh[kMaxVox];
    const int p = blockIdx.x;
    const int64_t b = blk_off[p], e = blk_off[p + 1];
    if (e == b) return;
    if (threadIdx.x < kMaxVox) sh[threadIdx.x] = 0ull;
    __syncthreads();
    for (int64_t t = b + threadIdx.x; t < e; t += 256) {
        const uint32_t x = vpairs[t];
        atomicOr(&sh[(x >> 6) & 63], 1ull << (x & 63));
    }
    __syncthreads();
    if (threadIdx.x < kMaxVox) rows[(size_t)(row0 + p) * kMaxVox + threadIdx.x] = sh[threadIdx.x];
}

hipError_t launch_vp_rows(int row0, int np, const int64_t *blk_off, const uint32_t *vpairs, unsigned long long *rows,
                          hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    PJ_GRID_CHECK(np, 256);
    hipLaunchKernelGGL(k_vp_rows, dim3(np), dim3(256), 0, st, row0, blk_off, vpairs, rows);
    return hipGetLastError();
}

hipError_t launch_vp_count(const int32_t *cr, const int32_t *cs, const int64_t *vp_off, int np, VoxSide R,
                           VoxSide S, const float *vp_lb, const float *op_lb, const float *op_ub, float tau,
                           int32_t *count, hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    PJ_GRID_CHECK(np, 256);
    hipLaunchKernelGGL(k_vp_count, dim3(np), dim3(256), 0, st, cr, cs, vp_off, R, S, vp_lb, op_lb, op_ub, tau, count);
    return hipGetLastError();
}

hipError_t launch_vp_write(const int32_t *cr, const int32_t *cs, const int64_t *vp_off, int np, VoxSide R,
                           VoxSide S, const float *vp_lb, const float *op_lb, const float *op_ub, float tau,
                           const int64_t *blk_off, uint32_t *vpairs, hipStream_t st)
{
    if (np <= 0) return hipSuccess;
    PJ_GRID_CHECK(np, 256);
    hipLaunchKernelGGL(k_vp_write, dim3(np), dim3(256), 0, st, cr, cs, vp_off, R, S, vp_lb, op_lb, op_ub, tau,
                       blk_off, vpairs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-NN object-pair pruning (Algorithm 6, corrected): one workgroup per query
// r.  From a snapshot of the undecided set U and kLeft = k - #confirmed:
//   n surely precedes m  iff  ub_n < lb_m, or ub_n == lb_m and id_n < id_m;
//   CONFIRM m if #{n in U\m : not (m surely precedes n)} < kLeft;
//   REMOVE  m if #{n in U\m : n surely precedes m} >= kLeft.
// Statuses are read from status_in and written to status_out.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_knn_prune(const int64_t *off, const double *lb, const double *ub,
                                                   const int32_t *ids, const int8_t *status_in, int8_t *status_out,
                                                   const int32_t *k_left)
{
    const int r = blockIdx.x;
    const int64_t o = off[r];
    const int N = (int)(off[r + 1] - o);
    const int kl = k_left[r];
    for (int m = threadIdx.x; m < N; m += 256) {
        const int8_t st = status_in[o + m];
        if (st != 0) {
            status_out[o + m] = st;
            continue;
        }
        if (kl <= 0) {
            status_out[o + m] = 2;
            continue;
        }
        const double lbm = lb[o + m], ubm = ub[o + m];
        const int idm = ids[o + m];
        int maybe = 0, surely = 0;
        for (int n = 0; n < N; ++n) {
            if (n == m || status_in[o + n] != 0) continue;
            const double lbn = lb[o + n], ubn = ub[o + n];
            const int idn = ids[o + n];
            const bool m_first = ubm < lbn || (ubm == lbn && idm < idn);
            const bool n_first = ubn < lbm || (ubn == lbm && idn < idm);
            maybe += m_first ? 0 : 1;
            surely += n_first ? 1 : 0;
        }
        status_out[o + m] = maybe < kl ? 1 : (surely >= kl ? 2 : 0);
    }
}

hipError_t launch_knn_prune(int nR, const int64_t *off, const double *lb, const double *ub, const int32_t *ids,
                            const int8_t *status_in, int8_t *status_out, const int32_t *k_left, hipStream_t st)
{
    if (nR == 0) return hipSuccess;
    PJ_GRID_CHECK(nR, 256);
    hipLaunchKernelGGL(k_knn_prune, dim3(nR), dim3(256), 0, st, off, lb, ub, ids, status_in, status_out, k_left);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Facet pairs given explicitly (tests): FP32 with a pair-local origin and the
// guard band 2^-16 M, or FP64 with the exact meet test.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void facet_pair_one(const float *p, const float *q, int prec, double *d, double *d_hi,
                                               int8_t *hit)
{
    if (prec == 0) {
        float lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(fminf(fminf(p[c], p[3 + c]), p[6 + c]), fminf(fminf(q[c], q[3 + c]), q[6 + c]));
            hi[c] = fmaxf(fmaxf(fmaxf(p[c], p[3 + c]), p[6 + c]), fmaxf(fmaxf(q[c], q[3 + c]), q[6 + c]));
        }
        V3 o{0.5f * (lo[0] + hi[0]), 0.5f * (lo[1] + hi[1]), 0.5f * (lo[2] + hi[2])};
        float M = fmaxf(fmaxf(hi[0] - o.x, o.x - lo[0]), fmaxf(fmaxf(hi[1] - o.y, o.y - lo[1]), fmaxf(hi[2] - o.z, o.z - lo[2])));
        float eps = 0x1p-16f * M;
        Rec A = make_rec(V3{p[0], p[1], p[2]} - o, V3{p[3], p[4], p[5]} - o, V3{p[6], p[7], p[8]} - o, 0.0f, 0.0f);
        Rec B = make_rec(V3{q[0], q[1], q[2]} - o, V3{q[3], q[4], q[5]} - o, V3{q[6], q[7], q[8]} - o, 0.0f, 0.0f);
        Pair32 r = pair_f32(A, B, eps);
        // a facet of (numerically) zero area has no plane for the crossing
        // test: its lower estimate is 0, as in the refinement kernel
        *d = r.lo * (A.ok * B.ok);
        *d_hi = r.hi;
        *hit = r.sure ? 1 : 0;
    } else {
        D3 A[3] = {D3{p[0], p[1], p[2]}, D3{p[3], p[4], p[5]}, D3{p[6], p[7], p[8]}};
        D3 B[3] = {D3{q[0], q[1], q[2]}, D3{q[3], q[4], q[5]}, D3{q[6], q[7], q[8]}};
        bool h;
        *d = pair_f64(A, B, h);
        *d_hi = *d;
        *hit = h ? 1 : 0;
    }
}

__global__ void k_facet_pairs(const float *t1, const float *t2, int64_t n, int prec, double *d, double *d_hi,
                              int8_t *hit)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        facet_pair_one(t1 + 9 * i, t2 + 9 * i, prec, d + i, d_hi + i, hit + i);
}

hipError_t launch_facet_pairs(const float *t1, const float *t2, int64_t n, int prec, double *d, double *d_hi,
                              int8_t *hit, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_facet_pairs, dim3((unsigned)std::min<int64_t>((n + 255) / 256, kStrideBlocks)), dim3(256), 0, st,
                       t1, t2, n, prec, d, d_hi, hit);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free entry point: one array per
// device, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address); it
// uses the address hipGetSymbolAddress returns on each device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **out)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace pj
