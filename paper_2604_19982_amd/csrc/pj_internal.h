// pj_internal.h -- types shared by the library's host code and kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pj.h"

namespace pj {

// Device view of one ingested object set (object-major).
struct MeshDev {
    const float *verts;    // [V][3]
    const int32_t *tris;   // [T][3] local vertex indices
    const int64_t *vbeg;   // [n] first vertex row
    const int64_t *tbeg;   // [n*L] first triangle row of (object, LoD)
    const int32_t *tcnt;   // [n*L]
    const int64_t *hpbeg;  // [n*L] start of (object, LoD) in hdph, -1 on the finest LoD
    const float2 *hdph;    // (hd, ph) per coarse facet
    const int64_t *bkbeg;  // [n*L] first block record of (object, LoD)
    const float4 *blk;     // per block of 64 consecutive facets: (lo.xyz, max hd), (hi.xyz, max ph)
    int32_t n, L;
    // voxels (null when the set has none): the voxel of every facet of every
    // (object, LoD), and per block record the set of voxels of its facets
    const uint8_t *vlab;               // labels, (object, LoD) ranges from lbeg
    const int64_t *lbeg;               // [n*L]
    const unsigned long long *bmask;   // [blocks] bit v set if a facet of the block is in voxel v
};

// Voxels: at most 64 per object, so that a set of voxels is one 64-bit mask.
constexpr int kMaxVox = 64;

// One refinement work item: an object pair at one LoD.  The facets of the
// "A" object are held in registers, those of "B" are streamed.
struct Item {
    int32_t a_obj, b_obj, lod, flags;
    float ox, oy, oz;  // pair-local origin (float32); coordinates are translated by it
    float eps;         // FP32 guard band of the pair
    float thr;         // collect-mode threshold
    int32_t cand;      // candidate index
    int32_t pad0, pad1;
};
static_assert(sizeof(Item) == 48, "item layout");
enum : int32_t { IT_SWAP = 1, IT_FINEST = 2 };

struct Tile {
    int32_t item, a0, b0, b1;    // A facets from a0, B facets [b0, b1)
    int32_t a1, pad0, pad1, pad2;  // A facets [a0, a1), walked in blocks of 64P
};

// FP32 results of an item: atomically reduced bit patterns of non-negative floats.
struct ItemOut {
    uint32_t lb, ub;
    int32_t hit, done;
};

// FP64 results of an item (bit patterns of non-negative doubles).
struct ItemOut64 {
    unsigned long long lb, ub;
    int32_t hit, pad;
};

// A facet pair kept by the collect pass: (item, A facet, B facet).
struct PairRef {
    int32_t item, a, b, pad;
};

struct RefineArgs {
    MeshDev R, S;
    const Item *items;
    const Tile *tiles;
    const int32_t *ntiles;   // device count (fixed-capacity buffers)
    int32_t *tile_next;      // next tile to take (zeroed by the host before each launch)
    int32_t *tile_cur;       // per tile: next A block to claim (zeroed before each launch)
    int32_t *wave_slot;      // per workgroup: the multi-block tile it owns, -1 if none
    unsigned long long *collected_n;  // collect mode: pairs offered (64-bit, compared with the capacity)
    ItemOut *out;
    unsigned long long *pairs_done;  // facet pairs evaluated (device counter)
    unsigned long long *chunks_culled;
    float tau;               // within-tau threshold for early confirmation; < 0: none
    int32_t early;           // 1: stop an item once it is confirmed
    int32_t cull;            // 1: box-gap test per streamed chunk
    long long collect_cap;   // collect mode: capacity of `collected`
    PairRef *collected;      // collect mode: facet pairs with d_lo <= item.thr
    int32_t *overflow;       // collect mode: per item, 1 if its pairs did not fit
    // voxel pairs that survived the voxel filter: vrow[item.cand] >= 0 picks a
    // block of 64 rows of 64 bits in vmask (row i = the S voxels paired with
    // R voxel i); null, or a negative index: every facet pair counts
    const unsigned long long *vmask;
    const int32_t *vrow;
};

struct Refine64Args {
    MeshDev R, S;
    const Item *items;
    const Tile *tiles;
    ItemOut64 *out;
};

// ---------------------------------------------------------------------------
// kernel launchers (pj_kernels.hip)
// ---------------------------------------------------------------------------
hipError_t launch_boxes(const MeshDev &m, float *box, float *anchor, hipStream_t st);
hipError_t launch_ph(const MeshDev &m, float2 *hdph_mut, const int32_t *parent, const int64_t *fine_job_off,
                     int64_t n_fine_total, hipStream_t st);
hipError_t launch_hd(const MeshDev &m, float2 *hdph_mut, const int64_t *job_off, int64_t n_jobs,
                     const int64_t *desc_base, const int32_t *desc_off, const int32_t *desc_list, int lod, int msub,
                     hipStream_t st);
hipError_t launch_lodmax(const MeshDev &m, float2 *lodmax, hipStream_t st);
hipError_t launch_blocks(const MeshDev &m, float4 *blk, const int64_t *blk_off, int64_t n_blocks, hipStream_t st);
hipError_t launch_filter(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS, int nS,
                         float tau, int32_t *blk_count, int64_t *blk_off, int64_t *total, int32_t *cr, int32_t *cs,
                         float *clb, float *cub, int write_pass, hipStream_t st);
hipError_t launch_filter_sweep(const float *boxR, const float *ancR, const int32_t *rord, int nR, const float *sbox,
                               const float *sanc, const int32_t *sid, const float *sxs, int nS, float tau2,
                               float w_lo, float w_hi, int32_t *blk_count, const int64_t *blk_off, int32_t *cr,
                               int32_t *cs, float *clb, float *cub, int write_pass, hipStream_t st);
hipError_t launch_scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t *total, int n, hipStream_t st);
hipError_t launch_init_round(ItemOut *out, const int32_t *ctr, int32_t *slots, int nslots, int32_t *cur,
                             hipStream_t st);
hipError_t launch_init_out64(ItemOut64 *out, int n, hipStream_t st);

hipError_t launch_refine_f32(const RefineArgs &a, int grid, int P, hipStream_t st);
hipError_t launch_collect_f32(const RefineArgs &a, int grid, hipStream_t st);
hipError_t launch_pairs_f64(const MeshDev &R, const MeshDev &S, const Item *items, const PairRef *pairs, int64_t n,
                            ItemOut64 *out, hipStream_t st);
hipError_t launch_knn_theta(const float *ancR, int nR, const float *ancS, int nS, int k, float *theta, hipStream_t st);
hipError_t launch_knn_cand(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS, int nS,
                           const float *theta, int32_t *count, const int64_t *off, int32_t *cs, float *clb,
                           float *cub, int write_pass, hipStream_t st);
// Uniform grid over the S anchors for the k-NN candidates (host-chosen).
struct KnnGrid {
    float ox, oy, oz;  // origin (lowest corner)
    float c, inv_c;    // cell edge and its reciprocal
    int32_t gx, gy, gz;
    float wx, wy, wz;  // widest anchor-to-box extent of S per axis
    float M;           // largest anchor coordinate magnitude (error margins)
};
constexpr int kGridMaxK = 16;  // k of the grid theta kernel (registers); larger k uses the all-pairs kernels
hipError_t launch_scan_large(const int32_t *in, int64_t *out, int64_t *total, int64_t n, hipStream_t st);
hipError_t launch_grid_build(const float *ancS, int nS, const KnnGrid &g, int32_t *cell_of, int32_t *count,
                             int64_t *beg, int64_t *total, int32_t *fill, int32_t *items, hipStream_t st);
// All-pairs MBB filter: a workgroup tests kFiltR objects of R (one per
// thread) against kFiltS objects of S staged in LDS.
constexpr int kFiltR = 256, kFiltS = 128;

// Grid filter passes.  count: per r (written by the count pass, read by the
// write pass); slot: kFilterSlots per r, the objects the count pass found
// for an r with at most that many.
constexpr int kFilterSlots = 2;
hipError_t launch_filter_grid(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS,
                              float tau, float tau2, const KnnGrid &g, const int64_t *beg, const int32_t *items,
                              int32_t *count, int32_t *slot, const int64_t *off, int32_t *cr, int32_t *cs, float *clb,
                              float *cub, int write_pass, hipStream_t st);
hipError_t launch_knn_theta_grid(const float *ancR, int nR, const float *ancS, int nS, int k, const KnnGrid &g,
                                 const int64_t *beg, const int32_t *items, float *theta, hipStream_t st);
hipError_t launch_knn_cand_grid(const float *boxR, const float *ancR, int nR, const float *boxS, const float *ancS,
                                int nS, const float *theta, const KnnGrid &g, const int64_t *beg,
                                const int32_t *items, int32_t *count, const int64_t *off, int32_t *cs, float *clb,
                                float *cub, int write_pass, hipStream_t st);
// Voxel-pair filtering (Algorithms 1-2) over a chunk of candidate pairs.
struct VoxSide {
    const float *vbox;      // [n*64][6] voxel boxes (lo, hi); empty voxels have lo > hi
    const float *vanc;      // [n*64][3] voxel anchors
    const int32_t *vcount;  // [n] voxels per object
};
hipError_t launch_vp_bound(const int32_t *cr, const int32_t *cs, const int64_t *vp_off, int np, VoxSide R, VoxSide S,
                           float *vp_lb, float *op_lb, float *op_ub, hipStream_t st);
hipError_t launch_vp_rows(int row0, int np, const int64_t *blk_off, const uint32_t *vpairs, unsigned long long *rows,
                          hipStream_t st);
hipError_t launch_vp_count(const int32_t *cr, const int32_t *cs, const int64_t *vp_off, int np, VoxSide R,
                           VoxSide S, const float *vp_lb, const float *op_lb, const float *op_ub, float tau,
                           int32_t *count, hipStream_t st);
hipError_t launch_vp_write(const int32_t *cr, const int32_t *cs, const int64_t *vp_off, int np, VoxSide R,
                           VoxSide S, const float *vp_lb, const float *op_lb, const float *op_ub, float tau,
                           const int64_t *blk_off, uint32_t *vpairs, hipStream_t st);
hipError_t launch_knn_prune(int nR, const int64_t *off, const double *lb, const double *ub, const int32_t *ids,
                            const int8_t *status_in, int8_t *status_out, const int32_t *k_left, hipStream_t st);
hipError_t launch_refine_f64_tiles(const Refine64Args &a, int64_t ntiles, hipStream_t st);
hipError_t launch_refine_f64_plain(const Refine64Args &a, int nitems, hipStream_t st);
hipError_t launch_facet_pairs(const float *t1, const float *t2, int64_t n, int prec, double *d, double *d_hi,
                              int8_t *hit, hipStream_t st);

hipError_t launch_fma_probe(int fp64, void *out, int blocks, int iters, hipStream_t st);
hipError_t launch_copy_probe(const void *src, void *dst, int64_t nbytes, int blocks, hipStream_t st);

// MLP (pj_mlp.hip); scratch holds 4*n*64 + n*4 floats
hipError_t launch_mlp_fwd_bwd(const float *params, const float *x, const int32_t *y, int n, float *logits,
                              float *loss_per, float *grads, float *scratch, hipStream_t st);
hipError_t launch_mlp_adam(float *params, float *m, float *v, const float *grads, int step, float lr, float b1,
                           float b2, float eps, hipStream_t st);
// First LoD of each undecided candidate from the network: its 16 features
// (the bounds below and the two objects' per-LoD facet counts and hd/ph
// maxima), normalised by the model's mean and deviation, the forward pass,
// and the start that minimises the expected work.
struct StartIn {
    int32_t r, s;
    double lb, ub, tau;  // the pair's bounds after the filters and its threshold
};
struct FeatSide {
    const float2 *lodmax;  // [n*L] (max hd, max ph) per (object, LoD)
    const int32_t *tcnt;   // [n*L] facets per (object, LoD)
    int32_t L;
};
hipError_t launch_mlp_start(const float *params, const float *norm, FeatSide R, FeatSide S, const StartIn *in, int n,
                            int32_t *start, hipStream_t st);

// Allocation-free entry point: the device scratch array (one per device,
// 4 MiB) and its layout limits.
constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;
constexpr int kNoAllocMaxPairs = 4096;    // items
constexpr int kNoAllocMaxTiles = 65536;   // tiles
constexpr int kNoAllocMaxGrid = 256 * 64; // persistent workgroups (one slot each)
// Device address of the scratch array on `device` (looked up once per device
// with hipGetSymbolAddress, that device current; cached for the process).
hipError_t scratch_address(int device, void **out);

constexpr int MLP_IN = 16, MLP_H = 64, MLP_OUT = 4;
constexpr int MLP_NPARAM = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H * MLP_OUT + MLP_OUT;

}  // namespace pj
