/*
 * pj.h -- C ABI of the MI355X progressive polyhedral spatial join.
 *
 * Problem (3DPipe, arXiv 2604.19982, Section 3 opening and Section 2.1):
 * objects are closed triangle meshes ("facets" are triangles); the distance
 * of two objects is the minimum Euclidean distance between points of their
 * surfaces.  For object sets R and S the library answers
 *   - intersection:  all (r, s) whose surfaces meet (distance 0),
 *   - within-tau:    all (r, s) with distance <= tau,
 *   - k-NN:          for each r, the k objects of S closest to r.
 * Each object carries a coarse-to-fine sequence of levels of detail (LoDs),
 * the finest being the original mesh (Section 2.1, "Level of Detail").  The
 * join filters candidate pairs by bounding boxes, then refines them LoD by
 * LoD with the facet-level bounds of Eq. (1) and Eq. (2) until every pair
 * is decided (Section 3.1, "Facet-Level Refinement").
 *
 * Conventions for every call:
 *   - every function returns pj_status; nothing throws across the ABI;
 *   - object ids are 0-based indices into R and S;
 *   - all pointers passed in are HOST pointers unless stated otherwise; the
 *     library copies what it keeps, so callers may free inputs on return;
 *   - results are allocated by the library and released with pj_*_free;
 *   - a context belongs to one host thread; mesh sets are immutable and may
 *     be used by any context on the same device;
 *   - on failure, pj_last_error(ctx) describes the cause.
 */
#ifndef PJ_H
#define PJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PJ_OK = 0,
    PJ_ERR_INVALID_ARG = 1,   /* bad pointer, size, index, NaN/Inf coordinate, tau < 0, k < 1, ... */
    PJ_ERR_OUT_OF_MEMORY = 2, /* device allocation failed or the memory cap cannot hold one tile */
    PJ_ERR_DEVICE = 3,        /* a HIP runtime call failed (text in pj_last_error) */
    PJ_ERR_UNSUPPORTED = 4,   /* valid request outside what this build implements */
    PJ_ERR_INTERNAL = 5
} pj_status;

/* Arithmetic of the refinement. */
typedef enum {
    PJ_PREC_FP32_BAND = 0, /* FP32 bulk; pairs within the guard band of the decision are redone in FP64 */
    PJ_PREC_FP64 = 1       /* FP64 for every facet pair */
} pj_precision;

/* How refinement work is scheduled. */
typedef enum {
    PJ_SCHED_BATCHED = 0, /* persistent load-balanced tile queue over all pairs of a LoD round */
    PJ_SCHED_PLAIN = 1    /* one workgroup per (pair, LoD), one launch per LoD (the paper's Algorithm 4) */
} pj_schedule;

/* Device-memory hooks.  alloc returns device memory of at least `bytes`
 * (256-byte aligned) or NULL when it cannot; free returns a block that alloc
 * handed out.  The library waits for all of its queued device work before it
 * calls free, so the caller's allocator may reuse the block at once.  Both
 * are called on the thread that called into the library. */
typedef void *(*pj_alloc_fn)(size_t bytes, void *user);
typedef void (*pj_free_fn)(void *ptr, void *user);

typedef struct {
    int32_t device;          /* HIP device ordinal */
    int32_t precision;       /* pj_precision */
    int32_t schedule;        /* pj_schedule */
    int32_t learned_skip;    /* 1: pick each pair's first LoD with the loaded LoD model (needs model_path) */
    int32_t want_dist;       /* within/intersect: also return FP64 distances of result pairs */
    int32_t use_graph;       /* 1: replay each LoD round's launches from a captured hipGraph */
    int32_t tile_cull;       /* 1: skip facet tiles whose box gap proves they cannot matter */
    int32_t tile_s;          /* streamed-side facets per tile, rounded up to 64 (0: tuned or 1024) */
    int32_t waves_per_cu;    /* persistent grid size in waves per CU (0: tuned or 12) */
    int32_t host_threads;    /* host threads for ingest (0: hardware concurrency) */
    int32_t chunk_tiles;     /* tiles per streamed refinement chunk (0: derived from mem_cap_bytes) */
    int32_t autotune;        /* 1: time candidate (tile_s, waves_per_cu) shapes on a sample of the first
                                round of each work class and keep the fastest (cached in autotune_path);
                                an explicit tile_s / waves_per_cu always wins */
    int32_t mesh_residency;  /* pj_residency of mesh sets created on this context */
    int32_t stage_sets;      /* staging buffer sets for streamed chunks, 2 or 3 (0: 2); 1 runs the chunks one
                                after another with no overlap of gather, copies and compute */
    int32_t filter_mode;     /* MBB filter: 0 auto (grid when |R|*|S| > 2^26, else all pairs), 1 all pairs,
                                2 x sweep, 3 grid over S's anchors (every mode keeps the same candidates).
                                k-NN candidates: 1 all pairs; otherwise a grid over S's anchors when
                                k <= 16 (all pairs for larger k) */
    int32_t knn_prune_host;  /* 1: run the k-NN pruning rule on host threads instead of the GPU kernel (the
                                CPU side of the pruning ablation; results are identical) */
    int64_t mem_cap_bytes;   /* device-memory budget for join work buffers (0: no cap) */
    const char *model_path;  /* LoD model weights written by pj_train_lod_model (NULL: none) */
    const char *log_path;    /* append per-pair resolution records here (NULL: no log) */
    const char *autotune_path; /* autotuner cache file (NULL: none) */
    void *stream;            /* hipStream_t to run on (NULL: the library creates one) */
    pj_alloc_fn dev_alloc;   /* device memory of the context and of the mesh sets created on it
                                (work buffers, ingested facet data); NULL: hipMalloc.  Set both or neither */
    pj_free_fn dev_free;     /* NULL: hipFree */
    void *alloc_user;        /* passed to dev_alloc / dev_free */
    const char *storage_dir; /* PJ_RESIDENT_FILE: directory (on an SSD) for the mesh sets' facet files;
                                copied at context creation */
    int32_t voxels;          /* 1: mesh sets created on this context are voxelized (Section 2.1, k-means
                                over the coarsest facets, at most 64 voxels per object) and the batched
                                joins run voxel-pair filtering (Section 3.2, Algorithms 1-3) before the LoD
                                rounds, which then evaluate only facets of surviving voxel pairs */
    int32_t reserved1;       /* must be 0 */
} pj_config;

/* Where a mesh set's facet data live.  DEVICE: uploaded once at ingest.
 * HOST: kept in host memory; each refinement chunk gathers the facets of
 * its objects at the round's LoD into pinned staging on host threads and
 * uploads them on a copy stream while the previous chunk computes (the
 * paper's pipelined data transfer, Section 4.2 and Algorithm 5).  The device
 * then holds only boxes, anchors and per-LoD maxima of the set, and the
 * streamed chunks are sized by mem_cap_bytes.
 * FILE: as HOST, but the facet data are written to a file in
 * cfg.storage_dir (unlinked at once; it goes away with the set) and read back
 * through a read-only mapping: out-of-core storage for sets larger than host
 * memory (the paper's future work, Section 6).  Each chunk's prep thread asks
 * the kernel to read ahead the next chunk's pages before it gathers its own,
 * so the reads overlap the previous chunk's upload and compute. */
typedef enum { PJ_RESIDENT_DEVICE = 0, PJ_RESIDENT_HOST = 1, PJ_RESIDENT_FILE = 2 } pj_residency;

/* Fill *cfg with defaults: device 0, FP32 band, batched, tile culling on,
 * graphs on, no learned skip, no cap, autotuner off (tile_s 1024, 12 waves
 * per CU), one streamed chunk unless the cap forces more. */
void pj_config_default(pj_config *cfg);

typedef struct pj_context pj_context;
typedef struct pj_meshes pj_meshes;

/* A set of objects (Section 2.1: polyhedra of triangle facets, each with a
 * sequence of LoDs).  Object-major layout; caller-owned, copied on create. */
typedef struct {
    int32_t n_objects;          /* >= 0 */
    int32_t n_lods;             /* L >= 1, the same for every object; LoD 0 coarsest, L-1 original */
    int64_t n_verts;            /* rows of verts */
    int64_t n_tris;             /* rows of tris */
    const float *verts;         /* [n_verts][3] float32 xyz, all objects concatenated */
    const int64_t *vert_begin;  /* [n_objects] first vertex row of each object */
    const int32_t *vert_count;  /* [n_objects] */
    const int32_t *tris;        /* [n_tris][3] vertex indices local to the object's vertex range */
    const int64_t *tri_begin;   /* [n_objects * n_lods] first row of (object, LoD); ranges may alias */
    const int32_t *tri_count;   /* [n_objects * n_lods] */
    const int32_t *parent;      /* [n_tris] for rows of LoD l > 0: index of the parent triangle within the
                                   same object's LoD l-1 list; ignored for LoD 0.  Required when n_lods > 1
                                   and hd/ph are not given */
    const float *hd;            /* optional [n_tris-aligned, per (object, LoD) range via hdph_begin]; NULL:
                                   the library computes hd and ph from the parent maps */
    const float *ph;
    const int64_t *hdph_begin;  /* [n_objects * n_lods] start of each (object, LoD) in hd/ph, when given */
} pj_mesh_desc;

/* Create/destroy a context bound to cfg->device.  cfg NULL = defaults. */
pj_status pj_context_create(const pj_config *cfg, pj_context **out);
pj_status pj_context_destroy(pj_context *ctx);

/* Validate and ingest one object set: copies it to the device and computes
 * per-object MBBs and vertex anchors (Section 2.1, "Object and Voxel
 * Centers"; anchors are always surface vertices) and per-facet hd/ph bounds
 * (Section 2.1, "Facet-Level Hausdorff Bounds") rounded up to float32.
 * Errors: INVALID_ARG for NaN/Inf coordinates, negative counts, indices out
 * of range, parent indices outside the coarser LoD; OUT_OF_MEMORY; DEVICE. */
pj_status pj_meshes_create(pj_context *ctx, const pj_mesh_desc *desc, pj_meshes **out);
pj_status pj_meshes_destroy(pj_meshes *m);

/* Result pairs, sorted by (r, s).  dist is NULL unless cfg.want_dist. */
typedef struct {
    int64_t n;
    int32_t *r;
    int32_t *s;
    double *dist;
} pj_pairs;

/* k-NN result: row-major n_r x k; row r holds count[r] = min(k, |S|) ids of
 * S ordered by (distance, id) and their FP64 distances. */
typedef struct {
    int32_t n_r, k;
    int32_t *count;
    int32_t *s;
    double *dist;
} pj_knn;

/* within-tau join (Section 3, query (2)); tau >= 0 and finite.
 * Meshes must have the same n_lods.  Empty R or S gives n = 0. */
pj_status pj_join_within(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, double tau, pj_pairs *out);
/* intersection join (Section 3, query (1)) == within(0): surfaces meet. */
pj_status pj_join_intersect(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, pj_pairs *out);
/* k-NN join (Section 3, query (3); pruning by Algorithm 6, corrected):
 * k >= 1; k > |S| returns |S| entries per row. */
pj_status pj_join_knn(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int32_t k, pj_knn *out);

void pj_pairs_free(pj_pairs *p);
void pj_knn_free(pj_knn *p);

/* Counters and timings of the last join on this context. */
typedef struct {
    double t_total_ms;          /* host wall time of the join call */
    double t_filter_ms;         /* MBB filter (+ k-NN candidate generation) */
    double t_refine_ms;         /* all LoD rounds incl. classification */
    double t_band_ms;           /* FP64 guard-band recheck and distance finalisation */
    double t_ingest_ms;         /* last pj_meshes_create on this context */
    double refine_kernel_ms;    /* summed device time of the bulk refinement launches (HIP events) */
    double band_kernel_ms;      /* summed device time of the FP64 pair kernel launches */
    int64_t refine_launches;
    int64_t candidates;         /* pairs passing the MBB filter */
    int64_t confirmed_filter;   /* decided by the anchor upper bound alone */
    int64_t facet_pairs;        /* facet pairs evaluated by the bulk refinement kernel */
    int64_t facet_pairs_fp64;   /* facet pairs evaluated in FP64 (plain kernel, band, distances) */
    int64_t tiles;              /* tiles issued to the bulk kernel */
    int64_t tiles_culled;       /* streamed chunks skipped by the box-gap test */
    int64_t band_pairs;         /* object pairs that needed the FP64 recheck */
    int64_t resolved_at_lod[8]; /* pairs decided in each LoD round */
    int64_t rounds;             /* LoD rounds executed */
    int64_t peak_device_bytes;  /* high-water mark of join work buffers */
    int64_t chunks;             /* streamed chunks of the bulk refinement */
    int64_t graph_replays;      /* bulk rounds replayed from a captured hipGraph */
    int64_t tile_s_used;        /* streamed-side tile length (configured or tuned) of the last bulk round;
                                   rounds of few object pairs cut it shorter to fill the GPU */
    int64_t waves_per_cu_used;  /* persistent grid of the last bulk round, waves per CU */
    double t_tune_ms;           /* host time spent in the autotuner during this join */
    int64_t staged_bytes;       /* host-to-device bytes of staged facet data (host-resident sets) */
    int64_t lod_items[8];       /* bulk FP32 work items per LoD round */
    int64_t lod_tiles[8];       /* bulk FP32 tiles per LoD round */
    int64_t lod_pairs[8];       /* facet pairs evaluated by the bulk kernel per LoD round */
    double lod_kernel_ms[8];    /* bulk kernel time per LoD round (HIP events) */
    int64_t collect_launches;   /* FP32 collect passes of the exact recheck (not in refine_*) */
    int64_t collect_pairs;      /* facet pairs they evaluated */
    double collect_kernel_ms;   /* their device time */
    int64_t collected_pairs;    /* facet pairs they kept for the FP64 recheck */
    int64_t collect_overflow;   /* object pairs whose kept pairs overflowed the list (full FP64 pass) */
    int64_t lod_planned_pairs[8]; /* facet pairs of the (pair, LoD) items each LoD round visits, before any
                                     culling (sum of n_r * n_s): fixed by the schedule's decisions alone, not by
                                     tile order or timing */
    int64_t knn_grid_cells;     /* cells of the k-NN candidate grid (0: all-pairs candidates) */
    double t_prune_ms;          /* host wall time of the k-NN pruning rounds (GPU kernel or host threads) */
    double t_prep_ms;           /* host time gathering streamed chunks' facet data (host/file residency), summed
                                   over chunks; it runs on a prep thread beside the upload and compute of the
                                   chunk before */
    int64_t vp_pairs;           /* voxel pairs bounded by the voxel filter */
    int64_t vp_kept;            /* voxel pairs that survived it */
    int64_t vp_chunks;          /* its chunks */
    int64_t voxel_decided;      /* object pairs its bounds decided (within: confirmed or pruned; k-NN: by the
                                   pruning rule on the tightened intervals) */
    double t_voxel_ms;          /* host wall time of the voxel filter */
    double planned_sqrt;        /* sum over the (pair, LoD) items visited of sqrt(n_r * n_s): the work measure
                                   the learned first LoD minimises (with box culling, the facet pairs evaluated
                                   grow like it); fixed by the schedule's decisions */
    int64_t collect_regrow;     /* collect passes run again with a list sized to what the first offered */
} pj_stats;

pj_status pj_get_stats(const pj_context *ctx, pj_stats *out);
const char *pj_last_error(const pj_context *ctx);

/* ------------------------------------------------------------------------
 * Learned LoD skip.  The join, when cfg.log_path is set,
 * appends one record per refined candidate pair: 16 float features and the
 * LoD that decided it.  Training runs the network's forward, backward and
 * Adam kernels on the GPU. */
typedef struct {
    int32_t epochs;
    int32_t batch;
    float lr;
    uint64_t seed;
} pj_train_opts;

pj_status pj_train_lod_model(pj_context *ctx, const char *log_path, const char *model_out,
                             const pj_train_opts *opts, float *final_loss);

/* ------------------------------------------------------------------------
 * Inspection entry points used by tests (all inputs and outputs are host
 * arrays; they run the same device code as the join).
 */
/* Per-object MBB (lo xyz, hi xyz) and anchor (xyz), float32. */
pj_status pj_meshes_boxes(const pj_meshes *m, float *mbb6, float *anchor3);
/* Per-facet hd and ph of one (object, LoD), float32 (0 on the finest LoD). */
pj_status pj_meshes_hdph(const pj_meshes *m, int32_t obj, int32_t lod, float *hd, float *ph);

/* Distance of n triangle pairs (t1[n][9], t2[n][9] float32 corners; the
 * surface distance of Section 2, 0 when the closed triangles meet).
 * precision FP32_BAND: d = lower and d_hi = upper FP32 estimate (equal unless
 * the FP32 crossing test can neither confirm nor exclude a crossing, or a
 * facet has numerically zero area; then d = 0 and d_hi = the vertex-face /
 * edge-edge minimum), hit = 1 where the
 * FP32 test is certain that the triangles cross.  FP64: exact meet test and
 * FP64 distance, d_hi = d.  All arrays are host memory of n entries;
 * PJ_ERR_INVALID_ARG for a null array with n > 0 or another precision. */
pj_status pj_facet_pairs(pj_context *ctx, const float *t1, const float *t2, int64_t n, int32_t precision,
                         double *d, double *d_hi, int8_t *hit);

/* LoD bounds of n object pairs (r[i], s[i]) at one LoD (Eq. (1), Eq. (2)),
 * with the given precision and schedule: lb, ub and the sure-meet flag. */
pj_status pj_pair_bounds(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int64_t n, const int32_t *r,
                         const int32_t *s, int32_t lod, double *lb, double *ub, int8_t *hit);

/* Allocation-free variant of pj_pair_bounds, for callers that cannot
 * allocate device memory (code running under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, layout and
 * results as pj_pair_bounds on a context with precision FP32_BAND and the
 * batched schedule, over device-resident mesh sets; inputs and outputs are
 * host arrays the caller owns.  The work lists live in a fixed 4 MiB device
 * array that the library holds on each device until the process ends; the
 * call makes no device or pinned allocation, no hipMalloc/hipFree and no
 * graph.  Limits: n <= 4096 pairs (INVALID_ARG beyond); UNSUPPORTED for
 * other precisions or schedules and for host-resident sets.  Every call on
 * a device shares that device's array: calls that overlap on one device
 * (from several threads or contexts) race and must be serialised by the
 * caller. */
pj_status pj_pair_bounds_noalloc(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int64_t n,
                                 const int32_t *r, const int32_t *s, int32_t lod, double *lb, double *ub,
                                 int8_t *hit);

/* The LoD-skip network on n feature rows (x[n][16]) with the given
 * parameters (FP32 master copies, layout W1[16][64] b1 W2[64][64] b2 W3[64][4]
 * b3), weights rounded to BF16 as in inference.  logits[n][4]; if y is not
 * NULL also the mean cross-entropy (loss) and FP32 gradients (grads, same
 * layout as params). */
pj_status pj_mlp_eval(pj_context *ctx, const float *params, const float *x, const int32_t *y, int64_t n,
                      float *logits, float *loss, float *grads);

/* Calibration: measured FMA throughput of this device in GFLOP/s (FMA = 2
 * flops) for scalar FP32 (fp64 = 0) or FP64 (fp64 = 1) register-only code. */
pj_status pj_probe_fma(pj_context *ctx, int32_t fp64, double *gflops);
/* Calibration: a plain device-to-device copy of nbytes (multiple of 16) with
 * one kernel launch; returns the achieved read+write bandwidth in GB/s. */
pj_status pj_probe_copy(pj_context *ctx, int64_t nbytes, double *gbps);

#ifdef __cplusplus
}
#endif
#endif /* PJ_H */
