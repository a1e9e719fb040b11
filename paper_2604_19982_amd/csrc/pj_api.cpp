// pj_api.cpp -- C ABI: contexts, mesh ingest, joins, inspection entry points.
//
// The join follows the filter-and-refine pipeline of 3DPipe (Section 3.1):
// an MBB filter produces candidate pairs with [lb, ub] (MINDIST of the boxes,
// distance of the vertex anchors); then, LoD by LoD from coarse to fine, the
// facet-level bounds of Eq. (1)/(2) are computed for every undecided pair and
// each pair is confirmed (ub <= tau), pruned (lb > tau) or carried to the
// next LoD; the finest LoD is exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <fcntl.h>
#include <sys/mman.h>
#include <unistd.h>

#include "pj_internal.h"

using namespace pj;

namespace {

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Device memory of the library: hipMalloc / hipFree, or the caller's hooks
// (pj_config.dev_alloc / dev_free).  Before a block goes back to the
// caller's allocator every queued device operation is waited for, since that
// allocator may hand the block out again at once.
struct DevAlloc {
    pj_alloc_fn fa = nullptr;
    pj_free_fn ff = nullptr;
    void *user = nullptr;
    hipError_t alloc(void **p, size_t bytes) const
    {
        if (!fa) return hipMalloc(p, bytes);
        *p = fa(bytes, user);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    void free(void *p) const
    {
        if (!p) return;
        if (!ff) {
            (void)hipFree(p);
            return;
        }
        (void)hipDeviceSynchronize();
        ff(p, user);
    }
};

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    int64_t *tracked = nullptr;      // context byte counter
    const DevAlloc *al = nullptr;  // allocator that gave p
    ~DevBuf()
    {
        if (p && al) al->free(p);
    }
    void release()
    {
        if (p && al) al->free(p);
        if (tracked) *tracked -= (int64_t)cap;
        p = nullptr;
        cap = 0;
    }
};

// Device blocks that live only during one call (ingest tables): freed when
// the holder goes out of scope, also on an early error return.
struct TmpDev {
    const DevAlloc &al;
    std::vector<void *> ps;
    explicit TmpDev(const DevAlloc &a) : al(a) {}
    ~TmpDev()
    {
        for (void *p : ps) al.free(p);
    }
    template <class T>
    hipError_t get(T **out, size_t count)
    {
        void *p = nullptr;
        const hipError_t e = al.alloc(&p, std::max<size_t>(count, 1) * sizeof(T));
        *out = static_cast<T *>(p);
        if (e == hipSuccess) ps.push_back(p);
        return e;
    }
};

enum Status : int8_t { ST_UNDEC = 0, ST_CONF = 1, ST_PRUNED = 2, ST_BAND = 3 };

struct Cand {
    int32_t r, s;
    float lb0, ub0;  // filter bounds
};

struct PairState {  // 80 bytes
    int8_t status = ST_UNDEC;
    int8_t lod_done = -1;
    int8_t res_lod = -1;    // LoD round that decided the pair
    int hit64 = 0;
    float eps = 0.0f;
    float ox = 0, oy = 0, oz = 0;
    float thr = INFINITY;   // collect threshold on the FP32 lower distance
    double LB = 0.0, UB = INFINITY;
    double M = 0.0;
    double d64 = INFINITY;  // FP64 finest distance once known
    // bounds when the first LoD was chosen (after the box and voxel
    // filters): the LoD model's gap and upper-bound features
    double f_lb = 0.0, f_ub = INFINITY;
};
static_assert(sizeof(PairState) == 80, "PairState layout");

}  // namespace

struct pj_meshes {
    int device = 0;
    DevAlloc al;  // allocator of the device arrays below
    int32_t n = 0, L = 1;
    int64_t nv = 0, nt = 0, nh = 0;
    float *d_verts = nullptr;
    int32_t *d_tris = nullptr;
    int64_t *d_vbeg = nullptr, *d_tbeg = nullptr, *d_hpbeg = nullptr;
    int32_t *d_tcnt = nullptr;
    float2 *d_hdph = nullptr;
    float *d_box = nullptr, *d_anchor = nullptr;
    float2 *d_lodmax = nullptr;
    int64_t *d_bkbeg = nullptr;
    float4 *d_blk = nullptr;
    int64_t nblk = 0;
    std::vector<int64_t> h_vbeg, h_tbeg, h_hpbeg, h_bkbeg;
    std::vector<int32_t> h_tcnt, h_vcnt;
    std::vector<float> h_box, h_anchor;
    std::vector<float2> h_lodmax;
    // x-sorted copy of the boxes for the sweep filter
    int32_t *d_xord = nullptr;
    float *d_xbox = nullptr, *d_xanc = nullptr, *d_xmin = nullptr;
    double max_w = 0.0, max_abs = 0.0;
    // host-resident sets: facet data in host memory (the device holds only
    // d_box, d_anchor, d_lodmax and the sorted boxes)
    bool host = false;
    std::vector<float> h_verts;
    std::vector<int32_t> h_tris;
    std::vector<float2> h_hdph;
    std::vector<float4> h_blk;
    // where staging reads them: the vectors above, or (file residency) a
    // read-only mapping of an unlinked file in cfg.storage_dir, the vectors
    // then being empty
    const float *p_verts = nullptr;
    const int32_t *p_tris = nullptr;
    const float2 *p_hdph = nullptr;
    const float4 *p_blk = nullptr;
    void *map = nullptr;
    size_t map_len = 0;
    int fd = -1;
    bool file = false;
    // voxels (Section 2.1 "Object Voxelization"): up to 64 per object, slot
    // 64*o + v; labels of every facet of every (object, LoD); per block
    // record the voxels of its facets.  Boxes, anchors and counts are device
    // resident for every residency; labels and block masks follow the facets.
    bool has_vox = false;
    std::vector<int32_t> h_vcount;
    std::vector<float> h_vbox, h_vanc;
    std::vector<uint8_t> h_vlab;
    std::vector<int64_t> h_lbeg;
    std::vector<unsigned long long> h_bmask;
    int32_t *d_vcount = nullptr;
    float *d_vbox = nullptr, *d_vanc = nullptr;
    uint8_t *d_vlab = nullptr;
    int64_t *d_lbeg = nullptr;
    unsigned long long *d_bmask = nullptr;
    MeshDev dev() const
    {
        return MeshDev{d_verts, d_tris, d_vbeg, d_tbeg, d_tcnt, d_hpbeg, d_hdph, d_bkbeg, d_blk, n, L,
                       has_vox ? d_vlab : nullptr, has_vox ? d_lbeg : nullptr, has_vox ? d_bmask : nullptr};
    }
    VoxSide vox() const { return VoxSide{d_vbox, d_vanc, d_vcount}; }
    // grids over the anchors for the filter (k = 1) and the k-NN candidates,
    // built on first use and kept with the set (sets are immutable)
    struct Grid {
        KnnGrid g;
        int64_t ncell = 0;
        int64_t *beg = nullptr;   // [ncell + 1 + tile sums] cell starts
        int32_t *items = nullptr; // [n] object ids by cell
    };
    mutable std::mutex grid_mu;
    mutable std::map<int, Grid> grids;
    int32_t count(int obj, int lod) const { return h_tcnt[(int64_t)obj * L + lod]; }
};

constexpr int kMaxSets = 3;  // staging buffer sets of the streamed rounds

// Persistent host workers for the per-candidate loops of a join (thread
// creation would cost more than the loop).  One job at a time, from the
// thread that owns the context; the caller works on the job too.  Every
// worker takes part in every job (a generation count wakes them) and the
// caller returns only once all of them have finished it, so the job's fields
// never change while a worker reads them.
struct HostPool {
    std::vector<std::thread> th;
    std::mutex m;
    std::condition_variable go, done;
    const std::function<void(int64_t)> *job = nullptr;
    int64_t n = 0, chunk = 1;
    std::atomic<int64_t> next{0};
    uint64_t gen = 0;
    size_t finished = 0;
    bool quit = false;

    explicit HostPool(int workers)
    {
        for (int w = 0; w < workers; ++w)
            th.emplace_back([this] {
                uint64_t seen = 0;
                for (;;) {
                    {
                        std::unique_lock<std::mutex> lk(m);
                        go.wait(lk, [&] { return quit || gen != seen; });
                        if (quit) return;
                        seen = gen;
                    }
                    work();
                    std::lock_guard<std::mutex> lk(m);
                    if (++finished == th.size()) done.notify_all();
                }
            });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(m);
            quit = true;
        }
        go.notify_all();
        for (auto &t : th) t.join();
    }
    void work()
    {
        for (;;) {
            const int64_t i0 = next.fetch_add(chunk);
            if (i0 >= n) return;
            const int64_t i1 = std::min(n, i0 + chunk);
            for (int64_t i = i0; i < i1; ++i) (*job)(i);
        }
    }
    void run(int64_t count, const std::function<void(int64_t)> &f)
    {
        if (count <= 0) return;
        {
            std::lock_guard<std::mutex> lk(m);
            job = &f;
            n = count;
            chunk = std::max<int64_t>(1, count / (int64_t)(8 * (th.size() + 1)));
            next.store(0);
            finished = 0;
            ++gen;
        }
        go.notify_all();
        work();
        std::unique_lock<std::mutex> lk(m);
        done.wait(lk, [&] { return finished == th.size(); });
        job = nullptr;
    }
};

struct pj_context {
    DevAlloc alloc;  // declared first: the work buffers below are freed through it
    double coll_per_item = 0.0;  // pairs the last collect pass offered per item (sizes the next list)
    std::unique_ptr<HostPool> pool;  // created on first use
    pj_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    pj_stats stats;
    int num_cu = 256;
    int64_t dev_bytes = 0, peak_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DevBuf b_fslot;  // the grid filter's per-r slots
    DevBuf b_items, b_tiles, b_out, b_out64, b_ctr, b_cand_r, b_cand_s, b_cand_lb, b_cand_ub, b_blk, b_blkoff,
        b_total, b_tmp0, b_tmp1, b_tmp2, b_tmp3, b_coll, b_ovf, b_theta, b_koff, b_klb, b_kub, b_kst0, b_kst1,
        b_kleft, b_gcell, b_gcnt, b_gfill, b_vplb, b_vpub, b_vmask, b_vrow,
        b_sched, b_model;
    const void *model_dev = nullptr;  // b_model's address when it received the loaded model (weights, feature scales)
    // voxel filter: per set of the double-buffered chunk pipeline, inputs
    // (pairs, voxel-pair offsets) and outputs (pair bounds, counts, offsets,
    // survivors), on the device and pinned
    DevBuf vx_in[2], vx_out[2];
  // scheduling state of the FP32 rounds: workgroup slots, then A-block cursors
    // chunked streaming: two buffer sets, upload/download streams, pinned staging
    struct PinBuf {
        void *p = nullptr;
        size_t cap = 0;
    };
    // A chunk's round data live in one buffer per set, on the device and
    // pinned alike: [results: ci x ItemOut][counters: 256 B][items: ci x Item]
    // [tiles: ct x Tile] for capacities ci and ct, so that a round takes one
    // upload (counters, items, tiles) and one download (results, counters),
    // and the addresses stay fixed while the capacities do (graph keys).
    DevBuf sb_rnd[kMaxSets], sb_stage[kMaxSets];
    PinBuf pin_rnd[kMaxSets], pin_stage[kMaxSets];
    int64_t rcap_i[kMaxSets] = {}, rcap_t[kMaxSets] = {};
    PinBuf pin_cand;  // the filter's candidate count and arrays on their way to the host
    PinBuf pin_start; // the learned skip's inputs up, first LoDs down
    PinBuf pin_vin[2];
    PinBuf pin_vrow;  // the voxel filter's row map up, its pair bounds and survivor counts down
    // a within join's candidates and their states, kept between joins so
    // that their host memory is reused
    std::vector<Cand> j_cand;
    std::vector<PairState> j_ps;
    hipEvent_t ev_vcomp[2] = {};
    const unsigned long long *vmask = nullptr;  // surviving voxel pairs of the join's candidates (device)
    const int32_t *vrow = nullptr;              // per candidate: its block of rows in vmask, -1 for none
    hipStream_t up_stream = nullptr, down_stream = nullptr;
    hipEvent_t ev_h2d[kMaxSets] = {}, ev_comp[kMaxSets] = {}, ev_d2h[kMaxSets] = {}, ev_k0[kMaxSets] = {},
               ev_k1[kMaxSets] = {};
    // launch shape of the bulk rounds: explicit config > tuned > defaults
    struct Shape {
        int tile_s = 1024, wpc = 8;
    };
    Shape cur;
    std::map<std::string, Shape> tuned;
    std::string arch;
    // captured FP32 rounds, keyed by their kernel arguments
    struct GraphEntry {
        std::vector<char> key;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    // LoD model (learned skip)
    std::vector<float> model;
    float feat_mean[MLP_IN], feat_std[MLP_IN];
    bool has_model = false;
    // device address of this device's fixed scratch array (allocation-free
    // entry point), looked up at context creation; null if the lookup failed
    void *scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    std::string storage_dir;  // file residency: where mesh sets spill their facet data
};

namespace {

pj_status fail(pj_context *ctx, pj_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

pj_status hipfail(pj_context *ctx, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? PJ_ERR_OUT_OF_MEMORY : PJ_ERR_DEVICE, m);
}

#define HIPTRY(ctx, expr)                                        \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return hipfail((ctx), e_, #expr);  \
    } while (0)

// grow-only device buffer with the context's memory cap
pj_status ensure(pj_context *ctx, DevBuf &b, size_t bytes, int line = __builtin_LINE())
{
    if (bytes <= b.cap) return PJ_OK;
    size_t nb = std::max(bytes, b.cap + b.cap / 2);
    nb = (nb + 255) & ~size_t(255);
    int64_t after = ctx->dev_bytes - (int64_t)b.cap + (int64_t)nb;
    if (ctx->cfg.mem_cap_bytes > 0 && after > ctx->cfg.mem_cap_bytes) {
        nb = bytes;
        after = ctx->dev_bytes - (int64_t)b.cap + (int64_t)nb;
        if (after > ctx->cfg.mem_cap_bytes)
            return fail(ctx, PJ_ERR_OUT_OF_MEMORY,
                        "work buffers exceed the configured device memory cap (" + std::to_string(bytes) +
                            " bytes requested at pj_api.cpp line " + std::to_string(line) + ", " +
                            std::to_string(ctx->dev_bytes) + " in use, cap " + std::to_string(ctx->cfg.mem_cap_bytes) +
                            ")");
    }
    if (b.p) b.al->free(b.p);
    ctx->dev_bytes -= (int64_t)b.cap;
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = ctx->alloc.alloc(&b.p, nb);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hipfail(ctx, e, "device allocation");
    }
    b.cap = nb;
    b.al = &ctx->alloc;
    b.tracked = &ctx->dev_bytes;
    ctx->dev_bytes += (int64_t)nb;
    ctx->peak_bytes = std::max(ctx->peak_bytes, ctx->dev_bytes);
    return PJ_OK;
}

#define PJTRY(expr)                        \
    do {                                   \
        pj_status s_ = (expr);             \
        if (s_ != PJ_OK) return s_;        \
    } while (0)

template <class T>
T *ptr(DevBuf &b)
{
    return reinterpret_cast<T *>(b.p);
}

// float >= x (smallest float not below x) for x >= 0
float up_float(double x)
{
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

}  // namespace

namespace {
bool load_model(pj_context *ctx, const char *path);
void load_tune_cache(pj_context *ctx);
}

// ===========================================================================
// configuration and contexts
// ===========================================================================
extern "C" void pj_config_default(pj_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->precision = PJ_PREC_FP32_BAND;
    cfg->schedule = PJ_SCHED_BATCHED;
    cfg->learned_skip = 0;
    cfg->want_dist = 0;
    cfg->use_graph = 1;
    cfg->tile_cull = 1;
    cfg->tile_s = 0;
    cfg->waves_per_cu = 0;
}

extern "C" pj_status pj_context_create(const pj_config *cfg, pj_context **out)
{
    if (!out) return PJ_ERR_INVALID_ARG;
    *out = nullptr;
    pj_config c;
    if (cfg) c = *cfg;
    else pj_config_default(&c);
    if (c.precision != PJ_PREC_FP32_BAND && c.precision != PJ_PREC_FP64) return PJ_ERR_INVALID_ARG;
    if (c.schedule != PJ_SCHED_BATCHED && c.schedule != PJ_SCHED_PLAIN) return PJ_ERR_INVALID_ARG;
    if (c.tile_s < 0 || c.waves_per_cu < 0 || c.mem_cap_bytes < 0) return PJ_ERR_INVALID_ARG;
    if ((c.dev_alloc == nullptr) != (c.dev_free == nullptr)) return PJ_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return PJ_ERR_DEVICE;
    if (c.device < 0 || c.device >= ndev) return PJ_ERR_INVALID_ARG;
    if (hipSetDevice(c.device) != hipSuccess) return PJ_ERR_DEVICE;
    pj_context *ctx = new pj_context();
    ctx->cfg = c;
    ctx->alloc = DevAlloc{c.dev_alloc, c.dev_free, c.alloc_user};
    std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) {
        ctx->num_cu = prop.multiProcessorCount;
        ctx->arch = prop.gcnArchName;
        const size_t colon = ctx->arch.find(':');
        if (colon != std::string::npos) ctx->arch.resize(colon);
    }
    if (ctx->arch.empty()) ctx->arch = "gpu";
    if (c.chunk_tiles < 0 || c.filter_mode < 0 || c.filter_mode > 3 || c.knn_prune_host < 0 || c.knn_prune_host > 1 ||
        c.voxels < 0 || c.voxels > 1 || c.reserved1 != 0 ||
        (c.mesh_residency != PJ_RESIDENT_DEVICE && c.mesh_residency != PJ_RESIDENT_HOST &&
         c.mesh_residency != PJ_RESIDENT_FILE) ||
        (c.mesh_residency == PJ_RESIDENT_FILE && (!c.storage_dir || !c.storage_dir[0])) ||
        (c.stage_sets < 0 || c.stage_sets > 3)) {
        delete ctx;
        return PJ_ERR_INVALID_ARG;
    }
    if (c.stream) {
        ctx->stream = (hipStream_t)c.stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return PJ_ERR_DEVICE;
        }
        ctx->own_stream = true;
    }
    if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
        delete ctx;
        return PJ_ERR_DEVICE;
    }
    ctx->scratch_err = scratch_address(c.device, &ctx->scratch);
    if (c.storage_dir) ctx->storage_dir = c.storage_dir;
    ctx->cfg.storage_dir = nullptr;  // the copy above is used
    load_tune_cache(ctx);
    // a missing or unreadable model leaves the plain progressive schedule
    if (c.model_path && !load_model(ctx, c.model_path)) ctx->err = "LoD model not loaded; plain schedule in use";
    *out = ctx;
    return PJ_OK;
}

extern "C" pj_status pj_context_destroy(pj_context *ctx)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->cfg.device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &g : ctx->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (int b = 0; b < kMaxSets; ++b) {
        for (auto *pb : {&ctx->pin_rnd[b], &ctx->pin_stage[b]})
            if (pb->p) (void)hipHostFree(pb->p);
        for (hipEvent_t e : {ctx->ev_h2d[b], ctx->ev_comp[b], ctx->ev_d2h[b], ctx->ev_k0[b], ctx->ev_k1[b]})
            if (e) (void)hipEventDestroy(e);
    }
    if (ctx->pin_cand.p) (void)hipHostFree(ctx->pin_cand.p);
    if (ctx->pin_start.p) (void)hipHostFree(ctx->pin_start.p);
    if (ctx->pin_vrow.p) (void)hipHostFree(ctx->pin_vrow.p);
    for (int b = 0; b < 2; ++b) {
        if (ctx->pin_vin[b].p) (void)hipHostFree(ctx->pin_vin[b].p);
        if (ctx->ev_vcomp[b]) (void)hipEventDestroy(ctx->ev_vcomp[b]);
    }
    if (ctx->up_stream) (void)hipStreamDestroy(ctx->up_stream);
    if (ctx->down_stream) (void)hipStreamDestroy(ctx->down_stream);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return PJ_OK;
}

extern "C" const char *pj_last_error(const pj_context *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" pj_status pj_get_stats(const pj_context *ctx, pj_stats *out)
{
    if (!ctx || !out) return PJ_ERR_INVALID_ARG;
    *out = ctx->stats;
    return PJ_OK;
}

// ===========================================================================
// mesh ingest
// ===========================================================================
namespace {

void free_meshes(pj_meshes *m)
{
    if (!m) return;
    for (void *p : {(void *)m->d_verts, (void *)m->d_tris, (void *)m->d_vbeg, (void *)m->d_tbeg, (void *)m->d_hpbeg,
                    (void *)m->d_tcnt, (void *)m->d_hdph, (void *)m->d_box, (void *)m->d_anchor,
                    (void *)m->d_lodmax, (void *)m->d_bkbeg, (void *)m->d_blk, (void *)m->d_xord, (void *)m->d_xbox,
                    (void *)m->d_xanc, (void *)m->d_xmin, (void *)m->d_vcount, (void *)m->d_vbox, (void *)m->d_vanc,
                    (void *)m->d_vlab, (void *)m->d_lbeg, (void *)m->d_bmask})
        if (p) m->al.free(p);
    for (auto &kv : m->grids) {
        if (kv.second.beg) m->al.free(kv.second.beg);
        if (kv.second.items) m->al.free(kv.second.items);
    }
    if (m->map) munmap(m->map, m->map_len);
    if (m->fd >= 0) close(m->fd);
    delete m;
}

template <class T>
hipError_t dev_new(const DevAlloc &al, T **dst, size_t n)
{
    void *p = nullptr;
    const hipError_t e = al.alloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    *dst = e == hipSuccess ? static_cast<T *>(p) : nullptr;
    return e;
}

template <class T>
hipError_t upload(const DevAlloc &al, T **dst, const T *src, size_t n, hipStream_t st)
{
    hipError_t e = dev_new(al, dst, n);
    if (e != hipSuccess) return e;
    if (n) e = hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, st);
    return e;
}

pj_status validate_desc(pj_context *ctx, const pj_mesh_desc *d)
{
    if (d->n_objects < 0 || d->n_lods < 1 || d->n_lods > 8 || d->n_verts < 0 || d->n_tris < 0)
        return fail(ctx, PJ_ERR_INVALID_ARG, "negative count or n_lods outside 1..8");
    if (d->n_objects == 0) return PJ_OK;
    if (!d->verts && d->n_verts) return fail(ctx, PJ_ERR_INVALID_ARG, "verts is NULL");
    if (!d->tris && d->n_tris) return fail(ctx, PJ_ERR_INVALID_ARG, "tris is NULL");
    if (!d->vert_begin || !d->vert_count || !d->tri_begin || !d->tri_count)
        return fail(ctx, PJ_ERR_INVALID_ARG, "NULL range array");
    const int64_t n = d->n_objects, L = d->n_lods;
    for (int64_t i = 0; i < 3 * d->n_verts; ++i)
        if (!std::isfinite(d->verts[i])) return fail(ctx, PJ_ERR_INVALID_ARG, "NaN or Inf coordinate");
    for (int64_t i = 0; i < n; ++i) {
        if (d->vert_begin[i] < 0 || d->vert_count[i] < 0 || d->vert_begin[i] + d->vert_count[i] > d->n_verts)
            return fail(ctx, PJ_ERR_INVALID_ARG, "vertex range out of bounds");
        for (int64_t l = 0; l < L; ++l) {
            int64_t k = i * L + l;
            if (d->tri_begin[k] < 0 || d->tri_count[k] < 0 || d->tri_begin[k] + d->tri_count[k] > d->n_tris)
                return fail(ctx, PJ_ERR_INVALID_ARG, "triangle range out of bounds");
        }
    }
    // triangle indices (blocks shared by many objects are checked once per vertex count)
    std::set<std::tuple<int64_t, int32_t, int32_t>> seen;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t l = 0; l < L; ++l) {
            int64_t k = i * L + l;
            auto key = std::make_tuple(d->tri_begin[k], d->tri_count[k], d->vert_count[i]);
            if (!seen.insert(key).second) continue;
            const int32_t *t = d->tris + 3 * d->tri_begin[k];
            for (int64_t q = 0; q < 3 * (int64_t)d->tri_count[k]; ++q)
                if (t[q] < 0 || t[q] >= d->vert_count[i])
                    return fail(ctx, PJ_ERR_INVALID_ARG, "triangle vertex index out of range");
        }
    if (L > 1 && !d->hd) {
        if (!d->parent) return fail(ctx, PJ_ERR_INVALID_ARG, "parent maps are required when n_lods > 1");
        std::set<std::tuple<int64_t, int32_t, int32_t>> pseen;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t l = 1; l < L; ++l) {
                int64_t k = i * L + l;
                int32_t nc = d->tri_count[k - 1];
                auto key = std::make_tuple(d->tri_begin[k], d->tri_count[k], nc);
                if (!pseen.insert(key).second) continue;
                const int32_t *p = d->parent + d->tri_begin[k];
                for (int32_t q = 0; q < d->tri_count[k]; ++q)
                    if (p[q] < 0 || p[q] >= nc) return fail(ctx, PJ_ERR_INVALID_ARG, "parent index outside the coarser LoD");
            }
    }
    if (d->hd) {
        if (!d->ph || !d->hdph_begin) return fail(ctx, PJ_ERR_INVALID_ARG, "hd given without ph or hdph_begin");
    }
    return PJ_OK;
}

}  // namespace

namespace {
void host_for(pj_context *ctx, int64_t n, const std::function<void(int64_t)> &f);
}  // namespace

// Voxelization (Section 2.1, "Object Voxelization", "Object and Voxel
// Centers", "Consistent Voxelization across LoDs"), on the host threads at
// ingest.  Per object: k = 2% of its finest facets, at least 1, at most 64
// and at most its coarsest facet count; k-means over the centroids of the
// coarsest facets, the k initial centres being vertices at evenly spaced
// indices, two update steps, then a final assignment (nearest centre, ties
// to the lower index; unused centres dropped).  Every facet of a finer LoD
// takes the voxel of its parent, so the partition is the same at every LoD.
// A voxel's box and anchor come from its finest facets: the box of their
// corners, and the corner nearest the box centre (ties: lowest vertex).
void voxelize(pj_context *ctx, const pj_mesh_desc *d, pj_meshes *m)
{
    const int64_t n = m->n, L = m->L;
    m->has_vox = true;
    m->h_vcount.assign(n, 1);
    m->h_vbox.assign((size_t)n * kMaxVox * 6, 0.0f);
    m->h_vanc.assign((size_t)n * kMaxVox * 3, 0.0f);
    m->h_lbeg.assign(n * L, 0);
    int64_t nl = 0;
    for (int64_t k = 0; k < n * L; ++k) {
        m->h_lbeg[k] = nl;
        nl += m->h_tcnt[k];
    }
    m->h_vlab.assign(nl, 0);
    m->h_bmask.assign(m->nblk, 0ull);
    host_for(ctx, n, [&](int64_t o) {
        const float *V = d->verts + 3 * m->h_vbeg[o];
        const int32_t nv = m->h_vcnt[o];
        auto tri = [&](int64_t l, int32_t f) { return d->tris + 3 * (m->h_tbeg[o * L + l] + f); };
        const int32_t F0 = m->h_tcnt[o * L], Ff = m->h_tcnt[o * L + L - 1];
        int k = (int)std::lround(0.02 * (double)Ff);
        k = std::max(1, std::min(k, std::min(kMaxVox, std::max(F0, 1))));
        if (L > 1 && !d->parent) k = 1;  // no parent maps: one voxel
        uint8_t *lab0 = m->h_vlab.data() + m->h_lbeg[o * L];
        if (k > 1 && nv > 0) {
            std::vector<double> cen(3 * F0), ctr(3 * k);
            for (int32_t f = 0; f < F0; ++f) {
                const int32_t *t = tri(0, f);
                for (int c = 0; c < 3; ++c)
                    cen[3 * f + c] = ((double)V[3 * t[0] + c] + V[3 * t[1] + c] + V[3 * t[2] + c]) / 3.0;
            }
            for (int i = 0; i < k; ++i) {
                const int64_t vi = (int64_t)i * nv / k;
                for (int c = 0; c < 3; ++c) ctr[3 * i + c] = V[3 * vi + c];
            }
            std::vector<int> as(F0);
            auto assign = [&] {
                for (int32_t f = 0; f < F0; ++f) {
                    double best = INFINITY;
                    int bi = 0;
                    for (int i = 0; i < k; ++i) {
                        const double dx = cen[3 * f] - ctr[3 * i], dy = cen[3 * f + 1] - ctr[3 * i + 1],
                                     dz = cen[3 * f + 2] - ctr[3 * i + 2];
                        const double q = dx * dx + dy * dy + dz * dz;
                        if (q < best) {
                            best = q;
                            bi = i;
                        }
                    }
                    as[f] = bi;
                }
            };
            for (int it = 0; it < 2; ++it) {
                assign();
                std::vector<double> sum(3 * k, 0.0);
                std::vector<int> cnt(k, 0);
                for (int32_t f = 0; f < F0; ++f) {
                    cnt[as[f]]++;
                    for (int c = 0; c < 3; ++c) sum[3 * as[f] + c] += cen[3 * f + c];
                }
                for (int i = 0; i < k; ++i)
                    if (cnt[i])
                        for (int c = 0; c < 3; ++c) ctr[3 * i + c] = sum[3 * i + c] / cnt[i];
            }
            assign();
            std::vector<int> remap(k, -1);
            for (int32_t f = 0; f < F0; ++f) remap[as[f]] = 1;
            int used = 0;
            for (int i = 0; i < k; ++i)
                if (remap[i] > 0) remap[i] = used++;
            for (int32_t f = 0; f < F0; ++f) lab0[f] = (uint8_t)remap[as[f]];
            k = used;
        } else {
            k = 1;
        }
        m->h_vcount[o] = k;
        for (int64_t l = 1; l < L; ++l) {
            const uint8_t *up = m->h_vlab.data() + m->h_lbeg[o * L + l - 1];
            uint8_t *lab = m->h_vlab.data() + m->h_lbeg[o * L + l];
            const int32_t nf = m->h_tcnt[o * L + l];
            const int32_t *par = d->parent ? d->parent + m->h_tbeg[o * L + l] : nullptr;
            for (int32_t f = 0; f < nf; ++f) lab[f] = (k > 1 && par) ? up[par[f]] : 0;
        }
        for (int64_t l = 0; l < L; ++l) {
            const uint8_t *lab = m->h_vlab.data() + m->h_lbeg[o * L + l];
            unsigned long long *bm = m->h_bmask.data() + m->h_bkbeg[o * L + l];
            for (int32_t f = 0; f < m->h_tcnt[o * L + l]; ++f) bm[f >> 6] |= 1ull << lab[f];
        }
        // boxes and anchors from the finest facets
        float *box = m->h_vbox.data() + (size_t)o * kMaxVox * 6;
        float *anc = m->h_vanc.data() + (size_t)o * kMaxVox * 3;
        for (int v = 0; v < kMaxVox; ++v)
            for (int c = 0; c < 3; ++c) {
                box[6 * v + c] = INFINITY;
                box[6 * v + 3 + c] = -INFINITY;
            }
        const uint8_t *labf = m->h_vlab.data() + m->h_lbeg[o * L + L - 1];
        for (int32_t f = 0; f < Ff; ++f) {
            const int32_t *t = tri(L - 1, f);
            float *b = box + 6 * labf[f];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) {
                    b[c] = std::min(b[c], V[3 * t[q] + c]);
                    b[3 + c] = std::max(b[3 + c], V[3 * t[q] + c]);
                }
        }
        std::vector<double> best(k, INFINITY);
        std::vector<int32_t> bv(k, INT32_MAX);
        for (int32_t f = 0; f < Ff; ++f) {
            const int32_t *t = tri(L - 1, f);
            const int v = labf[f];
            const float *b = box + 6 * v;
            for (int q = 0; q < 3; ++q) {
                double d2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double x = (double)V[3 * t[q] + c] - 0.5 * ((double)b[c] + (double)b[3 + c]);
                    d2 += x * x;
                }
                if (d2 < best[v] || (d2 == best[v] && t[q] < bv[v])) {
                    best[v] = d2;
                    bv[v] = t[q];
                }
            }
        }
        for (int v = 0; v < k; ++v)
            for (int c = 0; c < 3; ++c) anc[3 * v + c] = bv[v] == INT32_MAX ? 0.0f : V[3 * bv[v] + c];
    });
}

pj_status upload_voxels(pj_context *ctx, pj_meshes *m, bool with_facets)
{
    hipStream_t st = ctx->stream;
    hipError_t e;
    const int64_t n = m->n;
    if ((e = upload(m->al, &m->d_vcount, m->h_vcount.data(), n, st)) != hipSuccess) return hipfail(ctx, e, "voxel counts");
    if ((e = upload(m->al, &m->d_vbox, m->h_vbox.data(), m->h_vbox.size(), st)) != hipSuccess)
        return hipfail(ctx, e, "voxel boxes");
    if ((e = upload(m->al, &m->d_vanc, m->h_vanc.data(), m->h_vanc.size(), st)) != hipSuccess)
        return hipfail(ctx, e, "voxel anchors");
    if (with_facets) {
        if ((e = upload(m->al, &m->d_vlab, m->h_vlab.data(), std::max<size_t>(m->h_vlab.size(), 1), st)) != hipSuccess)
            return hipfail(ctx, e, "voxel labels");
        if ((e = upload(m->al, &m->d_lbeg, m->h_lbeg.data(), m->h_lbeg.size(), st)) != hipSuccess)
            return hipfail(ctx, e, "label offsets");
        if ((e = upload(m->al, &m->d_bmask, m->h_bmask.data(), std::max<size_t>(m->h_bmask.size(), 1), st)) !=
            hipSuccess)
            return hipfail(ctx, e, "block voxel masks");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(ctx, e, "voxel upload");
    if (with_facets) {
        // the host copies of facet-aligned arrays are not needed any more
        std::vector<uint8_t>().swap(m->h_vlab);
        std::vector<unsigned long long>().swap(m->h_bmask);
    }
    return PJ_OK;
}

// Device-resident ingest of a validated description into m (on failure the
// caller frees m).  Boxes, anchors, hd/ph, block records and per-LoD maxima
// are computed on the GPU; host copies of the small per-object arrays stay.
pj_status ingest_device(pj_context *ctx, const pj_mesh_desc *d, pj_meshes *m, bool with_voxels = true)
{
    hipStream_t st = ctx->stream;
    m->device = ctx->cfg.device;
    m->n = d->n_objects;
    m->L = d->n_lods;
    m->nv = d->n_verts;
    m->nt = d->n_tris;
    const int64_t n = m->n, L = m->L;
    auto bail = [&](hipError_t e, const char *what) { return hipfail(ctx, e, what); };
    if (n == 0) return PJ_OK;
    m->h_vcnt.assign(d->vert_count, d->vert_count + n);
    m->h_vbeg.assign(d->vert_begin, d->vert_begin + n);
    m->h_tbeg.assign(d->tri_begin, d->tri_begin + n * L);
    m->h_tcnt.assign(d->tri_count, d->tri_count + n * L);
    // hd/ph layout: one float2 per facet of every coarse LoD
    m->h_hpbeg.assign(n * L, -1);
    int64_t nh = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t l = 0; l + 1 < L; ++l) {
            m->h_hpbeg[i * L + l] = nh;
            nh += m->h_tcnt[i * L + l];
        }
    m->nh = nh;
    hipError_t e;
    if ((e = upload(m->al, &m->d_verts, d->verts, 3 * (size_t)d->n_verts, st)) != hipSuccess) return bail(e, "verts");
    if ((e = upload(m->al, &m->d_tris, d->tris, 3 * (size_t)d->n_tris, st)) != hipSuccess) return bail(e, "tris");
    if ((e = upload(m->al, &m->d_vbeg, m->h_vbeg.data(), n, st)) != hipSuccess) return bail(e, "vert_begin");
    if ((e = upload(m->al, &m->d_tbeg, m->h_tbeg.data(), n * L, st)) != hipSuccess) return bail(e, "tri_begin");
    if ((e = upload(m->al, &m->d_tcnt, m->h_tcnt.data(), n * L, st)) != hipSuccess) return bail(e, "tri_count");
    if ((e = upload(m->al, &m->d_hpbeg, m->h_hpbeg.data(), n * L, st)) != hipSuccess) return bail(e, "hdph_begin");
    if ((e = dev_new(m->al, &m->d_hdph, (size_t)std::max<int64_t>(nh, 1))) != hipSuccess)
        return bail(e, "hdph");
    if ((e = hipMemsetAsync(m->d_hdph, 0, std::max<int64_t>(nh, 1) * sizeof(float2), st)) != hipSuccess)
        return bail(e, "hdph clear");
    if ((e = dev_new(m->al, &m->d_box, n * 6)) != hipSuccess) return bail(e, "boxes");
    if ((e = dev_new(m->al, &m->d_anchor, n * 3)) != hipSuccess) return bail(e, "anchors");
    if ((e = dev_new(m->al, &m->d_lodmax, n * L)) != hipSuccess) return bail(e, "lodmax");
    MeshDev md = m->dev();
    if ((e = launch_boxes(md, m->d_box, m->d_anchor, st)) != hipSuccess) return bail(e, "boxes kernel");

    if (L > 1 && d->hd) {
        // caller-supplied bounds, stored as float2 (hd, ph)
        std::vector<float2> hp(nh);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t l = 0; l + 1 < L; ++l) {
                int64_t src = d->hdph_begin[i * L + l], dst = m->h_hpbeg[i * L + l];
                for (int32_t q = 0; q < m->h_tcnt[i * L + l]; ++q) {
                    float a = d->hd[src + q], b = d->ph[src + q];
                    if (!(a >= 0.0f) || !(b >= 0.0f) || !std::isfinite(a) || !std::isfinite(b))
                        return fail(ctx, PJ_ERR_INVALID_ARG, "hd/ph must be finite and non-negative");
                    hp[dst + q] = make_float2(a, b);
                }
            }
        if ((e = hipMemcpyAsync(m->d_hdph, hp.data(), nh * sizeof(float2), hipMemcpyHostToDevice, st)) != hipSuccess)
            return bail(e, "hdph upload");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "sync");
    } else if (L > 1) {
        // ph: one thread per finest facet
        std::vector<int64_t> fine_off(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) fine_off[i + 1] = fine_off[i] + m->h_tcnt[i * L + L - 1];
        // device tables of this call only (freed on every return)
        TmpDev tmp(m->al);
        int32_t *d_parent = nullptr;
        int64_t *d_off = nullptr;
        if ((e = tmp.get(&d_parent, (size_t)d->n_tris)) != hipSuccess) return bail(e, "parent");
        if (d->n_tris && (e = hipMemcpyAsync(d_parent, d->parent, (size_t)d->n_tris * 4, hipMemcpyHostToDevice, st)) !=
                             hipSuccess)
            return bail(e, "parent");
        if ((e = tmp.get(&d_off, n + 1)) != hipSuccess) return bail(e, "offsets");
        if ((e = hipMemcpyAsync(d_off, fine_off.data(), (n + 1) * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
            return bail(e, "offsets");
        e = launch_ph(md, m->d_hdph, d_parent, d_off, fine_off[n], st);
        if (e != hipSuccess) return bail(e, "ph kernel");
        // hd: descendants of each coarse facet, grouped per distinct connectivity
        std::map<std::vector<int64_t>, int64_t> keymap;  // connectivity -> index into desc_base table
        std::vector<int64_t> desc_base(n * L, 0);        // (obj, lod) -> start in desc_off
        std::vector<int64_t> desc_off;
        std::vector<int32_t> desc_list;
        for (int64_t i = 0; i < n; ++i) {
            std::vector<int64_t> key(2 * L);
            for (int64_t l = 0; l < L; ++l) {
                key[2 * l] = m->h_tbeg[i * L + l];
                key[2 * l + 1] = m->h_tcnt[i * L + l];
            }
            auto it = keymap.find(key);
            if (it == keymap.end()) {
                int64_t slot = (int64_t)desc_off.size();
                const int32_t nf = m->h_tcnt[i * L + L - 1];
                std::vector<int32_t> anc(nf);
                for (int32_t g = 0; g < nf; ++g) anc[g] = g;
                std::vector<int64_t> bases(L, 0);
                for (int64_t l = L - 2; l >= 0; --l) {
                    const int32_t *par = d->parent + m->h_tbeg[i * L + l + 1];
                    for (int32_t g = 0; g < nf; ++g) anc[g] = par[anc[g]];
                    const int32_t nc = m->h_tcnt[i * L + l];
                    bases[l] = (int64_t)desc_off.size();
                    std::vector<int64_t> cnt(nc + 1, 0);
                    for (int32_t g = 0; g < nf; ++g) cnt[anc[g] + 1]++;
                    for (int32_t f = 0; f < nc; ++f) cnt[f + 1] += cnt[f];
                    int64_t lb = (int64_t)desc_list.size();
                    desc_list.resize(lb + nf);
                    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
                    for (int32_t g = 0; g < nf; ++g) desc_list[lb + pos[anc[g]]++] = g;
                    for (int32_t f = 0; f <= nc; ++f) desc_off.push_back(lb + cnt[f]);
                }
                (void)slot;
                it = keymap.emplace(key, (int64_t)keymap.size()).first;
                for (int64_t l = 0; l < L; ++l) desc_base[i * L + l] = bases[l];
                // remember bases for later objects sharing the key
                it->second = i;
            } else {
                int64_t src = it->second;
                for (int64_t l = 0; l < L; ++l) desc_base[i * L + l] = desc_base[src * L + l];
            }
        }
        if (desc_list.size() > (size_t)INT32_MAX || desc_off.size() > (size_t)INT64_MAX)
            return fail(ctx, PJ_ERR_UNSUPPORTED, "descendant tables too large");
        std::vector<int32_t> desc_off32(desc_off.begin(), desc_off.end());
        int64_t *d_dbase = nullptr;
        int32_t *d_doff = nullptr, *d_dlist = nullptr;
        int64_t *d_joboff = nullptr;
        auto tmp_upload = [&](auto **dst, const auto *src, size_t cnt) {
            hipError_t r = tmp.get(dst, cnt);
            if (r == hipSuccess && cnt) r = hipMemcpyAsync(*dst, src, cnt * sizeof(*src), hipMemcpyHostToDevice, st);
            return r;
        };
        if ((e = tmp_upload(&d_dbase, desc_base.data(), desc_base.size())) != hipSuccess) return bail(e, "desc");
        if ((e = tmp_upload(&d_doff, desc_off32.data(), desc_off32.size())) != hipSuccess) return bail(e, "desc");
        if ((e = tmp_upload(&d_dlist, desc_list.data(), desc_list.size())) != hipSuccess) return bail(e, "desc");
        if ((e = tmp.get(&d_joboff, n + 1)) != hipSuccess) return bail(e, "jobs");
        std::vector<std::vector<int64_t>> joboffs(L);
        for (int64_t l = 0; l + 1 < L; ++l) {
            std::vector<int64_t> &jo = joboffs[l];
            jo.assign(n + 1, 0);
            for (int64_t i = 0; i < n; ++i) jo[i + 1] = jo[i] + m->h_tcnt[i * L + l];
            if ((e = hipMemcpyAsync(d_joboff, jo.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st)) !=
                hipSuccess)
                return bail(e, "jobs");
            if ((e = launch_hd(md, m->d_hdph, d_joboff, jo[n], d_dbase, d_doff, d_dlist, (int)l, 8, st)) != hipSuccess)
                return bail(e, "hd kernel");
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "hd sync");
        }
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "ingest sync");
    }
    // block records (64 consecutive facets each) for chunk culling
    m->h_bkbeg.assign(n * L + 1, 0);
    for (int64_t k = 0; k < n * L; ++k) m->h_bkbeg[k + 1] = m->h_bkbeg[k] + (m->h_tcnt[k] + 63) / 64;
    m->nblk = m->h_bkbeg[n * L];
    if ((e = upload(m->al, &m->d_bkbeg, m->h_bkbeg.data(), n * L + 1, st)) != hipSuccess) return bail(e, "block offsets");
    if ((e = dev_new(m->al, &m->d_blk, (size_t)std::max<int64_t>(m->nblk, 1) * 2)) != hipSuccess)
        return bail(e, "block records");
    md = m->dev();
    if ((e = launch_blocks(md, m->d_blk, m->d_bkbeg, m->nblk, st)) != hipSuccess) return bail(e, "blocks kernel");
    if ((e = launch_lodmax(md, m->d_lodmax, st)) != hipSuccess) return bail(e, "lodmax kernel");
    if (ctx->cfg.voxels && with_voxels) {
        voxelize(ctx, d, m);
        PJTRY(upload_voxels(ctx, m, true));
    }
    m->h_box.resize(n * 6);
    m->h_anchor.resize(n * 3);
    m->h_lodmax.resize(n * L);
    if ((e = hipMemcpyAsync(m->h_box.data(), m->d_box, n * 6 * sizeof(float), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return bail(e, "boxes D2H");
    if ((e = hipMemcpyAsync(m->h_anchor.data(), m->d_anchor, n * 3 * sizeof(float), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return bail(e, "anchors D2H");
    if ((e = hipMemcpyAsync(m->h_lodmax.data(), m->d_lodmax, n * L * sizeof(float2), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return bail(e, "lodmax D2H");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "ingest sync");
    return PJ_OK;
}

// Host-resident ingest: the per-object preprocessing runs on the GPU over
// batches of objects (each batch a compact device-resident set of its own,
// released afterwards); hd/ph and block records come back to host memory.
pj_status spill_to_file(pj_context *ctx, pj_meshes *m);

pj_status ingest_host(pj_context *ctx, const pj_mesh_desc *d, pj_meshes *m)
{
    hipStream_t st = ctx->stream;
    m->host = true;
    m->device = ctx->cfg.device;
    m->n = d->n_objects;
    m->L = d->n_lods;
    m->nv = d->n_verts;
    m->nt = d->n_tris;
    const int64_t n = m->n, L = m->L;
    if (n == 0) return PJ_OK;
    m->h_vbeg.assign(d->vert_begin, d->vert_begin + n);
    m->h_vcnt.assign(d->vert_count, d->vert_count + n);
    m->h_tbeg.assign(d->tri_begin, d->tri_begin + n * L);
    m->h_tcnt.assign(d->tri_count, d->tri_count + n * L);
    m->h_verts.assign(d->verts, d->verts + 3 * d->n_verts);
    m->h_tris.assign(d->tris, d->tris + 3 * d->n_tris);
    m->h_hpbeg.assign(n * L, -1);
    int64_t nh = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t l = 0; l + 1 < L; ++l) {
            m->h_hpbeg[i * L + l] = nh;
            nh += m->h_tcnt[i * L + l];
        }
    m->nh = nh;
    m->h_bkbeg.assign(n * L + 1, 0);
    for (int64_t k = 0; k < n * L; ++k) m->h_bkbeg[k + 1] = m->h_bkbeg[k] + (m->h_tcnt[k] + 63) / 64;
    m->nblk = m->h_bkbeg[n * L];
    m->h_hdph.assign(nh, make_float2(0.0f, 0.0f));
    m->h_blk.resize(2 * m->nblk);
    m->h_box.resize(n * 6);
    m->h_anchor.resize(n * 3);
    m->h_lodmax.resize(n * L);
    const int64_t budget =
        ctx->cfg.mem_cap_bytes > 0 ? std::max<int64_t>(ctx->cfg.mem_cap_bytes / 4, int64_t(1) << 20) : int64_t(2) << 30;
    for (int64_t o0 = 0; o0 < n;) {
        // batch [o0, o1): vertices, the distinct triangle ranges, their
        // parents and (when given) the caller's hd/ph
        int64_t o1 = o0, bytes = 0;
        while (o1 < n) {
            int64_t b = 12 * (int64_t)m->h_vcnt[o1] + 64;
            for (int64_t l = 0; l < L; ++l) b += 64 * (int64_t)m->h_tcnt[o1 * L + l] + 64;
            if (o1 > o0 && bytes + b > budget) break;
            bytes += b;
            ++o1;
        }
        const int64_t nb = o1 - o0;
        std::vector<float> sv;
        std::vector<int64_t> svb(nb), stb(nb * L), shb;
        std::vector<int32_t> svc(nb), stc(nb * L), stris, spar;
        std::vector<float> shd, sph;
        std::map<std::pair<int64_t, int32_t>, int64_t> ranges;
        for (int64_t i = 0; i < nb; ++i) {
            const int64_t o = o0 + i;
            svb[i] = (int64_t)sv.size() / 3;
            svc[i] = m->h_vcnt[o];
            sv.insert(sv.end(), d->verts + 3 * m->h_vbeg[o], d->verts + 3 * (m->h_vbeg[o] + m->h_vcnt[o]));
            for (int64_t l = 0; l < L; ++l) {
                const int64_t tb = m->h_tbeg[o * L + l];
                const int32_t tc = m->h_tcnt[o * L + l];
                auto it = ranges.find({tb, tc});
                if (it == ranges.end()) {
                    it = ranges.emplace(std::make_pair(tb, tc), (int64_t)stris.size() / 3).first;
                    stris.insert(stris.end(), d->tris + 3 * tb, d->tris + 3 * (tb + tc));
                    if (d->parent) spar.insert(spar.end(), d->parent + tb, d->parent + tb + tc);
                }
                stb[i * L + l] = it->second;
                stc[i * L + l] = tc;
            }
        }
        if (d->hd) {
            shb.assign(nb * L, 0);
            for (int64_t i = 0; i < nb; ++i)
                for (int64_t l = 0; l + 1 < L; ++l) {
                    const int64_t src = d->hdph_begin[(o0 + i) * L + l];
                    const int32_t tc = stc[i * L + l];
                    shb[i * L + l] = (int64_t)shd.size();
                    shd.insert(shd.end(), d->hd + src, d->hd + src + tc);
                    sph.insert(sph.end(), d->ph + src, d->ph + src + tc);
                }
        }
        pj_mesh_desc sub;
        std::memset(&sub, 0, sizeof(sub));
        sub.n_objects = (int32_t)nb;
        sub.n_lods = (int32_t)L;
        sub.n_verts = (int64_t)sv.size() / 3;
        sub.n_tris = (int64_t)stris.size() / 3;
        sub.verts = sv.data();
        sub.vert_begin = svb.data();
        sub.vert_count = svc.data();
        sub.tris = stris.data();
        sub.tri_begin = stb.data();
        sub.tri_count = stc.data();
        sub.parent = d->parent ? spar.data() : nullptr;
        if (d->hd) {
            sub.hd = shd.data();
            sub.ph = sph.data();
            sub.hdph_begin = shb.data();
        }
        pj_meshes *tmp = new pj_meshes();
        tmp->al = ctx->alloc;
        pj_status s = ingest_device(ctx, &sub, tmp, false);
        if (s == PJ_OK) {
            std::vector<float2> hp(std::max<int64_t>(tmp->nh, 1));
            std::vector<float4> bk(std::max<int64_t>(2 * tmp->nblk, 1));
            hipError_t e = hipMemcpyAsync(hp.data(), tmp->d_hdph, tmp->nh * sizeof(float2), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(bk.data(), tmp->d_blk, 2 * tmp->nblk * sizeof(float4), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                s = hipfail(ctx, e, "host-resident ingest download");
            } else {
                for (int64_t i = 0; i < nb; ++i) {
                    const int64_t o = o0 + i;
                    std::memcpy(&m->h_box[6 * o], &tmp->h_box[6 * i], 6 * sizeof(float));
                    std::memcpy(&m->h_anchor[3 * o], &tmp->h_anchor[3 * i], 3 * sizeof(float));
                    for (int64_t l = 0; l < L; ++l) {
                        const int64_t kf = o * L + l, ks = i * L + l;
                        m->h_lodmax[kf] = tmp->h_lodmax[ks];
                        const int32_t tc = m->h_tcnt[kf];
                        if (l + 1 < L && tc)
                            std::memcpy(&m->h_hdph[m->h_hpbeg[kf]], &hp[tmp->h_hpbeg[ks]], tc * sizeof(float2));
                        const int64_t nbk = (tc + 63) / 64;
                        if (nbk)
                            std::memcpy(&m->h_blk[2 * m->h_bkbeg[kf]], &bk[2 * tmp->h_bkbeg[ks]],
                                        2 * nbk * sizeof(float4));
                    }
                }
            }
        }
        free_meshes(tmp);
        if (s != PJ_OK) return s;
        o0 = o1;
    }
    hipError_t e;
    if ((e = upload(m->al, &m->d_box, m->h_box.data(), 6 * n, st)) != hipSuccess) return hipfail(ctx, e, "boxes");
    if ((e = upload(m->al, &m->d_anchor, m->h_anchor.data(), 3 * n, st)) != hipSuccess) return hipfail(ctx, e, "anchors");
    if ((e = upload(m->al, &m->d_lodmax, m->h_lodmax.data(), n * L, st)) != hipSuccess) return hipfail(ctx, e, "lodmax");
    // facet counts stay on the device too (features of the learned skip)
    if ((e = upload(m->al, &m->d_tcnt, m->h_tcnt.data(), n * L, st)) != hipSuccess) return hipfail(ctx, e, "tri_count");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(ctx, e, "ingest sync");
    if (ctx->cfg.voxels) {
        voxelize(ctx, d, m);
        PJTRY(upload_voxels(ctx, m, false));
    }
    m->p_verts = m->h_verts.data();
    m->p_tris = m->h_tris.data();
    m->p_hdph = m->h_hdph.data();
    m->p_blk = m->h_blk.data();
    if (ctx->cfg.mesh_residency == PJ_RESIDENT_FILE) return spill_to_file(ctx, m);
    return PJ_OK;
}

// Out-of-core storage: the facet data of a host-resident set move to a file
// in cfg.storage_dir (unlinked at once, so it disappears with the set or the
// process) that is mapped read-only; the pages are written back and dropped
// from the page cache, so the join reads them from the device (an SSD)
// while the previous chunk computes.
pj_status spill_to_file(pj_context *ctx, pj_meshes *m)
{
    const std::string tmpl = ctx->storage_dir + "/pj_meshes_XXXXXX";
    std::vector<char> name(tmpl.begin(), tmpl.end());
    name.push_back('\0');
    const int fd = mkstemp(name.data());
    if (fd < 0) return fail(ctx, PJ_ERR_INVALID_ARG, "cannot create a file in storage_dir");
    unlink(name.data());
    m->fd = fd;
    const size_t pg = 4096;
    auto up = [&](size_t x) { return (x + pg - 1) / pg * pg; };
    const size_t b_verts = m->h_verts.size() * sizeof(float), b_tris = m->h_tris.size() * sizeof(int32_t),
                 b_hdph = m->h_hdph.size() * sizeof(float2), b_blk = m->h_blk.size() * sizeof(float4);
    const size_t o_verts = 0, o_tris = up(o_verts + b_verts), o_hdph = up(o_tris + b_tris), o_blk = up(o_hdph + b_hdph),
                 len = std::max(up(o_blk + b_blk), pg);
    if (ftruncate(fd, (off_t)len) != 0) return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "storage_dir: cannot size the file");
    auto put = [&](const void *src, size_t bytes, size_t off) -> bool {
        const char *p = (const char *)src;
        while (bytes > 0) {
            const ssize_t w = pwrite(fd, p, std::min<size_t>(bytes, size_t(1) << 30), (off_t)off);
            if (w <= 0) return false;
            p += w;
            off += (size_t)w;
            bytes -= (size_t)w;
        }
        return true;
    };
    if (!put(m->h_verts.data(), b_verts, o_verts) || !put(m->h_tris.data(), b_tris, o_tris) ||
        !put(m->h_hdph.data(), b_hdph, o_hdph) || !put(m->h_blk.data(), b_blk, o_blk) || fsync(fd) != 0)
        return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "storage_dir: write failed (disk full?)");
    (void)posix_fadvise(fd, 0, (off_t)len, POSIX_FADV_DONTNEED);
    void *map = mmap(nullptr, len, PROT_READ, MAP_SHARED, fd, 0);
    if (map == MAP_FAILED) return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "storage_dir: mmap failed");
    m->map = map;
    m->map_len = len;
    const char *b = (const char *)map;
    m->p_verts = (const float *)(b + o_verts);
    m->p_tris = (const int32_t *)(b + o_tris);
    m->p_hdph = (const float2 *)(b + o_hdph);
    m->p_blk = (const float4 *)(b + o_blk);
    std::vector<float>().swap(m->h_verts);
    std::vector<int32_t>().swap(m->h_tris);
    std::vector<float2>().swap(m->h_hdph);
    std::vector<float4>().swap(m->h_blk);
    m->file = true;
    return PJ_OK;
}

// Ask the kernel to read ahead the file pages of these objects at one LoD
// (file residency; the next chunk's data, while this one is gathered).
void advise_objects(const pj_meshes *m, const std::vector<int32_t> &objs, int lod, bool finest)
{
    if (!m->file) return;
    const uintptr_t pg = 4096;
    auto will = [&](const void *p, size_t bytes) {
        if (!bytes) return;
        const uintptr_t a = (uintptr_t)p & ~(pg - 1), e = ((uintptr_t)p + bytes + pg - 1) & ~(pg - 1);
        (void)madvise((void *)a, e - a, MADV_WILLNEED);
    };
    const int64_t L = m->L;
    for (int o : objs) {
        const int64_t key = (int64_t)o * L + lod;
        const int32_t tc = m->h_tcnt[key];
        will(m->p_verts + 3 * m->h_vbeg[o], 12 * (size_t)m->h_vcnt[o]);
        will(m->p_tris + 3 * m->h_tbeg[key], 12 * (size_t)tc);
        if (!finest) will(m->p_hdph + m->h_hpbeg[key], 8 * (size_t)tc);
        will(m->p_blk + 2 * m->h_bkbeg[key], 32 * (size_t)((tc + 63) / 64));
    }
}

// Boxes sorted by xmin (ties by id) for the sweep filter, with their anchors
// and ids, plus the widest box and the largest coordinate magnitude.
pj_status sort_boxes(pj_context *ctx, pj_meshes *m)
{
    const int64_t n = m->n;
    if (n == 0) return PJ_OK;
    std::vector<int32_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        const float xa = m->h_box[6 * (int64_t)a], xb = m->h_box[6 * (int64_t)b];
        return xa < xb || (xa == xb && a < b);
    });
    std::vector<float> xb(6 * n), xa(3 * n), xm(n);
    double mw = 0.0, ma = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        const float *b = &m->h_box[6 * (int64_t)ord[k]];
        std::copy(b, b + 6, &xb[6 * k]);
        std::copy(&m->h_anchor[3 * (int64_t)ord[k]], &m->h_anchor[3 * (int64_t)ord[k]] + 3, &xa[3 * k]);
        xm[k] = b[0];
        mw = std::max(mw, (double)b[3] - (double)b[0]);
        for (int c = 0; c < 6; ++c) ma = std::max(ma, std::fabs((double)b[c]));
    }
    m->max_w = mw;
    m->max_abs = ma;
    hipStream_t st = ctx->stream;
    hipError_t e;
    if ((e = upload(m->al, &m->d_xord, ord.data(), n, st)) != hipSuccess) return hipfail(ctx, e, "sorted ids");
    if ((e = upload(m->al, &m->d_xbox, xb.data(), 6 * n, st)) != hipSuccess) return hipfail(ctx, e, "sorted boxes");
    if ((e = upload(m->al, &m->d_xanc, xa.data(), 3 * n, st)) != hipSuccess) return hipfail(ctx, e, "sorted anchors");
    if ((e = upload(m->al, &m->d_xmin, xm.data(), n, st)) != hipSuccess) return hipfail(ctx, e, "sorted xmin");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(ctx, e, "sort sync");
    return PJ_OK;
}

extern "C" pj_status pj_meshes_create(pj_context *ctx, const pj_mesh_desc *d, pj_meshes **out)
{
    if (!ctx || !d || !out) return fail(ctx, PJ_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    const double t0 = now_ms();
    PJTRY(validate_desc(ctx, d));
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    pj_meshes *m = new pj_meshes();
    m->al = ctx->alloc;
    pj_status s = ctx->cfg.mesh_residency != PJ_RESIDENT_DEVICE ? ingest_host(ctx, d, m) : ingest_device(ctx, d, m);
    if (s == PJ_OK) s = sort_boxes(ctx, m);
    if (s != PJ_OK) {
        free_meshes(m);
        return s;
    }
    ctx->stats.t_ingest_ms = now_ms() - t0;
    *out = m;
    return PJ_OK;
}

extern "C" pj_status pj_meshes_destroy(pj_meshes *m)
{
    if (!m) return PJ_ERR_INVALID_ARG;
    (void)hipSetDevice(m->device);
    free_meshes(m);
    return PJ_OK;
}

extern "C" pj_status pj_meshes_boxes(const pj_meshes *m, float *mbb6, float *anchor3)
{
    if (!m) return PJ_ERR_INVALID_ARG;
    if (mbb6) std::copy(m->h_box.begin(), m->h_box.end(), mbb6);
    if (anchor3) std::copy(m->h_anchor.begin(), m->h_anchor.end(), anchor3);
    return PJ_OK;
}

extern "C" pj_status pj_meshes_hdph(const pj_meshes *m, int32_t obj, int32_t lod, float *hd, float *ph)
{
    if (!m || obj < 0 || obj >= m->n || lod < 0 || lod >= m->L || !hd || !ph) return PJ_ERR_INVALID_ARG;
    const int64_t k = (int64_t)obj * m->L + lod;
    const int32_t nf = m->h_tcnt[k];
    if (m->h_hpbeg[k] < 0) {
        std::fill(hd, hd + nf, 0.0f);
        std::fill(ph, ph + nf, 0.0f);
        return PJ_OK;
    }
    std::vector<float2> tmp(nf);
    if (m->host) {
        if (nf) std::memcpy(tmp.data(), m->p_hdph + m->h_hpbeg[k], nf * sizeof(float2));
    } else {
        if (hipSetDevice(m->device) != hipSuccess) return PJ_ERR_DEVICE;
        if (nf &&
            hipMemcpy(tmp.data(), m->d_hdph + m->h_hpbeg[k], nf * sizeof(float2), hipMemcpyDeviceToHost) != hipSuccess)
            return PJ_ERR_DEVICE;
    }
    for (int32_t q = 0; q < nf; ++q) {
        hd[q] = tmp[q].x;
        ph[q] = tmp[q].y;
    }
    return PJ_OK;
}

// ===========================================================================
// join machinery
// ===========================================================================
namespace {

constexpr int kP = 1;  // A facets per lane in the FP32 kernel

void pair_frame(const pj_meshes *R, int r, const pj_meshes *S, int s, PairState &ps)
{
    const float *a = &R->h_box[6 * (int64_t)r], *b = &S->h_box[6 * (int64_t)s];
    float lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(a[c], b[c]);
        hi[c] = std::max(a[3 + c], b[3 + c]);
    }
    ps.ox = 0.5f * (lo[0] + hi[0]);
    ps.oy = 0.5f * (lo[1] + hi[1]);
    ps.oz = 0.5f * (lo[2] + hi[2]);
    double M = 0.0;
    const float o[3] = {ps.ox, ps.oy, ps.oz};
    for (int c = 0; c < 3; ++c) M = std::max(M, std::max((double)hi[c] - o[c], (double)o[c] - lo[c]));
    ps.M = M;
    ps.eps = up_float(std::ldexp(M, -16));
    // absolute coordinate scale for FP64 bounds
}

struct TilePlan {
    std::vector<Item> items;
    std::vector<Tile> tiles;
    int64_t pairs = 0;
    int tile_s = 0;
};

// Expand items into tiles: the A side (registers) is the object whose block
// padding wastes less; B ranges are split into chunks of tile_s facets.
// Items are emitted in descending cost order, to within a quarter octave
// (longest processing time first).
void plan_tiles(const pj_meshes *R, const pj_meshes *S, const std::vector<int> &act, const std::vector<Cand> &cand,
                const std::vector<PairState> &ps, int lod, int finest, int BR, int TS, bool allow_swap, TilePlan &pl,
                int64_t target_tiles = 0)
{
    struct C {
        double cost;
        int idx;
    };
    // Largest items first (for the persistent rounds' balance), by a stable
    // counting sort on quarter-octave buckets of the facet-pair count: linear
    // in the item count (a comparison sort of a 30k-item round costs more
    // host time than its planning otherwise), deterministic, and the order
    // within a bucket is the input order.
    const int na = (int)act.size();
    std::vector<C> order(na);
    std::vector<uint8_t> bucket(na);
    int cnt[257] = {0};
    for (int i = 0; i < na; ++i) {
        const Cand &c = cand[act[i]];
        const uint64_t nr = (uint64_t)R->count(c.r, lod), ns = (uint64_t)S->count(c.s, lod);
        const uint64_t q = std::max<uint64_t>(nr * ns, 1);
        const int oct = 63 - __builtin_clzll(q);
        const int sub = oct >= 2 ? (int)((q >> (oct - 2)) & 3) : (int)((q << (2 - oct)) & 3);
        bucket[i] = (uint8_t)(255 - std::min(255, oct * 4 + sub));  // 0 = largest
        cnt[bucket[i] + 1]++;
    }
    for (int k = 0; k < 256; ++k) cnt[k + 1] += cnt[k];
    for (int i = 0; i < na; ++i) {
        const Cand &c = cand[act[i]];
        order[cnt[bucket[i]]++] = C{(double)R->count(c.r, lod) * (double)S->count(c.s, lod), i};
    }
    pl.items.clear();
    pl.tiles.clear();
    pl.pairs = 0;
    pl.tile_s = TS;
    // register side: the object whose block padding wastes less
    auto swapped = [&](int64_t nr, int64_t ns) {
        const int64_t cr = (nr + BR - 1) / BR * BR * ns, cs = (ns + BR - 1) / BR * BR * nr;
        return allow_swap && cs < cr;
    };
    // A side of a tile: one block for the FP64 kernels (a workgroup per
    // tile); the whole A side for the persistent FP32 rounds, whose waves
    // claim a tile's A blocks one at a time and, once the list is used up,
    // join the tiles still in progress (few large tiles cost less setup and
    // still balance)
    const bool whole_a = target_tiles > 0;
    // A round of few object pairs has few claimable units (A block x B
    // range): below about four per wave slot the B ranges are halved until
    // there are (at most down to one chunk), so that the round's waves are not
    // left idle.
    if (whole_a && (int64_t)act.size() < target_tiles / 4) {  // every item is at least one unit
        auto units = [&](int64_t ts) {
            int64_t u = 0;
            for (const C &oc : order) {
                const Cand &c = cand[act[oc.idx]];
                const int64_t nr = R->count(c.r, lod), ns = S->count(c.s, lod);
                const bool sw = swapped(nr, ns);
                const int64_t nA = sw ? ns : nr, nB = sw ? nr : ns;
                u += ((nA + BR - 1) / BR) * ((nB + ts - 1) / ts);
            }
            return u;
        };
        while (TS > 64 && units(TS) < target_tiles / 4) TS = std::max(64, TS / 2 / 64 * 64);
        pl.tile_s = TS;
    }
    for (const C &oc : order) {
        const int ci = act[oc.idx];
        const Cand &c = cand[ci];
        const PairState &p = ps[ci];
        int nr = R->count(c.r, lod), ns = S->count(c.s, lod);
        if (nr == 0 || ns == 0) continue;
        const bool swap = swapped(nr, ns);
        Item it;
        std::memset(&it, 0, sizeof(it));
        it.a_obj = swap ? c.s : c.r;
        it.b_obj = swap ? c.r : c.s;
        it.lod = lod;
        it.flags = (swap ? IT_SWAP : 0) | (finest ? IT_FINEST : 0);
        it.ox = p.ox;
        it.oy = p.oy;
        it.oz = p.oz;
        it.eps = p.eps;
        it.thr = p.thr;
        it.cand = ci;
        const int item = (int)pl.items.size();
        pl.items.push_back(it);
        const int nA = swap ? ns : nr, nB = swap ? nr : ns;
        const int64_t astep = whole_a ? (int64_t)nA : (int64_t)BR;
        for (int64_t a0 = 0; a0 < nA; a0 += astep) {
            const int a1 = (int)std::min<int64_t>(nA, a0 + astep);
            for (int b0 = 0; b0 < nB; b0 += TS)
                pl.tiles.push_back(Tile{item, (int)a0, b0, std::min(nB, b0 + TS), a1, 0, 0, 0});
        }
        pl.pairs += (int64_t)nA * nB;
    }
}

// Work of a LoD round as the schedule planned it: the facet pairs of its
// items before any culling.
void count_planned(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int lod, const TilePlan &pl)
{
    if (lod >= 0 && lod < 8) ctx->stats.lod_planned_pairs[lod] += pl.pairs;
    // the LoD model's cost of these items: sqrt(n_r * n_s) each
    double c = 0.0;
    for (const Item &it : pl.items) {
        const bool sw = it.flags & IT_SWAP;
        c += std::sqrt((double)R->count(sw ? it.b_obj : it.a_obj, lod) * (double)S->count(sw ? it.a_obj : it.b_obj, lod));
    }
    ctx->stats.planned_sqrt += c;
}

// Tile-count hint of the persistent FP32 rounds (any positive value selects
// their whole-A-side tiles; 16 per resident wave).
int64_t tile_target(const pj_context *ctx, int wpc) { return (int64_t)ctx->num_cu * wpc * 16; }
// Rounds are planned for the largest grid the tuner tries, whatever waves
// per CU it picks: the plan a round runs is the plan its shape was timed on.
constexpr int kPlanWPC = 12;

// ---------------------------------------------------------------------------
// Launch-shape autotuner.  Work is classed by (device, mode, size bucket of
// the mean facet pairs per item, item-count bucket, chunk culling on or
// off); the first bulk round of a class without a
// cached shape times every (tile_s, waves_per_cu) candidate on a sample of
// its items (eager launches; wall time of planning plus the streamed round,
// best of two) and keeps the fastest.  Results never depend on the shape: the per-item minima are
// order independent.  The cache is a text file of lines
// "<class> <tile_s> <waves_per_cu> <ms>".
// B ranges below 1024 facets are not offered: on a sample they win by
// parallelism, but over a full round many small tiles of one pair start
// before its running minimum has tightened and cull far less (the finest
// k-NN round of 20k x 20k evaluated 1.6x the pairs at 256).
// ---------------------------------------------------------------------------
constexpr int kTuneTS[] = {1024, 2048, 4096, 8192, 16384};
// waves per CU: the refinement kernel holds two waves per SIMD (eight per
// CU), so a larger grid only queues waves that find the list used up
// waves per CU: at most 12, the refinement kernel's residency (3 per SIMD),
// so that no wave of the persistent grid starts late
constexpr int kTuneWPC[] = {4, 8, 12};

void load_tune_cache(pj_context *ctx)
{
    if (!ctx->cfg.autotune_path) return;
    FILE *f = std::fopen(ctx->cfg.autotune_path, "r");
    if (!f) return;
    char key[256];
    int ts, wpc;
    double ms;
    while (std::fscanf(f, "%255s %d %d %lf", key, &ts, &wpc, &ms) == 4)
        if (ts >= 64 && ts % 64 == 0 && ts <= (1 << 20) && wpc >= 1 && wpc <= 64)
            ctx->tuned[key] = pj_context::Shape{ts, wpc};
    std::fclose(f);
}

void save_tune_cache(pj_context *ctx, const std::string &key, const pj_context::Shape &sh, double ms)
{
    if (!ctx->cfg.autotune_path) return;
    FILE *f = std::fopen(ctx->cfg.autotune_path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %.6f\n", key.c_str(), sh.tile_s, sh.wpc, ms);
    std::fclose(f);
}

std::string tune_class(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, const std::vector<int> &act,
                       const std::vector<Cand> &cand, int lod, float tau)
{
    double sum = 0.0;
    for (int i : act) sum += (double)R->count(cand[i].r, lod) * (double)S->count(cand[i].s, lod);
    const double mean = act.empty() ? 0.0 : sum / (double)act.size();
    const int bucket = mean > 1.0 ? (int)std::floor(std::log(mean) / std::log(4.0)) : 0;
    // and the round's size: a few large items and thousands of them want
    // different tiles and grids even at the same mean
    const int nbucket = act.size() > 1 ? (int)std::floor(std::log((double)act.size()) / std::log(4.0)) : 0;
    // rounds without chunk culling evaluate every planned pair: their own class
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s/%dcu/%s/b%d/n%d%s", ctx->arch.c_str(), ctx->num_cu,
                  tau >= 0.0f ? "within" : "min", bucket, nbucket, ctx->cfg.tile_cull ? "" : "/nocull");
    return buf;
}

pj_status run_f32(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, TilePlan &pl, float tau, bool early,
                  std::vector<ItemOut> &out, int wpc_override);

// Set ctx->cur for a bulk round over `act` (explicit config values win).
pj_status choose_shape(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, const std::vector<int> &act,
                       const std::vector<Cand> &cand, const std::vector<PairState> &ps, int lod, int finest,
                       float tau, bool early)
{
    const int cfg_ts = ctx->cfg.tile_s > 0 ? (ctx->cfg.tile_s + 63) / 64 * 64 : 0;
    const int cfg_wpc = ctx->cfg.waves_per_cu;
    pj_context::Shape sh;
    if (cfg_ts && cfg_wpc) {
        ctx->cur = pj_context::Shape{cfg_ts, cfg_wpc};
        return PJ_OK;
    }
    const std::string key = tune_class(ctx, R, S, act, cand, lod, tau);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) {
        sh = it->second;
    } else if (ctx->cfg.autotune && !act.empty()) {
        const double t0 = now_ms();
        // The candidates are timed on the round itself when it plans at most
        // 2e11 facet pairs (a tenth of that typically survives culling, so a
        // timing costs milliseconds); a larger round is sampled evenly down
        // to about that.  A sample of a few items would need more splitting
        // than the round to fill the GPU and so favour short B ranges.
        std::vector<int> idx(act.begin(), act.end());
        std::vector<int> sample;
        double pairs = 0.0, total = 0.0;
        for (int i : idx) total += (double)R->count(cand[i].r, lod) * (double)S->count(cand[i].s, lod);
        // without culling every planned pair is evaluated: a tenth of the sample
        const double budget = ctx->cfg.tile_cull ? 2e11 : 2e10;
        const size_t stride = std::max<size_t>(1, (size_t)std::ceil(total / budget));
        for (size_t i = 0; i < idx.size() && pairs < budget; i += stride) {
            sample.push_back(idx[i]);
            pairs += (double)R->count(cand[idx[i]].r, lod) * (double)S->count(cand[idx[i]].s, lod);
        }
        const pj_stats saved = ctx->stats;
        double best = INFINITY, t_default = INFINITY;
        pj_context::Shape bs;
        const pj_context::Shape def{};
        std::vector<int> ts_list(std::begin(kTuneTS), std::end(kTuneTS)), wpc_list(std::begin(kTuneWPC), std::end(kTuneWPC));
        if (cfg_ts) ts_list.assign(1, cfg_ts);  // an explicit value is the only candidate
        if (cfg_wpc) wpc_list.assign(1, cfg_wpc);
        for (int ts : ts_list) {
            // wall time of planning + the streamed round (host work per tile
            // counts as much as the kernel when items have many tiles)
            const double tp = now_ms();
            TilePlan pl;
            plan_tiles(R, S, sample, cand, ps, lod, finest, 64 * kP, ts, true, pl, tile_target(ctx, kPlanWPC));
            const double plan_ms = now_ms() - tp;
            // waves per CU from the most down: a smaller count must be 3%
            // faster to be taken.  A round of fewer units than the smaller
            // grids launches the same waves for every count (the grid per
            // round), so its timings tie, and the larger count keeps the
            // class's bigger rounds (and its tile plan) from running short
            // of waves.
            double best_ts = INFINITY;
            int wpc_ts = 0;
            for (auto w = wpc_list.rbegin(); w != wpc_list.rend(); ++w) {
                const int wpc = *w;
                double t = INFINITY;
                for (int rep = 0; rep < 3; ++rep) {
                    std::vector<ItemOut> out;
                    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
                    const double tr = now_ms();
                    PJTRY(run_f32(ctx, R, S, pl, tau, early, out, wpc));
                    t = std::min(t, plan_ms + (now_ms() - tr));
                }
                if (t < (wpc_ts ? 0.97 * best_ts : INFINITY)) {
                    best_ts = t;
                    wpc_ts = wpc;
                }
                if (ts == def.tile_s && wpc == def.wpc) t_default = t;
            }
            if (best_ts < best) {
                best = best_ts;
                bs = pj_context::Shape{ts, wpc_ts};
            }
        }
        // within 3% the default wins: run-to-run timing noise should not
        // move the shape
        if (t_default <= 1.03 * best) {
            bs = def;
            best = t_default;
        }
        ctx->stats = saved;
        ctx->stats.t_tune_ms += now_ms() - t0;
        sh = bs;
        ctx->tuned[key] = sh;
        save_tune_cache(ctx, key, sh, best);
    }
    if (cfg_ts) sh.tile_s = cfg_ts;
    if (cfg_wpc) sh.wpc = cfg_wpc;
    ctx->cur = sh;
    return PJ_OK;
}

pj_status ensure_pinned(pj_context *ctx, pj_context::PinBuf &b, size_t bytes)
{
    if (bytes <= b.cap) return PJ_OK;
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    size_t nb = std::max<size_t>(bytes, 4096);
    nb = std::max(nb, b.cap + b.cap / 2);
    hipError_t e = hipHostMalloc(&b.p, nb, hipHostMallocDefault);
    if (e != hipSuccess) return hipfail(ctx, e, "hipHostMalloc");
    b.cap = nb;
    return PJ_OK;
}

pj_status ensure_streams(pj_context *ctx)
{
    if (ctx->up_stream) return PJ_OK;
    HIPTRY(ctx, hipStreamCreateWithFlags(&ctx->up_stream, hipStreamNonBlocking));
    HIPTRY(ctx, hipStreamCreateWithFlags(&ctx->down_stream, hipStreamNonBlocking));
    for (int b = 0; b < kMaxSets; ++b) {
        HIPTRY(ctx, hipEventCreateWithFlags(&ctx->ev_h2d[b], hipEventDisableTiming));
        HIPTRY(ctx, hipEventCreateWithFlags(&ctx->ev_comp[b], hipEventDisableTiming));
        HIPTRY(ctx, hipEventCreateWithFlags(&ctx->ev_d2h[b], hipEventDisableTiming));
        HIPTRY(ctx, hipEventCreate(&ctx->ev_k0[b]));
        HIPTRY(ctx, hipEventCreate(&ctx->ev_k1[b]));
    }
    return PJ_OK;
}

// ---------------------------------------------------------------------------
// Staging of host-resident facet data.  The objects a chunk needs from one
// side are packed, at the chunk's LoD, as a mesh set of their own (same
// arrays as a device-resident set, one buffer, rows renumbered; triangle
// ranges shared by several objects are staged once), so the kernels read
// staged and resident sets alike.  Only the round's LoD entries of the
// per-(object, LoD) arrays are filled.
// ---------------------------------------------------------------------------
struct SideStage {
    int lod = 0;
    bool finest = false;
    std::vector<int32_t> objs;                  // original ids, in local order
    std::vector<int64_t> vdst, tdst, hdst, bdst;  // staged first rows per object
    std::vector<char> tcopy;                    // object copies its triangle range
    int64_t V = 0, T = 0, H = 0, B = 0;
    std::vector<int64_t> ldst;  // staged first label row per object (voxels)
    int64_t NL = 0;
    size_t o_verts = 0, o_tris = 0, o_vbeg = 0, o_tbeg = 0, o_tcnt = 0, o_hpbeg = 0, o_hdph = 0, o_bkbeg = 0,
           o_blk = 0, o_lbeg = 0, o_vlab = 0, o_bmask = 0, end = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int64_t kStageFixed = 13 * 256;

// staged bytes of one object at one LoD (an upper bound: no range sharing)
int64_t stage_obj_bytes(const pj_meshes *m, int obj, int lod, bool finest)
{
    const int64_t tc = m->count(obj, lod);
    return 12 * (int64_t)m->h_vcnt[obj] + 12 * tc + (finest ? 0 : 8 * tc) + 32 * ((tc + 63) / 64) + 8 +
           28 * (int64_t)m->L + 5 * 256 / 64 + (m->has_vox ? tc + 8 * ((tc + 63) / 64) + 8 * (int64_t)m->L + 3 * 256 / 64 : 0);
}

void stage_plan(const pj_meshes *m, SideStage &s, size_t base)
{
    const int64_t n = (int64_t)s.objs.size(), L = m->L;
    s.vdst.resize(n);
    s.tdst.resize(n);
    s.hdst.resize(n);
    s.bdst.resize(n);
    s.tcopy.assign(n, 0);
    s.ldst.assign(n, 0);
    s.NL = 0;
    std::unordered_map<int64_t, std::pair<int32_t, int64_t>> rows;  // source row -> (count, staged row)
    s.V = s.T = s.H = s.B = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int o = s.objs[k];
        const int64_t key = (int64_t)o * L + s.lod;
        const int64_t tb = m->h_tbeg[key];
        const int32_t tc = m->h_tcnt[key];
        s.vdst[k] = s.V;
        s.V += m->h_vcnt[o];
        auto it = rows.find(tb);
        if (it != rows.end() && it->second.first == tc) {
            s.tdst[k] = it->second.second;
        } else {
            s.tdst[k] = s.T;
            s.tcopy[k] = 1;
            rows[tb] = {tc, s.T};
            s.T += tc;
        }
        s.hdst[k] = s.finest ? -1 : s.H;
        if (!s.finest) s.H += tc;
        s.bdst[k] = s.B;
        s.B += (tc + 63) / 64;
        s.ldst[k] = s.NL;
        if (m->has_vox) s.NL += tc;
    }
    size_t off = base;
    auto put = [&](size_t &o, size_t bytes) {
        o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
    };
    put(s.o_verts, 12 * s.V);
    put(s.o_tris, 12 * s.T);
    put(s.o_vbeg, 8 * n);
    put(s.o_tbeg, 8 * n * L);
    put(s.o_tcnt, 4 * n * L);
    put(s.o_hpbeg, 8 * n * L);
    put(s.o_hdph, 8 * s.H);
    put(s.o_bkbeg, 8 * (n * L + 1));
    put(s.o_blk, 32 * s.B);
    if (m->has_vox) {
        put(s.o_lbeg, 8 * n * L);
        put(s.o_vlab, (size_t)s.NL);
        put(s.o_bmask, 8 * s.B);
    }
    s.end = off;
}

template <class F>
void parallel_for(int64_t n, int nthreads, F f)
{
    if (n <= 0) return;
    nthreads = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, n / 16));
    if (nthreads <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
        th.emplace_back([=, &f] {
            for (int64_t i = t; i < n; i += nthreads) f(i);
        });
    for (auto &x : th) x.join();
}

void stage_fill(const pj_meshes *m, const SideStage &s, char *base, int nthreads)
{
    const int64_t n = (int64_t)s.objs.size(), L = m->L;
    float *verts = reinterpret_cast<float *>(base + s.o_verts);
    int32_t *tris = reinterpret_cast<int32_t *>(base + s.o_tris);
    int64_t *vbeg = reinterpret_cast<int64_t *>(base + s.o_vbeg);
    int64_t *tbeg = reinterpret_cast<int64_t *>(base + s.o_tbeg);
    int32_t *tcnt = reinterpret_cast<int32_t *>(base + s.o_tcnt);
    int64_t *hpbeg = reinterpret_cast<int64_t *>(base + s.o_hpbeg);
    float2 *hdph = reinterpret_cast<float2 *>(base + s.o_hdph);
    int64_t *bkbeg = reinterpret_cast<int64_t *>(base + s.o_bkbeg);
    float4 *blk = reinterpret_cast<float4 *>(base + s.o_blk);
    for (int64_t k = 0; k < n; ++k) {
        vbeg[k] = s.vdst[k];
        for (int64_t l = 0; l < L; ++l) {
            const bool here = l == s.lod;
            tbeg[k * L + l] = here ? s.tdst[k] : 0;
            tcnt[k * L + l] = here ? m->h_tcnt[(int64_t)s.objs[k] * L + l] : 0;
            hpbeg[k * L + l] = here ? s.hdst[k] : -1;
            bkbeg[k * L + l] = here ? s.bdst[k] : 0;
        }
    }
    bkbeg[n * L] = s.B;
    if (m->has_vox) {
        int64_t *lbeg = reinterpret_cast<int64_t *>(base + s.o_lbeg);
        for (int64_t k = 0; k < n; ++k)
            for (int64_t l = 0; l < L; ++l) lbeg[k * L + l] = l == s.lod ? s.ldst[k] : 0;
    }
    parallel_for(n, nthreads, [&](int64_t k) {
        const int o = s.objs[k];
        const int64_t key = (int64_t)o * L + s.lod;
        const int32_t tc = m->h_tcnt[key];
        std::memcpy(verts + 3 * s.vdst[k], m->p_verts + 3 * m->h_vbeg[o], 12 * (size_t)m->h_vcnt[o]);
        if (s.tcopy[k]) std::memcpy(tris + 3 * s.tdst[k], m->p_tris + 3 * m->h_tbeg[key], 12 * (size_t)tc);
        if (!s.finest && tc) std::memcpy(hdph + s.hdst[k], m->p_hdph + m->h_hpbeg[key], 8 * (size_t)tc);
        const int64_t nb = (tc + 63) / 64;
        if (nb) std::memcpy(blk + 2 * s.bdst[k], m->p_blk + 2 * m->h_bkbeg[key], 32 * (size_t)nb);
        if (m->has_vox) {
            if (tc) std::memcpy(base + s.o_vlab + s.ldst[k], m->h_vlab.data() + m->h_lbeg[key], (size_t)tc);
            if (nb)
                std::memcpy(reinterpret_cast<unsigned long long *>(base + s.o_bmask) + s.bdst[k],
                            m->h_bmask.data() + m->h_bkbeg[key], 8 * (size_t)nb);
        }
    });
}

MeshDev stage_view(const pj_meshes *m, const SideStage &s, char *dbase)
{
    return MeshDev{reinterpret_cast<const float *>(dbase + s.o_verts),
                   reinterpret_cast<const int32_t *>(dbase + s.o_tris),
                   reinterpret_cast<const int64_t *>(dbase + s.o_vbeg),
                   reinterpret_cast<const int64_t *>(dbase + s.o_tbeg),
                   reinterpret_cast<const int32_t *>(dbase + s.o_tcnt),
                   reinterpret_cast<const int64_t *>(dbase + s.o_hpbeg),
                   reinterpret_cast<const float2 *>(dbase + s.o_hdph),
                   reinterpret_cast<const int64_t *>(dbase + s.o_bkbeg),
                   reinterpret_cast<const float4 *>(dbase + s.o_blk),
                   (int32_t)s.objs.size(),
                   m->L,
                   m->has_vox ? reinterpret_cast<const uint8_t *>(dbase + s.o_vlab) : nullptr,
                   m->has_vox ? reinterpret_cast<const int64_t *>(dbase + s.o_lbeg) : nullptr,
                   m->has_vox ? reinterpret_cast<const unsigned long long *>(dbase + s.o_bmask) : nullptr};
}

int prep_threads(pj_context *ctx)
{
    int t = ctx->cfg.host_threads > 0 ? ctx->cfg.host_threads : (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(t, 16));
}

// A per-candidate host loop of a join: serial when short, else on the
// context's persistent workers (at most 7 besides the caller; created on the
// first long loop).
void host_for(pj_context *ctx, int64_t n, const std::function<void(int64_t)> &f)
{
    if (n < 2048 || prep_threads(ctx) <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    if (!ctx->pool) ctx->pool.reset(new HostPool(std::min(7, prep_threads(ctx) - 1)));
    ctx->pool->run(n, f);
}

// Items of a plan split into groups whose staged objects fit `budget`; each
// group is staged (synchronously, buffer set 0) and handed to fn with a
// sub-plan whose object ids are local to the staged views, and the plan
// index of each of its items.  Resident sets: one call with the full plan.
template <class F>
pj_status for_staged(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, TilePlan &pl, F fn)
{
    const int ni = (int)pl.items.size();
    if (!R->host && !S->host) {
        std::vector<int> orig(ni);
        std::iota(orig.begin(), orig.end(), 0);
        return fn(pl, R->dev(), S->dev(), orig);
    }
    if (ni == 0) return PJ_OK;
    hipStream_t st = ctx->stream;
    HIPTRY(ctx, hipStreamSynchronize(st));
    int64_t budget = int64_t(1) << 30;
    if (ctx->cfg.mem_cap_bytes > 0) {
        ctx->sb_stage[0].release();
        budget = (ctx->cfg.mem_cap_bytes - ctx->dev_bytes) / 2;
    }
    const int lod = pl.items[0].lod;
    const bool finest = pl.items[0].flags & IT_FINEST;
    // tiles of each item (an item's tiles are contiguous in a plan)
    std::vector<int64_t> tfirst(ni + 1, 0);
    for (const Tile &t : pl.tiles) tfirst[t.item + 1]++;
    for (int i = 0; i < ni; ++i) tfirst[i + 1] += tfirst[i];
    std::vector<int32_t> stampR(R->host ? R->n : 0, -1), stampS(S->host ? S->n : 0, -1);
    std::vector<int32_t> locR(stampR.size()), locS(stampS.size());
    int group = 0;
    for (int i0 = 0; i0 < ni; ++group) {
        SideStage sR, sS;
        sR.lod = sS.lod = lod;
        sR.finest = sS.finest = finest;
        int64_t bytes = 2 * kStageFixed;
        TilePlan sp;
        sp.tile_s = pl.tile_s;
        std::vector<int> orig;
        int i = i0;
        for (; i < ni; ++i) {
            Item it = pl.items[i];
            const bool sw = it.flags & IT_SWAP;
            const int ro = sw ? it.b_obj : it.a_obj, so = sw ? it.a_obj : it.b_obj;
            int64_t need = 0;
            if (R->host && stampR[ro] != group) need += stage_obj_bytes(R, ro, lod, finest);
            if (S->host && stampS[so] != group) need += stage_obj_bytes(S, so, lod, finest);
            if (i > i0 && bytes + need > budget) break;
            if (bytes + need > budget)
                return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "an object pair does not fit the staging budget of the cap");
            bytes += need;
            int lr = ro, ls = so;
            if (R->host) {
                if (stampR[ro] != group) {
                    stampR[ro] = group;
                    locR[ro] = (int32_t)sR.objs.size();
                    sR.objs.push_back(ro);
                }
                lr = locR[ro];
            }
            if (S->host) {
                if (stampS[so] != group) {
                    stampS[so] = group;
                    locS[so] = (int32_t)sS.objs.size();
                    sS.objs.push_back(so);
                }
                ls = locS[so];
            }
            it.a_obj = sw ? ls : lr;
            it.b_obj = sw ? lr : ls;
            const int local = (int)sp.items.size();
            sp.items.push_back(it);
            orig.push_back(i);
            for (int64_t t = tfirst[i]; t < tfirst[i + 1]; ++t) {
                Tile x = pl.tiles[t];
                x.item = local;
                sp.tiles.push_back(x);
            }
            sp.pairs += (int64_t)R->count(ro, lod) * S->count(so, lod);
        }
        stage_plan(R, sR, 0);
        stage_plan(S, sS, R->host ? sR.end : 0);
        const size_t total = std::max(R->host ? sR.end : 0, S->host ? sS.end : 0);
        PJTRY(ensure(ctx, ctx->sb_stage[0], total));
        PJTRY(ensure_pinned(ctx, ctx->pin_stage[0], total));
        char *hb = (char *)ctx->pin_stage[0].p;
        if (R->host) stage_fill(R, sR, hb, prep_threads(ctx));
        if (S->host) stage_fill(S, sS, hb, prep_threads(ctx));
        HIPTRY(ctx, hipMemcpyAsync(ctx->sb_stage[0].p, hb, total, hipMemcpyHostToDevice, st));
        ctx->stats.staged_bytes += (int64_t)total;
        char *db = (char *)ctx->sb_stage[0].p;
        const MeshDev Rv = R->host ? stage_view(R, sR, db) : R->dev();
        const MeshDev Sv = S->host ? stage_view(S, sS, db) : S->dev();
        PJTRY(fn(sp, Rv, Sv, orig));
        HIPTRY(ctx, hipStreamSynchronize(st));
        i0 = i;
    }
    return PJ_OK;
}

// Launch one chunk's refinement on `st`: the round's init kernel, then the
// refinement kernel (from a cached hipGraph of that one launch, or directly),
// with the events `e0`, `e1` (if given) around the latter only, so that they
// time the refinement kernel.
// Waves of a round's persistent launch: wpc per CU, or, for a round of fewer
// claimable units (A blocks x B ranges), the next power of two (at least 64)
// above their count.  More waves than units would only contend for the
// tile counters; the power-of-two steps keep few graph variants.
int round_grid(const pj_context *ctx, int wpc, int64_t units)
{
    const int full = ctx->num_cu * wpc;
    if (units <= 0 || units >= full) return full;
    int g = 64;
    while (g < units) g *= 2;
    return std::min(g, full);
}

pj_status launch_round(pj_context *ctx, const RefineArgs &a, int32_t *ctr, int ni, int nt, int wpc, bool graph,
                       hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, int64_t units = 0)
{
    // persistent grid of a fixed size per shape: the kernel reads the tile
    // count from memory; the slots of the full grid are reset
    const int full = ctx->num_cu * wpc;
    const int grid = round_grid(ctx, wpc, units);
    HIPTRY(ctx, launch_init_round(a.out, ctr, a.wave_slot, full, a.tile_cur, st));
    if (e0) HIPTRY(ctx, hipEventRecord(e0, st));
    if (!graph) {
        HIPTRY(ctx, launch_refine_f32(a, units > 0 ? grid : std::min<int64_t>(nt, grid), kP, st));
        if (e1) HIPTRY(ctx, hipEventRecord(e1, st));
        return PJ_OK;
    }
    std::vector<char> key(sizeof(a) + sizeof(int));
    std::memcpy(key.data(), &a, sizeof(a));
    std::memcpy(key.data() + sizeof(a), &grid, sizeof(int));
    hipGraphExec_t exec = nullptr;
    for (auto &g : ctx->graphs)
        if (g.key == key) exec = g.exec;
    if (!exec) {
        if (!ctx->cap_stream) HIPTRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIPTRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e2 = launch_refine_f32(a, grid, kP, ctx->cap_stream);
        hipError_t e3 = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (e2 != hipSuccess) return hipfail(ctx, e2, "capture of the refinement round");
        if (e3 != hipSuccess) return hipfail(ctx, e3, "hipStreamEndCapture");
        hipError_t e4 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e4 != hipSuccess) return hipfail(ctx, e4, "hipGraphInstantiate");
        if (ctx->graphs.size() >= 32) {
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back(pj_context::GraphEntry{key, exec});
    }
    HIPTRY(ctx, hipGraphLaunch(exec, st));
    if (e1) HIPTRY(ctx, hipEventRecord(e1, st));
    ctx->stats.graph_replays++;
    return PJ_OK;
}

// Offsets in a set's round buffer for an item capacity ci (see pj_context).
size_t rnd_ctr_off(int64_t ci) { return (size_t)ci * sizeof(ItemOut); }
size_t rnd_items_off(int64_t ci) { return rnd_ctr_off(ci) + 256; }
size_t rnd_tiles_off(int64_t ci) { return rnd_items_off(ci) + (size_t)ci * sizeof(Item); }

// FP32 bulk pass over a plan, streamed in chunks (the refinement pipeline of
// Section 3.3, Algorithm 5, on HIP streams).  A prep thread gathers chunk
// c+1 (items, tiles and, for host-resident sets, the chunk's facet data)
// into pinned staging while chunk c uploads on a copy stream, computes on the
// join stream and returns its per-item results on a third stream; two or
// three buffer sets rotate, and a set is refilled only after its previous
// chunk's results were merged.  A chunk ends at `max_tiles` tiles or when its
// staged objects fill the staging budget; an item whose tiles span chunks
// appears in each and its minima are merged on the host.
pj_status run_f32(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, TilePlan &pl, float tau, bool early,
                  std::vector<ItemOut> &out, int wpc_override)
{
    const int wpc = wpc_override > 0 ? wpc_override : ctx->cur.wpc;
    const bool graph = ctx->cfg.use_graph && wpc_override == 0;
    hipStream_t st = ctx->stream;
    const int ni = (int)pl.items.size(), nt = (int)pl.tiles.size();
    out.assign(ni, ItemOut{0x7f800000u, 0x7f800000u, 0, 0});
    if (ni == 0 || nt == 0) return PJ_OK;
    PJTRY(ensure_streams(ctx));
    // one set: every chunk is gathered, uploaded, computed and downloaded
    // before the next is gathered (no overlap; the comparison for the
    // pipelined two and three sets)
    const int nsets = ctx->cfg.stage_sets == 3 ? 3 : (ctx->cfg.stage_sets == 1 ? 1 : 2);
    const bool hostR = R->host, hostS = S->host, staged = hostR || hostS;
    const int lod = pl.items[0].lod;
    const bool finest = pl.items[0].flags & IT_FINEST;
    const int grid = ctx->num_cu * wpc;  // persistent grid of the rounds
    // worst case one item per tile; each tile also has an A-block cursor
    const int64_t per_tile = sizeof(Tile) + sizeof(Item) + sizeof(ItemOut);
    int64_t max_tiles = ctx->cfg.chunk_tiles > 0 ? ctx->cfg.chunk_tiles : int64_t(1) << 22;
    int64_t stage_budget = int64_t(1) << 30;
    if (ctx->cfg.mem_cap_bytes > 0) {
        // size the chunks for what the cap leaves once the chunk buffers are
        // given back (the join stream is idle between rounds)
        HIPTRY(ctx, hipStreamSynchronize(st));
        for (int b = 0; b < kMaxSets; ++b)
            for (DevBuf *x : {&ctx->sb_rnd[b], &ctx->sb_stage[b]})
                x->release();
        for (int b = 0; b < kMaxSets; ++b) ctx->rcap_i[b] = ctx->rcap_t[b] = 0;
        ctx->b_sched.release();
        // the shared scheduling buffer: a slot per workgroup (reserved here)
        // and a cursor per tile of a chunk (charged with each tile below)
        const int64_t room = ctx->cfg.mem_cap_bytes - ctx->dev_bytes - 4 * grid - 256;
        const int64_t per_set = room / nsets - (5 * 256 + 64);
        int64_t tile_part = per_set;
        if (staged) {
            stage_budget = per_set * 3 / 4;
            tile_part = per_set - stage_budget;
        }
        max_tiles = std::min<int64_t>(max_tiles, tile_part / (per_tile + 4) - 1);
        if (max_tiles < 1 || (staged && stage_budget < 4 * kStageFixed))
            return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "the memory cap cannot hold one refinement chunk");
    }
    struct Chunk {
        int64_t t0 = 0, t1 = 0;
        std::vector<int> items;           // plan item indices, in chunk-local order
        std::vector<int32_t> locR, locS;  // per chunk item: object ids in the chunk's views
        SideStage sR, sS;
        size_t stage_bytes = 0;
    };
    std::vector<Chunk> chunks;
    std::vector<int32_t> tile_local(nt);  // chunk-local item index of each tile
    {
        std::vector<int> local(ni, -1);
        std::vector<int32_t> stampR(hostR ? R->n : 0, -1), stampS(hostS ? S->n : 0, -1);
        std::vector<int32_t> locR_of(stampR.size()), locS_of(stampS.size());
        Chunk c;
        int cid = 0;
        int64_t sbytes = 2 * kStageFixed;
        auto close = [&](int64_t t) {
            c.t1 = t;
            for (int it : c.items) local[it] = -1;
            chunks.push_back(std::move(c));
            c = Chunk();
            c.t0 = t;
            ++cid;
            sbytes = 2 * kStageFixed;
        };
        for (int64_t t = 0; t < nt; ++t) {
            if (t - c.t0 >= max_tiles) close(t);
            const int it = pl.tiles[t].item;
            if (local[it] < 0) {
                const Item &I = pl.items[it];
                const bool sw = I.flags & IT_SWAP;
                const int ro = sw ? I.b_obj : I.a_obj, so = sw ? I.a_obj : I.b_obj;
                auto need_of = [&]() {
                    int64_t need = 0;
                    if (hostR && stampR[ro] != cid) need += stage_obj_bytes(R, ro, lod, finest);
                    if (hostS && stampS[so] != cid) need += stage_obj_bytes(S, so, lod, finest);
                    return need;
                };
                int64_t need = need_of();
                if (need && sbytes + need > stage_budget && t > c.t0) {
                    close(t);
                    need = need_of();
                }
                if (sbytes + need > stage_budget)
                    return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "an object pair does not fit the staging budget of the cap");
                sbytes += need;
                int lr = ro, ls = so;
                if (hostR) {
                    if (stampR[ro] != cid) {
                        stampR[ro] = cid;
                        locR_of[ro] = (int32_t)c.sR.objs.size();
                        c.sR.objs.push_back(ro);
                    }
                    lr = locR_of[ro];
                }
                if (hostS) {
                    if (stampS[so] != cid) {
                        stampS[so] = cid;
                        locS_of[so] = (int32_t)c.sS.objs.size();
                        c.sS.objs.push_back(so);
                    }
                    ls = locS_of[so];
                }
                local[it] = (int)c.items.size();
                c.items.push_back(it);
                c.locR.push_back(lr);
                c.locS.push_back(ls);
            }
            tile_local[t] = local[it];
        }
        close(nt);
    }
    const int nch = (int)chunks.size();
    for (Chunk &c : chunks) {
        c.sR.lod = c.sS.lod = lod;
        c.sR.finest = c.sS.finest = finest;
        if (hostR) stage_plan(R, c.sR, 0);
        if (hostS) stage_plan(S, c.sS, hostR ? c.sR.end : 0);
        c.stage_bytes = std::max(hostR ? c.sR.end : 0, hostS ? c.sS.end : 0);
    }
    const int nthreads = prep_threads(ctx);
    // the largest chunk of the round sizes every set's buffers once
    int64_t rnd_ni = 0, rnd_nt = 0, rnd_stage = 0;
    for (const Chunk &c : chunks) {
        rnd_ni = std::max<int64_t>(rnd_ni, (int64_t)c.items.size());
        rnd_nt = std::max<int64_t>(rnd_nt, c.t1 - c.t0);
        rnd_stage = std::max<int64_t>(rnd_stage, (int64_t)c.stage_bytes);
    }
    // buffers of chunk j's set (main thread: HIP allocation calls stay here)
    auto alloc = [&](int j) -> pj_status {
        const int b = j % nsets;
        const int64_t cni = rnd_ni, cnt = rnd_nt;
        if (cni > ctx->rcap_i[b] || cnt > ctx->rcap_t[b]) {
            // grow by half at least (new addresses mean a new graph); under a
            // memory cap exactly (the chunks were sized to what it leaves)
            const bool exact = ctx->cfg.mem_cap_bytes > 0;
            auto grow = [exact](int64_t need, int64_t have) {
                return exact ? need : std::max(need, have + have / 2 + 64) / 64 * 64 + 64;
            };
            if (cni > ctx->rcap_i[b]) ctx->rcap_i[b] = grow(cni, ctx->rcap_i[b]);
            if (cnt > ctx->rcap_t[b]) ctx->rcap_t[b] = grow(cnt, ctx->rcap_t[b]);
        }
        const size_t bytes = rnd_tiles_off(ctx->rcap_i[b]) + (size_t)ctx->rcap_t[b] * sizeof(Tile);
        PJTRY(ensure(ctx, ctx->sb_rnd[b], bytes));
        PJTRY(ensure_pinned(ctx, ctx->pin_rnd[b], bytes));
        if (staged) {
            PJTRY(ensure(ctx, ctx->sb_stage[b], (size_t)rnd_stage));
            PJTRY(ensure_pinned(ctx, ctx->pin_stage[b], (size_t)rnd_stage));
        }
        return PJ_OK;
    };
    std::vector<double> prep_ms(nch, 0.0);  // host gather time per chunk (written by its prep)
    // host preparation of chunk j into the pinned buffers of its set (no HIP calls)
    auto prep = [&, nthreads](int j) {
        const int b = j % nsets;
        const Chunk &c = chunks[j];
        const int cni = (int)c.items.size();
        char *hb = (char *)ctx->pin_rnd[b].p;
        Item *hi = (Item *)(hb + rnd_items_off(ctx->rcap_i[b]));
        Tile *ht = (Tile *)(hb + rnd_tiles_off(ctx->rcap_i[b]));
        for (int q = 0; q < cni; ++q) {
            Item x = pl.items[c.items[q]];
            const bool sw = x.flags & IT_SWAP;
            x.a_obj = sw ? c.locS[q] : c.locR[q];
            x.b_obj = sw ? c.locR[q] : c.locS[q];
            hi[q] = x;
        }
        for (int64_t t = c.t0; t < c.t1; ++t) {
            Tile x = pl.tiles[t];
            x.item = tile_local[t];
            ht[t - c.t0] = x;
        }
        int32_t *hc = (int32_t *)(hb + rnd_ctr_off(ctx->rcap_i[b]));
        // counter block: [1] tiles, [2..3] pairs evaluated, [4..5] chunks
        // culled, [6] items, [10] next tile to take (all others 0)
        std::memset(hc, 0, 64);
        hc[1] = (int32_t)(c.t1 - c.t0);
        hc[6] = cni;
        char *hs = (char *)ctx->pin_stage[b].p;
        const double tp = now_ms();
        if (j + 1 < (int)chunks.size()) {
            // file residency: start reading the next chunk's pages now
            if (hostR) advise_objects(R, chunks[j + 1].sR.objs, lod, finest);
            if (hostS) advise_objects(S, chunks[j + 1].sS.objs, lod, finest);
        }
        if (hostR) stage_fill(R, c.sR, hs, nthreads);
        if (hostS) stage_fill(S, c.sS, hs, nthreads);
        prep_ms[j] = now_ms() - tp;
    };
    // A round of one chunk on device-resident sets has nothing to overlap:
    // its copies go on the join stream, which saves two hand-offs between
    // hardware queues per round.
    const bool one = nch == 1 && !staged;
    hipStream_t ups = one ? st : ctx->up_stream, downs = one ? st : ctx->down_stream;
    auto enqueue = [&](int j) -> pj_status {
        const int b = j % nsets;
        const Chunk &c = chunks[j];
        const int cni = (int)c.items.size(), cnt = (int)(c.t1 - c.t0);
        const int64_t ci = ctx->rcap_i[b];
        char *db = (char *)ctx->sb_rnd[b].p, *hb = (char *)ctx->pin_rnd[b].p;
        int32_t *dctr = (int32_t *)(db + rnd_ctr_off(ci));
        if (staged) {
            HIPTRY(ctx, hipMemcpyAsync(ctx->sb_stage[b].p, ctx->pin_stage[b].p, c.stage_bytes, hipMemcpyHostToDevice,
                                       ctx->up_stream));
            ctx->stats.staged_bytes += (int64_t)c.stage_bytes;
        }
        // counters, items and tiles in one copy
        HIPTRY(ctx, hipMemcpyAsync(db + rnd_ctr_off(ci), hb + rnd_ctr_off(ci),
                                   rnd_tiles_off(ci) - rnd_ctr_off(ci) + (size_t)cnt * sizeof(Tile),
                                   hipMemcpyHostToDevice, ups));
        if (!one) HIPTRY(ctx, hipEventRecord(ctx->ev_h2d[b], ups));
        RefineArgs a;
        std::memset(&a, 0, sizeof(a));
        char *ds = (char *)ctx->sb_stage[b].p;
        a.R = hostR ? stage_view(R, c.sR, ds) : R->dev();
        a.S = hostS ? stage_view(S, c.sS, ds) : S->dev();
        a.items = (Item *)(db + rnd_items_off(ci));
        a.tiles = (Tile *)(db + rnd_tiles_off(ci));
        a.ntiles = dctr + 1;
        a.tile_next = dctr + 10;
        // rounds run one after another on the join stream, so all chunks
        // share one set of slots and cursors (reset by the round's init kernel)
        a.wave_slot = ptr<int32_t>(ctx->b_sched);
        a.tile_cur = ptr<int32_t>(ctx->b_sched) + grid;
        a.out = (ItemOut *)db;
        a.pairs_done = reinterpret_cast<unsigned long long *>(dctr + 2);
        a.chunks_culled = reinterpret_cast<unsigned long long *>(dctr + 4);
        a.tau = tau;
        a.early = early ? 1 : 0;
        a.cull = ctx->cfg.tile_cull ? 1 : 0;
        a.vmask = ctx->vmask;
        a.vrow = ctx->vrow;
        if (!one) HIPTRY(ctx, hipStreamWaitEvent(st, ctx->ev_h2d[b], 0));
        int64_t units = 0;  // claimable (A block, B range) units of the chunk
        for (int64_t t = c.t0; t < c.t1; ++t)
            units += (pl.tiles[t].a1 - pl.tiles[t].a0 + 64 * kP - 1) / (64 * kP);
        PJTRY(launch_round(ctx, a, dctr, cni, cnt, wpc, graph, st, ctx->ev_k0[b], ctx->ev_k1[b], units));
        if (!one) {
            HIPTRY(ctx, hipEventRecord(ctx->ev_comp[b], st));
            HIPTRY(ctx, hipStreamWaitEvent(downs, ctx->ev_comp[b], 0));
        }
        // results and counters in one copy
        HIPTRY(ctx, hipMemcpyAsync(hb, db, rnd_ctr_off(ci) + 64, hipMemcpyDeviceToHost, downs));
        HIPTRY(ctx, hipEventRecord(ctx->ev_d2h[b], downs));
        ctx->stats.chunks++;
        return PJ_OK;
    };
    std::vector<char> merged(nch, 0);
    auto merge = [&](int j) -> pj_status {
        if (merged[j]) return PJ_OK;
        const int b = j % nsets;
        HIPTRY(ctx, hipEventSynchronize(ctx->ev_d2h[b]));
        const Chunk &c = chunks[j];
        const ItemOut *o = (const ItemOut *)ctx->pin_rnd[b].p;
        for (size_t q = 0; q < c.items.size(); ++q) {
            ItemOut &d = out[c.items[q]];
            d.lb = std::min(d.lb, o[q].lb);
            d.ub = std::min(d.ub, o[q].ub);
            d.hit |= o[q].hit;
        }
        const int32_t *hc = (const int32_t *)((const char *)ctx->pin_rnd[b].p + rnd_ctr_off(ctx->rcap_i[b]));
        unsigned long long pairs, culled;
        std::memcpy(&pairs, hc + 2, 8);
        std::memcpy(&culled, hc + 4, 8);
        ctx->stats.facet_pairs += (int64_t)pairs;
        ctx->stats.tiles_culled += (int64_t)culled;
        float ms = 0;
        HIPTRY(ctx, hipEventElapsedTime(&ms, ctx->ev_k0[b], ctx->ev_k1[b]));
        ctx->stats.refine_kernel_ms += ms;
        ctx->stats.refine_launches += 1;
        if (lod < 8) {
            ctx->stats.lod_pairs[lod] += (int64_t)pairs;
            ctx->stats.lod_kernel_ms[lod] += ms;
        }
        merged[j] = 1;
        return PJ_OK;
    };
    int64_t max_cnt = 0;
    for (const Chunk &c : chunks) max_cnt = std::max<int64_t>(max_cnt, c.t1 - c.t0);
    PJTRY(ensure(ctx, ctx->b_sched, 4 * (grid + max_cnt)));
    PJTRY(alloc(0));
    prep(0);
    std::thread worker;
    pj_status st_all = PJ_OK;
    for (int ci = 0; ci < nch && st_all == PJ_OK; ++ci) {
        if (worker.joinable()) worker.join();  // chunk ci is prepared
        st_all = enqueue(ci);
        if (st_all != PJ_OK) break;
        const int j = ci + 1;
        if (j < nch) {
            // the set of chunk j is free once chunk j - nsets is merged
            if (j - nsets >= 0) st_all = merge(j - nsets);
            if (st_all == PJ_OK) st_all = alloc(j);
            if (st_all != PJ_OK) break;
            worker = std::thread(prep, j);
        }
        if (ci >= 1) st_all = merge(ci - 1);
    }
    if (worker.joinable()) worker.join();
    if (st_all != PJ_OK) {
        (void)hipStreamSynchronize(ctx->down_stream);
        return st_all;
    }
    for (int j = 0; j < nch; ++j) PJTRY(merge(j));
    for (double x : prep_ms) ctx->stats.t_prep_ms += x;
    // the join stream must not run ahead of the downloads
    if (!one) HIPTRY(ctx, hipStreamWaitEvent(st, ctx->ev_d2h[(nch - 1) % nsets], 0));
    ctx->stats.tiles += nt;
    if (lod < 8) {
        ctx->stats.lod_items[lod] += ni;
        ctx->stats.lod_tiles[lod] += nt;
    }
    ctx->stats.tile_s_used = wpc_override > 0 ? pl.tile_s : ctx->cur.tile_s;
    ctx->stats.waves_per_cu_used = wpc;
    if (ctx->cfg.mem_cap_bytes > 0) {
        // under a cap the chunk buffers were sized to what the cap left:
        // give them back so that the next phase has the same room
        HIPTRY(ctx, hipStreamSynchronize(st));
        for (int b = 0; b < kMaxSets; ++b)
            for (DevBuf *x : {&ctx->sb_rnd[b], &ctx->sb_stage[b]})
                x->release();
        for (int b = 0; b < kMaxSets; ++b) ctx->rcap_i[b] = ctx->rcap_t[b] = 0;
        ctx->b_sched.release();
    }
    return PJ_OK;
}

pj_status run_f64_view(pj_context *ctx, const MeshDev &Rv, const MeshDev &Sv, TilePlan &pl, bool plain,
                       std::vector<ItemOut64> &out)
{
    hipStream_t st = ctx->stream;
    const int ni = (int)pl.items.size(), nt = (int)pl.tiles.size();
    out.assign(ni, ItemOut64{0x7ff0000000000000ull, 0x7ff0000000000000ull, 0, 0});
    if (ni == 0) return PJ_OK;
    PJTRY(ensure(ctx, ctx->b_items, ni * sizeof(Item)));
    PJTRY(ensure(ctx, ctx->b_out64, ni * sizeof(ItemOut64)));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_items.p, pl.items.data(), ni * sizeof(Item), hipMemcpyHostToDevice, st));
    Refine64Args a;
    a.R = Rv;
    a.S = Sv;
    a.items = ptr<Item>(ctx->b_items);
    a.out = ptr<ItemOut64>(ctx->b_out64);
    a.tiles = nullptr;
    HIPTRY(ctx, launch_init_out64(a.out, ni, st));
    HIPTRY(ctx, hipEventRecord(ctx->ev0, st));
    if (plain) {
        HIPTRY(ctx, launch_refine_f64_plain(a, ni, st));
    } else {
        // tiles in chunks that fit what a cap leaves (the item results are
        // minima, so the chunks simply run one after another)
        int64_t per = nt;
        if (ctx->cfg.mem_cap_bytes > 0) {
            HIPTRY(ctx, hipStreamSynchronize(st));
            ctx->b_tiles.release();
            per = std::max<int64_t>(1, std::min<int64_t>(nt, (ctx->cfg.mem_cap_bytes - ctx->dev_bytes - 512) /
                                                                  (int64_t)sizeof(Tile)));
        }
        PJTRY(ensure(ctx, ctx->b_tiles, per * sizeof(Tile)));
        a.tiles = ptr<Tile>(ctx->b_tiles);
        for (int64_t t0 = 0; t0 < nt; t0 += per) {
            const int64_t n = std::min<int64_t>(per, nt - t0);
            HIPTRY(ctx, hipMemcpyAsync(ctx->b_tiles.p, pl.tiles.data() + t0, n * sizeof(Tile), hipMemcpyHostToDevice,
                                       st));
            HIPTRY(ctx, launch_refine_f64_tiles(a, n, st));
        }
    }
    HIPTRY(ctx, hipEventRecord(ctx->ev1, st));
    HIPTRY(ctx, hipMemcpyAsync(out.data(), a.out, ni * sizeof(ItemOut64), hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    float ms = 0;
    HIPTRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->stats.band_kernel_ms += ms;
    ctx->stats.facet_pairs_fp64 += pl.pairs;
    return PJ_OK;
}

// FP64 pass over a plan (plain schedule, FP64 precision and the overflow
// path of the band recheck); host-resident sets are staged in item groups.
pj_status run_f64(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, TilePlan &pl, bool plain,
                  std::vector<ItemOut64> &out)
{
    out.assign(pl.items.size(), ItemOut64{0x7ff0000000000000ull, 0x7ff0000000000000ull, 0, 0});
    return for_staged(ctx, R, S, pl,
                      [&](TilePlan &sp, const MeshDev &Rv, const MeshDev &Sv, const std::vector<int> &orig) {
                          std::vector<ItemOut64> o;
                          PJTRY(run_f64_view(ctx, Rv, Sv, sp, plain, o));
                          for (size_t k = 0; k < o.size(); ++k) out[orig[k]] = o[k];
                          return PJ_OK;
                      });
}

// Exact FP64 finest-LoD distance of the candidates `which`: one FP32 pass
// keeps the facet pairs whose lower distance is within the item's threshold
// and within 2 eps of the running minimum (this always includes the pair that
// realises the minimum), then FP64 with the exact meet test recomputes only
// those.  Items whose pairs overflow the buffer are recomputed in full FP64.
pj_status exact_finest(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, std::vector<Cand> &cand,
                       std::vector<PairState> &ps, const std::vector<int> &which);

double bits_to_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, 8);
    return d;
}
float bits_to_float(uint32_t b)
{
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

int pick_tile_s(pj_context *ctx);

// collect + FP64 pass of one (staged) plan; overflowed candidates go to redo
pj_status exact_finest_view(pj_context *ctx, const MeshDev &Rv, const MeshDev &Sv, TilePlan &pl,
                            std::vector<PairState> &ps, std::vector<int> &redo)
{
    hipStream_t st = ctx->stream;
    const int ni = (int)pl.items.size(), nt = (int)pl.tiles.size();
    if (ni == 0) return PJ_OK;
    const int cgrid = (int)std::min<int64_t>(nt, (int64_t)ctx->num_cu * ctx->cur.wpc);
    // The list is sized from what the last collect pass offered per item
    // (256 before the first), with a quarter more, at least 2^20 pairs and at
    // most 2^28.  A pass that offers more than the list holds is run once
    // more with room for what it offered (the thresholds tighten as minima
    // are published, so the count can differ a little between runs); items
    // that overflow again are recomputed in full FP64 by the caller.
    const int64_t kMaxColl = int64_t(1) << 28;
    auto want = [&](double n) {
        return std::min<int64_t>(std::max<int64_t>(int64_t(1) << 20, (int64_t)(1.25 * n) + 65536), kMaxColl);
    };
    int64_t cap = want((ctx->coll_per_item > 0.0 ? ctx->coll_per_item : 256.0) * ni);
    int64_t room = kMaxColl;
    if (ctx->cfg.mem_cap_bytes > 0) {
        // the collect list takes what the cap leaves
        HIPTRY(ctx, hipStreamSynchronize(st));
        for (DevBuf *x : {&ctx->b_items, &ctx->b_tiles, &ctx->b_out, &ctx->b_out64, &ctx->b_ovf, &ctx->b_coll,
                          &ctx->b_ctr})
            x->release();
        const int64_t fixed = (int64_t)(ni * (sizeof(Item) + sizeof(ItemOut) + sizeof(ItemOut64) + sizeof(int32_t)) +
                                        nt * (sizeof(Tile) + 4) + 64 + 4 * cgrid + 7 * 256);
        room = std::min<int64_t>(room, (ctx->cfg.mem_cap_bytes - ctx->dev_bytes - fixed) / (int64_t)sizeof(PairRef));
        cap = std::min<int64_t>(cap, room);
        if (cap < 256) return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "the memory cap leaves no room for the FP64 recheck");
    }
    PJTRY(ensure(ctx, ctx->b_items, ni * sizeof(Item)));
    PJTRY(ensure(ctx, ctx->b_tiles, nt * sizeof(Tile)));
    PJTRY(ensure(ctx, ctx->b_out, ni * sizeof(ItemOut)));
    PJTRY(ensure(ctx, ctx->b_out64, ni * sizeof(ItemOut64)));
    PJTRY(ensure(ctx, ctx->b_ovf, ni * sizeof(int32_t)));
    PJTRY(ensure(ctx, ctx->b_ctr, 64 + 4 * (cgrid + nt)));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_items.p, pl.items.data(), ni * sizeof(Item), hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_tiles.p, pl.tiles.data(), nt * sizeof(Tile), hipMemcpyHostToDevice, st));
    int32_t *ctr = ptr<int32_t>(ctx->b_ctr);
    int32_t host_ctr[16];
    RefineArgs a;
    unsigned long long offered = 0;
    for (int attempt = 0;; ++attempt) {
        PJTRY(ensure(ctx, ctx->b_coll, cap * sizeof(PairRef)));
        std::memset(host_ctr, 0, sizeof(host_ctr));
        host_ctr[1] = nt;
        host_ctr[6] = ni;
        HIPTRY(ctx, hipMemcpyAsync(ctr, host_ctr, sizeof(host_ctr), hipMemcpyHostToDevice, st));
        HIPTRY(ctx, hipMemsetAsync(ctx->b_ovf.p, 0, ni * sizeof(int32_t), st));
        HIPTRY(ctx, launch_init_round(ptr<ItemOut>(ctx->b_out), ctr, ctr + 16, cgrid, ctr + 16 + cgrid, st));
        HIPTRY(ctx, launch_init_out64(ptr<ItemOut64>(ctx->b_out64), ni, st));
        std::memset(&a, 0, sizeof(a));
        a.R = Rv;
        a.S = Sv;
        a.items = ptr<Item>(ctx->b_items);
        a.tiles = ptr<Tile>(ctx->b_tiles);
        a.ntiles = ctr + 1;
        a.tile_next = ctr + 10;
        a.wave_slot = ctr + 16;
        a.tile_cur = ctr + 16 + cgrid;
        a.collected_n = reinterpret_cast<unsigned long long *>(ctr + 8);
        a.out = ptr<ItemOut>(ctx->b_out);
        a.pairs_done = reinterpret_cast<unsigned long long *>(ctr + 2);
        a.chunks_culled = reinterpret_cast<unsigned long long *>(ctr + 4);
        a.tau = -1.0f;
        a.cull = ctx->cfg.tile_cull ? 1 : 0;
        a.collect_cap = cap;
        a.collected = ptr<PairRef>(ctx->b_coll);
        a.overflow = ptr<int32_t>(ctx->b_ovf);
        a.vmask = ctx->vmask;
        a.vrow = ctx->vrow;
        HIPTRY(ctx, hipEventRecord(ctx->ev0, st));
        HIPTRY(ctx, launch_collect_f32(a, cgrid, st));
        HIPTRY(ctx, hipEventRecord(ctx->ev1, st));
        HIPTRY(ctx, hipMemcpyAsync(host_ctr, ctr, sizeof(host_ctr), hipMemcpyDeviceToHost, st));
        HIPTRY(ctx, hipStreamSynchronize(st));
        float ms = 0;
        HIPTRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->stats.collect_kernel_ms += ms;
        ctx->stats.collect_launches += 1;
        unsigned long long pairs;
        std::memcpy(&pairs, host_ctr + 2, 8);
        std::memcpy(&offered, host_ctr + 8, 8);
        ctx->stats.collect_pairs += (int64_t)pairs;
        ctx->coll_per_item = (double)offered / ni;
        if (offered <= (unsigned long long)cap || attempt > 0) break;
        const int64_t grow = std::min<int64_t>(want((double)offered), room);
        if (grow <= cap) break;
        cap = grow;
        ctx->stats.collect_regrow++;
    }
    const int64_t ncoll = (int64_t)std::min<unsigned long long>(offered, (unsigned long long)cap);
    ctx->stats.collected_pairs += (int64_t)offered;
    float ms = 0;
    HIPTRY(ctx, hipEventRecord(ctx->ev0, st));
    HIPTRY(ctx, launch_pairs_f64(Rv, Sv, a.items, a.collected, ncoll, ptr<ItemOut64>(ctx->b_out64), st));
    HIPTRY(ctx, hipEventRecord(ctx->ev1, st));
    std::vector<ItemOut64> out(ni);
    std::vector<int32_t> ovf(ni);
    HIPTRY(ctx, hipMemcpyAsync(out.data(), ctx->b_out64.p, ni * sizeof(ItemOut64), hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipMemcpyAsync(ovf.data(), ctx->b_ovf.p, ni * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    HIPTRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->stats.band_kernel_ms += ms;
    ctx->stats.facet_pairs_fp64 += ncoll;
    for (int k = 0; k < ni; ++k) {
        PairState &p = ps[pl.items[k].cand];
        if (ovf[k]) {
            ctx->stats.collect_overflow++;
            redo.push_back(pl.items[k].cand);
            continue;
        }
        p.hit64 = out[k].hit;
        p.d64 = p.hit64 ? 0.0 : bits_to_double(out[k].lb);
    }
    return PJ_OK;
}

pj_status exact_finest(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, std::vector<Cand> &cand,
                       std::vector<PairState> &ps, const std::vector<int> &which)
{
    if (which.empty()) return PJ_OK;
    const int L = R->L;
    PJTRY(choose_shape(ctx, R, S, which, cand, ps, L - 1, 1, -1.0f, false));
    // An open threshold is closed from the pair's upper bound UB (filter
    // anchors or a coarser LoD): the facet pair that realises the exact
    // minimum d* <= UB has FP32 lower distance <= d* + eps <= UB + 2 eps (one
    // eps more covers the FP64 rounding of d*).  The collect pass tightens it
    // with the item's running FP32 minimum as it goes, which it shares across
    // lanes and tiles only with culling on.  A pair with no finite UB, or any
    // open pair with culling off, gets an FP32 minimum pass first: with u its
    // FP32 upper distance, the bound is u + 2 eps.
    std::vector<int> open;
    for (int i : which) {
        PairState &p = ps[i];
        if (std::isfinite(p.thr)) continue;
        if (std::isfinite(p.UB) && ctx->cfg.tile_cull) p.thr = up_float(p.UB + 2.0 * (double)p.eps);
        else open.push_back(i);
    }
    if (!open.empty()) {
        TilePlan po;
        plan_tiles(R, S, open, cand, ps, L - 1, 1, 64 * kP, ctx->cur.tile_s, true, po, tile_target(ctx, kPlanWPC));
        std::vector<ItemOut> o32;
        PJTRY(run_f32(ctx, R, S, po, -1.0f, false, o32, 0));
        for (size_t k = 0; k < po.items.size(); ++k) {
            PairState &p = ps[po.items[k].cand];
            const float u = bits_to_float(o32[k].ub);
            if (std::isfinite(u)) p.thr = std::min(p.thr, up_float((double)u + 2.0 * (double)p.eps));
        }
    }
    TilePlan pl;
    plan_tiles(R, S, which, cand, ps, L - 1, 1, 64, ctx->cur.tile_s, true, pl, tile_target(ctx, kPlanWPC));
    std::vector<int> redo;
    PJTRY(for_staged(ctx, R, S, pl,
                     [&](TilePlan &sp, const MeshDev &Rv, const MeshDev &Sv, const std::vector<int> &) {
                         return exact_finest_view(ctx, Rv, Sv, sp, ps, redo);
                     }));
    if (!redo.empty()) {
        if (ctx->cfg.mem_cap_bytes > 0) {
            // under a cap the collect list took all the room it could: give
            // the collect buffers back before the full FP64 pass
            HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
            for (DevBuf *x : {&ctx->b_items, &ctx->b_tiles, &ctx->b_out, &ctx->b_out64, &ctx->b_ovf, &ctx->b_coll,
                              &ctx->b_ctr})
                x->release();
        }
        TilePlan p2;
        plan_tiles(R, S, redo, cand, ps, R->L - 1, 1, 64, pick_tile_s(ctx), true, p2);
        std::vector<ItemOut64> o2;
        PJTRY(run_f64(ctx, R, S, p2, false, o2));
        for (size_t k = 0; k < p2.items.size(); ++k) {
            PairState &p = ps[p2.items[k].cand];
            p.hit64 = o2[k].hit;
            p.d64 = p.hit64 ? 0.0 : bits_to_double(o2[k].lb);
        }
    }
    if (ctx->cfg.mem_cap_bytes > 0) {
        HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
        for (DevBuf *x : {&ctx->b_items, &ctx->b_tiles, &ctx->b_out, &ctx->b_out64, &ctx->b_ovf, &ctx->b_coll,
                          &ctx->b_ctr, &ctx->sb_stage[0]})
            x->release();
    }
    return PJ_OK;
}

pj_status check_pair_args(pj_context *ctx, const pj_meshes *R, const pj_meshes *S)
{
    if (!R || !S) return fail(ctx, PJ_ERR_INVALID_ARG, "NULL mesh set");
    if (R->device != ctx->cfg.device || S->device != ctx->cfg.device)
        return fail(ctx, PJ_ERR_INVALID_ARG, "mesh set lives on another device");
    if (R->n > 0 && S->n > 0 && R->L != S->L) return fail(ctx, PJ_ERR_INVALID_ARG, "n_lods differ between R and S");
    return PJ_OK;
}

// The filter's count pass leaves the candidate total on the device; it comes
// back through pinned memory.
pj_status read_cand_total(pj_context *ctx, int64_t &total)
{
    PJTRY(ensure_pinned(ctx, ctx->pin_cand, 4096));
    HIPTRY(ctx, hipMemcpyAsync(ctx->pin_cand.p, ctx->b_total.p, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(&total, ctx->pin_cand.p, 8);
    return PJ_OK;
}

// The write pass stores the candidates as four arrays of `total` (r, s, lb,
// ub) in one device buffer, which comes back in one copy through pinned memory.
pj_status download_cands(pj_context *ctx, int64_t total, std::vector<Cand> &cand)
{
    PJTRY(ensure_pinned(ctx, ctx->pin_cand, (size_t)total * 16));
    HIPTRY(ctx, hipMemcpyAsync(ctx->pin_cand.p, ctx->b_cand_r.p, (size_t)total * 16, hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(ctx, hipStreamSynchronize(ctx->stream));
    const int32_t *cr = static_cast<const int32_t *>(ctx->pin_cand.p), *cs = cr + total;
    const float *lb = reinterpret_cast<const float *>(cs + total), *ub = lb + total;
    cand.resize(total);
    for (int64_t i = 0; i < total; ++i) cand[i] = Cand{cr[i], cs[i], lb[i], ub[i]};
    return PJ_OK;
}

// Sweep filter: same candidates and bounds as the all-pairs test (order:
// R by xmin, then S by xmin).  The window around each r is widened by the
// widest S box and by relative margins that cover every rounding in the
// FP32 gap test, so each s the all-pairs test keeps lies inside it.
pj_status mbb_filter_sweep(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, float tau2,
                           std::vector<Cand> &cand)
{
    hipStream_t st = ctx->stream;
    const int nR = R->n, nS = S->n;
    const double T = std::sqrt((double)tau2) * (1.0 + std::ldexp(1.0, -20));
    const double cmax = std::max(R->max_abs, S->max_abs) + T;
    const float w_hi = up_float(T * (1.0 + std::ldexp(1.0, -20)) + std::ldexp(cmax, -20));
    const float w_lo = up_float((double)w_hi + S->max_w * (1.0 + std::ldexp(1.0, -20)) + std::ldexp(cmax, -20));
    const int nb = (nR + 255) / 256;
    PJTRY(ensure(ctx, ctx->b_blk, nb * sizeof(int32_t)));
    PJTRY(ensure(ctx, ctx->b_blkoff, (nb + 1) * sizeof(int64_t)));
    PJTRY(ensure(ctx, ctx->b_total, 16));
    HIPTRY(ctx, launch_filter_sweep(R->d_box, R->d_anchor, R->d_xord, nR, S->d_xbox, S->d_xanc, S->d_xord, S->d_xmin,
                                    nS, tau2, w_lo, w_hi, ptr<int32_t>(ctx->b_blk), nullptr, nullptr, nullptr,
                                    nullptr, nullptr, 0, st));
    HIPTRY(ctx, launch_scan_i32_to_i64(ptr<int32_t>(ctx->b_blk), ptr<int64_t>(ctx->b_blkoff), ptr<int64_t>(ctx->b_total),
                                       nb, st));
    int64_t total = 0;
    PJTRY(read_cand_total(ctx, total));
    if (total == 0) return PJ_OK;
    if (total > INT32_MAX) return fail(ctx, PJ_ERR_UNSUPPORTED, "more than 2^31 candidate pairs");
    PJTRY(ensure(ctx, ctx->b_cand_r, total * 16));
    int32_t *d_cr = ptr<int32_t>(ctx->b_cand_r), *d_cs = d_cr + total;
    float *d_lb = reinterpret_cast<float *>(d_cs + total), *d_ub = d_lb + total;
    HIPTRY(ctx, launch_filter_sweep(R->d_box, R->d_anchor, R->d_xord, nR, S->d_xbox, S->d_xanc, S->d_xord, S->d_xmin,
                                    nS, tau2, w_lo, w_hi, ptr<int32_t>(ctx->b_blk), ptr<int64_t>(ctx->b_blkoff),
                                    d_cr, d_cs, d_lb, d_ub, 1, st));
    return download_cands(ctx, total, cand);
}

KnnGrid knn_grid_params(const pj_meshes *S, int k);

// The set's grid for k (k = 1: the within filter), built on first use on
// this context's stream and kept with the set; later joins, on any context,
// reuse it.
pj_status set_grid(pj_context *ctx, const pj_meshes *S, int k, const pj_meshes::Grid **out)
{
    std::lock_guard<std::mutex> lock(S->grid_mu);
    auto it = S->grids.find(k);
    if (it != S->grids.end()) {
        *out = &it->second;
        return PJ_OK;
    }
    pj_meshes::Grid G;
    G.g = knn_grid_params(S, k);
    G.ncell = (int64_t)G.g.gx * G.g.gy * G.g.gz;
    const int nS = S->n;
    hipStream_t st = ctx->stream;
    hipError_t e;
    if ((e = S->al.alloc((void **)&G.beg, (size_t)(G.ncell + 3 + G.ncell / 4096) * 8)) != hipSuccess)
        return hipfail(ctx, e, "grid cells");
    if ((e = S->al.alloc((void **)&G.items, (size_t)std::max(nS, 1) * 4)) != hipSuccess) {
        S->al.free(G.beg);
        return hipfail(ctx, e, "grid items");
    }
    pj_status ps = ensure(ctx, ctx->b_gcell, (size_t)nS * 4);
    if (ps == PJ_OK) ps = ensure(ctx, ctx->b_gcnt, (size_t)G.ncell * 4);
    if (ps == PJ_OK) ps = ensure(ctx, ctx->b_gfill, (size_t)G.ncell * 4);
    if (ps == PJ_OK) ps = ensure(ctx, ctx->b_total, 16);
    if (ps == PJ_OK) {
        e = launch_grid_build(S->d_anchor, nS, G.g, ptr<int32_t>(ctx->b_gcell), ptr<int32_t>(ctx->b_gcnt), G.beg,
                              ptr<int64_t>(ctx->b_total) + 1, ptr<int32_t>(ctx->b_gfill), G.items, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) ps = hipfail(ctx, e, "grid build");
    }
    if (ps != PJ_OK) {
        S->al.free(G.beg);
        S->al.free(G.items);
        return ps;
    }
    *out = &S->grids.emplace(k, G).first->second;
    return PJ_OK;
}

// Grid filter: the all-pairs test and bounds, applied only to the S objects
// binned (by anchor) in the grid cells each r's box can reach; candidates in
// (r, s) order.
pj_status mbb_filter_grid(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, float tau2, std::vector<Cand> &cand)
{
    hipStream_t st = ctx->stream;
    const int nR = R->n;
    const pj_meshes::Grid *G = nullptr;
    PJTRY(set_grid(ctx, S, 1, &G));
    const KnnGrid g = G->g;
    const int64_t ncell = G->ncell;
    PJTRY(ensure(ctx, ctx->b_total, 16));
    PJTRY(ensure(ctx, ctx->b_blk, (size_t)nR * 4));
    PJTRY(ensure(ctx, ctx->b_blkoff, (size_t)(nR + 3 + nR / 4096) * 8));
    PJTRY(ensure(ctx, ctx->b_fslot, (size_t)nR * kFilterSlots * 4));
    int32_t *slot = ptr<int32_t>(ctx->b_fslot);
    // reach: the largest gap the squared test can keep, rounded up
    const float reach = up_float(std::sqrt((double)tau2) * (1.0 + std::ldexp(1.0, -20)));
    HIPTRY(ctx, launch_filter_grid(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, reach, tau2, g, G->beg,
                                   G->items, ptr<int32_t>(ctx->b_blk), slot, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, 0, st));
    HIPTRY(ctx, launch_scan_large(ptr<int32_t>(ctx->b_blk), ptr<int64_t>(ctx->b_blkoff), ptr<int64_t>(ctx->b_total), nR,
                                  st));
    int64_t total = 0;
    PJTRY(read_cand_total(ctx, total));
    ctx->stats.knn_grid_cells = ncell;
    if (total == 0) return PJ_OK;
    if (total > INT32_MAX) return fail(ctx, PJ_ERR_UNSUPPORTED, "more than 2^31 candidate pairs");
    PJTRY(ensure(ctx, ctx->b_cand_r, total * 16));
    int32_t *d_cr = ptr<int32_t>(ctx->b_cand_r), *d_cs = d_cr + total;
    float *d_lb = reinterpret_cast<float *>(d_cs + total), *d_ub = d_lb + total;
    HIPTRY(ctx, launch_filter_grid(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, reach, tau2, g, G->beg,
                                   G->items, ptr<int32_t>(ctx->b_blk), slot, ptr<int64_t>(ctx->b_blkoff), d_cr, d_cs,
                                   d_lb, d_ub, 1, st));
    return download_cands(ctx, total, cand);
}

// MBB filter on the device: candidates with box gap <= tau.
pj_status mbb_filter(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, double tau, std::vector<Cand> &cand)
{
    cand.clear();
    hipStream_t st = ctx->stream;
    const int nR = R->n, nS = S->n;
    double t2 = tau * (1.0 + std::ldexp(1.0, -20));
    float tau2 = up_float(t2 * t2);
    const bool big = (double)nR * (double)nS > (double)(int64_t(1) << 26);
    if (ctx->cfg.filter_mode == 2) return mbb_filter_sweep(ctx, R, S, tau2, cand);
    if (ctx->cfg.filter_mode == 3 || (ctx->cfg.filter_mode == 0 && big)) return mbb_filter_grid(ctx, R, S, tau2, cand);
    const int gx = (nR + kFiltR - 1) / kFiltR, gy = (nS + kFiltS - 1) / kFiltS;
    const int nb = gx * gy;
    PJTRY(ensure(ctx, ctx->b_blk, nb * sizeof(int32_t)));
    PJTRY(ensure(ctx, ctx->b_blkoff, (nb + 1) * sizeof(int64_t)));
    PJTRY(ensure(ctx, ctx->b_total, 16));
    HIPTRY(ctx, launch_filter(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, nS, tau2, ptr<int32_t>(ctx->b_blk),
                              nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st));
    HIPTRY(ctx, launch_scan_i32_to_i64(ptr<int32_t>(ctx->b_blk), ptr<int64_t>(ctx->b_blkoff), ptr<int64_t>(ctx->b_total),
                                       nb, st));
    int64_t total = 0;
    PJTRY(read_cand_total(ctx, total));
    if (total == 0) return PJ_OK;
    if (total > INT32_MAX) return fail(ctx, PJ_ERR_UNSUPPORTED, "more than 2^31 candidate pairs");
    PJTRY(ensure(ctx, ctx->b_cand_r, total * 16));
    int32_t *d_cr = ptr<int32_t>(ctx->b_cand_r), *d_cs = d_cr + total;
    float *d_lb = reinterpret_cast<float *>(d_cs + total), *d_ub = d_lb + total;
    HIPTRY(ctx, launch_filter(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, nS, tau2, ptr<int32_t>(ctx->b_blk),
                              ptr<int64_t>(ctx->b_blkoff), nullptr, d_cr, d_cs, d_lb, d_ub, 1, st));
    return download_cands(ctx, total, cand);
}

// streamed-side facets per tile: a multiple of 64 so that chunks are blocks
int pick_tile_s(pj_context *ctx) { return ctx->cur.tile_s; }

// per-join reset: counters (the ingest time stays) and the launch shape
pj_status voxel_filter(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, const std::vector<Cand> &cand,
                       std::vector<PairState> &ps, const std::vector<int> &idx, float tau);

void begin_join(pj_context *ctx)
{
    ctx->vmask = nullptr;
    const double ingest = ctx->stats.t_ingest_ms;
    std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->stats.t_ingest_ms = ingest;
    ctx->cur = pj_context::Shape{};
    if (ctx->cfg.tile_s > 0) ctx->cur.tile_s = (ctx->cfg.tile_s + 63) / 64 * 64;
    if (ctx->cfg.waves_per_cu > 0) ctx->cur.wpc = ctx->cfg.waves_per_cu;
    ctx->peak_bytes = ctx->dev_bytes;
}

// Progressive refinement of within-tau candidates (Section 3.1).  `live`
// holds the undecided candidates in index order; each round refines those
// whose first LoD has come and drops the decided ones from the list.
pj_status refine_within(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, double tau, std::vector<Cand> &cand,
                        std::vector<PairState> &ps, std::vector<int> &start_lod, std::vector<int> &live)
{
    const int L = R->L;
    const bool plain = ctx->cfg.schedule == PJ_SCHED_PLAIN;
    const bool fp64 = plain || ctx->cfg.precision == PJ_PREC_FP64;
    const int TS = pick_tile_s(ctx);
    TilePlan pl;
    std::vector<int> act;
    for (int lod = 0; lod < L; ++lod) {
        const bool finest = lod == L - 1;
        act.clear();
        size_t nl = 0;
        for (int i : live)
            if (ps[i].status == ST_UNDEC) {
                live[nl++] = i;
                if (start_lod[i] <= lod) act.push_back(i);
            }
        live.resize(nl);
        if (live.empty()) break;
        if (act.empty()) continue;
        ctx->stats.rounds++;
        if (fp64) {
            plan_tiles(R, S, act, cand, ps, lod, finest, 64, TS, !plain, pl);
            count_planned(ctx, R, S, lod, pl);
            std::vector<ItemOut64> out;
            PJTRY(run_f64(ctx, R, S, pl, plain, out));
            for (size_t k = 0; k < pl.items.size(); ++k) {
                PairState &p = ps[pl.items[k].cand];
                double lb = bits_to_double(out[k].lb), ub = bits_to_double(out[k].ub);
                p.lod_done = lod;
                if (finest) {
                    p.d64 = lb;
                    p.hit64 = out[k].hit;
                    bool in = out[k].hit || (tau > 0.0 && lb <= tau);
                    p.status = in ? ST_CONF : ST_PRUNED;
                } else {
                    double e64 = std::ldexp(p.M, -40);
                    p.LB = std::max(p.LB, lb - e64);
                    p.UB = std::min(p.UB, ub + e64);
                    if (p.UB <= tau) p.status = ST_CONF;
                    else if (p.LB > tau) p.status = ST_PRUNED;
                }
                if (p.status != ST_UNDEC) {
                    ctx->stats.resolved_at_lod[lod]++;
                    p.res_lod = (int8_t)lod;
                }
            }
        } else {
            PJTRY(choose_shape(ctx, R, S, act, cand, ps, lod, finest, (float)tau, true));
            plan_tiles(R, S, act, cand, ps, lod, finest, 64 * kP, ctx->cur.tile_s, true, pl,
                       tile_target(ctx, kPlanWPC));
            count_planned(ctx, R, S, lod, pl);
            std::vector<ItemOut> out;
            PJTRY(run_f32(ctx, R, S, pl, (float)tau, true, out, 0));
            for (size_t k = 0; k < pl.items.size(); ++k) {
                PairState &p = ps[pl.items[k].cand];
                double lb = bits_to_float(out[k].lb), ub = bits_to_float(out[k].ub), e = p.eps;
                p.lod_done = lod;
                if (finest) {
                    if (out[k].hit) p.status = ST_CONF;
                    else if (tau > 0.0 && ub + e <= tau) p.status = ST_CONF;
                    else if (lb - e > tau) p.status = ST_PRUNED;
                    else p.status = ST_BAND;
                } else {
                    p.LB = std::max(p.LB, lb - e);
                    p.UB = std::min(p.UB, ub + e);
                    if (p.UB <= tau) p.status = ST_CONF;
                    else if (p.LB > tau) p.status = ST_PRUNED;
                }
                if (p.status == ST_CONF || p.status == ST_PRUNED) {
                    ctx->stats.resolved_at_lod[lod]++;
                    p.res_lod = (int8_t)lod;
                }
                if (p.status == ST_BAND) p.res_lod = (int8_t)lod;
            }
        }
    }
    // guard band: FP64 with the exact meet test on the facet pairs that can
    // still decide (FP32 lower distance <= tau + eps); they were undecided
    // when the finest round began
    std::vector<int> band;
    for (int i : act)
        if (ps[i].status == ST_BAND) {
            band.push_back(i);
            ps[i].thr = (float)tau + ps[i].eps;
        }
    if (!band.empty()) {
        double tb = now_ms();
        ctx->stats.band_pairs += (int64_t)band.size();
        PJTRY(exact_finest(ctx, R, S, cand, ps, band));
        for (int i : band) {
            PairState &p = ps[i];
            bool in = p.hit64 || (tau > 0.0 && p.d64 <= tau);
            p.status = in ? ST_CONF : ST_PRUNED;
            ctx->stats.resolved_at_lod[L - 1]++;
        }
        ctx->stats.t_band_ms += now_ms() - tb;
    }
    return PJ_OK;
}

// FP64 finest-LoD distances for the given candidates (where not known yet)
pj_status finest_distances(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, std::vector<Cand> &cand,
                           std::vector<PairState> &ps, const std::vector<int> &which)
{
    std::vector<int> need;
    for (int i : which)
        if (!std::isfinite(ps[i].d64) && !ps[i].hit64) {
            need.push_back(i);
            ps[i].thr = INFINITY;
        }
    return exact_finest(ctx, R, S, cand, ps, need);
}

// Features of a candidate pair for the LoD model: MBB gap, tau, anchor
// bound, where tau sits in [gap, anchor bound], and for each LoD l = 0..3 the
// pair's largest hd sum, largest ph sum and log2 of the facet-pair count.
void pair_features(const pj_meshes *R, int r, const pj_meshes *S, int s, double tau, double lb0, double ub0, float *f)
{
    f[0] = (float)std::log1p(std::max(lb0, 0.0));
    f[1] = (float)std::log1p(tau);
    f[2] = (float)std::log1p(std::max(ub0, 0.0));
    f[3] = (float)std::min(1.0, std::max(0.0, (tau - lb0) / std::max(ub0 - lb0, 1e-9)));
    for (int l = 0; l < 4; ++l) {
        const int lr = std::min(l, R->L - 1);
        const float2 a = R->h_lodmax[(int64_t)r * R->L + lr], b = S->h_lodmax[(int64_t)s * S->L + lr];
        const double nr = R->count(r, lr), ns = S->count(s, lr);
        f[4 + 3 * l] = (float)std::log1p((double)a.x + b.x);
        f[5 + 3 * l] = (float)std::log1p((double)a.y + b.y);
        f[6 + 3 * l] = (float)(std::log2(std::max(nr * ns, 1.0)) / 16.0);
    }
}

// Resolution log record: 16 float features, int32 label (deciding LoD), int32 n_lods.
struct LogRec {
    float f[MLP_IN];
    int32_t label, n_lods;
};

// tau_of: per-candidate threshold (k-NN: the query's theta_r) instead of tau
void append_log(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, double tau, const std::vector<Cand> &cand,
                const std::vector<PairState> &ps, const std::vector<float> *tau_of = nullptr)
{
    if (!ctx->cfg.log_path || R->L != 4) return;
    FILE *fp = std::fopen(ctx->cfg.log_path, "ab");
    if (!fp) return;
    for (size_t i = 0; i < cand.size(); ++i) {
        if (ps[i].res_lod < 0) continue;
        LogRec rec;
        pair_features(R, cand[i].r, S, cand[i].s, tau_of ? (double)(*tau_of)[cand[i].r] : tau, ps[i].f_lb,
                      ps[i].f_ub, rec.f);
        rec.label = ps[i].res_lod;
        rec.n_lods = R->L;
        std::fwrite(&rec, sizeof(rec), 1, fp);
    }
    std::fclose(fp);
}

struct ModelFile {
    char magic[4];
    uint32_t version, n_in, n_h, n_out;
    float mean[MLP_IN], stdv[MLP_IN];
};

bool load_model(pj_context *ctx, const char *path)
{
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return false;
    ModelFile h;
    std::vector<float> w(MLP_NPARAM);
    bool ok = std::fread(&h, sizeof(h), 1, fp) == 1 && std::memcmp(h.magic, "PJLM", 4) == 0 && h.version == 1 &&
              h.n_in == MLP_IN && h.n_h == MLP_H && h.n_out == MLP_OUT &&
              std::fread(w.data(), 4, MLP_NPARAM, fp) == (size_t)MLP_NPARAM;
    std::fclose(fp);
    if (!ok) return false;
    for (float x : w)
        if (!std::isfinite(x)) return false;
    ctx->model = w;
    std::memcpy(ctx->feat_mean, h.mean, sizeof(h.mean));
    std::memcpy(ctx->feat_std, h.stdv, sizeof(h.stdv));
    ctx->has_model = true;
    ctx->model_dev = nullptr;
    return true;
}

// First LoD per candidate from the model (learned skip); 0 where undecided
// pairs have no prediction.
pj_status learned_start(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, double tau, const std::vector<Cand> &cand,
                        const std::vector<PairState> &ps, std::vector<int> &start,
                        const std::vector<float> *tau_of = nullptr, const std::vector<int> *live = nullptr)
{
    // the undecided candidates (all of them in `live` when it is given)
    std::vector<int> idx;
    if (live)
        idx = *live;
    else
        for (size_t i = 0; i < cand.size(); ++i)
            if (ps[i].status == ST_UNDEC) idx.push_back((int)i);
    const int n = (int)idx.size();
    if (n == 0) return PJ_OK;
    hipStream_t st = ctx->stream;
    // the features, the network and the choice run on the GPU: only the
    // pairs' ids and bounds go up and the first LoDs come back
    PJTRY(ensure_pinned(ctx, ctx->pin_start, (size_t)n * sizeof(StartIn)));
    StartIn *hin = (StartIn *)ctx->pin_start.p;
    for (int q = 0; q < n; ++q) {
        const Cand &c = cand[idx[q]];
        hin[q] = StartIn{c.r, c.s, ps[idx[q]].f_lb, ps[idx[q]].f_ub, tau_of ? (double)(*tau_of)[c.r] : tau};
    }
    PJTRY(ensure(ctx, ctx->b_tmp0, (size_t)n * sizeof(StartIn)));
    PJTRY(ensure(ctx, ctx->b_tmp1, (size_t)n * 4));
    PJTRY(ensure(ctx, ctx->b_model, (MLP_NPARAM + 2 * MLP_IN) * 4));
    float *dpar = ptr<float>(ctx->b_model);
    int32_t *dstart = ptr<int32_t>(ctx->b_tmp1);
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_tmp0.p, hin, (size_t)n * sizeof(StartIn), hipMemcpyHostToDevice, st));
    if (ctx->model_dev != ctx->b_model.p) {  // the weights and feature scales, once per loaded model
        std::vector<float> hp(MLP_NPARAM + 2 * MLP_IN);
        std::memcpy(hp.data(), ctx->model.data(), MLP_NPARAM * 4);
        std::memcpy(hp.data() + MLP_NPARAM, ctx->feat_mean, MLP_IN * 4);
        std::memcpy(hp.data() + MLP_NPARAM + MLP_IN, ctx->feat_std, MLP_IN * 4);
        HIPTRY(ctx, hipMemcpyAsync(dpar, hp.data(), hp.size() * 4, hipMemcpyHostToDevice, st));
        HIPTRY(ctx, hipStreamSynchronize(st));
        ctx->model_dev = ctx->b_model.p;
    }
    const FeatSide fr{R->d_lodmax, R->d_tcnt, R->L}, fs{S->d_lodmax, S->d_tcnt, S->L};
    HIPTRY(ctx, launch_mlp_start(dpar, dpar + MLP_NPARAM, fr, fs, ptr<StartIn>(ctx->b_tmp0), n, dstart, st));
    int32_t *s0 = (int32_t *)ctx->pin_start.p;  // the inputs have been read by now (same stream)
    HIPTRY(ctx, hipMemcpyAsync(s0, dstart, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    for (int q = 0; q < n; ++q) start[idx[q]] = std::min(std::max(s0[q], 0), R->L - 1);
    return PJ_OK;
}

}  // namespace

extern "C" pj_status pj_join_within(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, double tau, pj_pairs *out)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    if (!out) return fail(ctx, PJ_ERR_INVALID_ARG, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    PJTRY(check_pair_args(ctx, R, S));
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(ctx, PJ_ERR_INVALID_ARG, "tau must be finite and >= 0");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    begin_join(ctx);
    double t0 = now_ms();
    if (R->n == 0 || S->n == 0) {
        ctx->stats.t_total_ms = now_ms() - t0;
        return PJ_OK;
    }
    std::vector<Cand> &cand = ctx->j_cand;
    PJTRY(mbb_filter(ctx, R, S, tau, cand));
    const int nc = (int)cand.size();
    ctx->stats.candidates = nc;
    std::vector<PairState> &ps = ctx->j_ps;
    ps.assign(nc, PairState{});
    std::vector<int> start(nc, 0);
    host_for(ctx, nc, [&](int64_t i) {
        pair_frame(R, cand[i].r, S, cand[i].s, ps[i]);
        ps[i].LB = cand[i].lb0;
        ps[i].UB = cand[i].ub0;
        // the anchors are surface points: their distance bounds d from above
        if (cand[i].ub0 <= tau) ps[i].status = ST_CONF;
        else if (cand[i].lb0 > tau) ps[i].status = ST_PRUNED;
    });
    // the undecided candidates in index order: the later passes visit only
    // these (most candidates are decided by their box bounds)
    std::vector<int> live;
    for (int i = 0; i < nc; ++i) {
        ctx->stats.confirmed_filter += ps[i].status == ST_CONF;
        if (ps[i].status == ST_UNDEC) live.push_back(i);
    }
    if (ctx->cfg.voxels && ctx->cfg.schedule == PJ_SCHED_BATCHED) {
        // voxel-pair filtering of the undecided pairs (Section 3.2)
        PJTRY(voxel_filter(ctx, R, S, cand, ps, live, (float)tau));
        if (ctx->vmask) {
            size_t nl = 0;
            for (int i : live) {
                if (ps[i].UB <= tau) ps[i].status = ST_CONF;
                else if (ps[i].LB > tau) ps[i].status = ST_PRUNED;
                ctx->stats.voxel_decided += ps[i].status != ST_UNDEC;
                if (ps[i].status == ST_UNDEC) live[nl++] = i;
            }
            live.resize(nl);
        }
    }
    for (int i : live) {
        ps[i].f_lb = ps[i].LB;
        ps[i].f_ub = ps[i].UB;
    }
    const bool learned = ctx->cfg.learned_skip && ctx->has_model && R->L == MLP_OUT &&
                         ctx->cfg.schedule == PJ_SCHED_BATCHED;
    if (learned) PJTRY(learned_start(ctx, R, S, tau, cand, ps, start, nullptr, &live));
    double t1 = now_ms();
    ctx->stats.t_filter_ms = t1 - t0;
    PJTRY(refine_within(ctx, R, S, tau, cand, ps, start, live));
    if (!learned) append_log(ctx, R, S, tau, cand, ps);
    ctx->stats.t_refine_ms = now_ms() - t1 - ctx->stats.t_band_ms;
    std::vector<int> res;
    for (int i = 0; i < nc; ++i)
        if (ps[i].status == ST_CONF) res.push_back(i);
    if (ctx->cfg.want_dist) {
        double tb = now_ms();
        PJTRY(finest_distances(ctx, R, S, cand, ps, res));
        ctx->stats.t_band_ms += now_ms() - tb;
    }
    // results in (r, s) order (each pair occurs once): two stable counting
    // passes, by s and then by r, when the result count is comparable to the
    // object counts; otherwise a comparison sort
    if ((int64_t)res.size() * 8 >= (int64_t)R->n + S->n) {
        std::vector<int> tmp(res.size()), cnt((size_t)std::max(R->n, S->n) + 1);
        std::fill(cnt.begin(), cnt.begin() + S->n + 1, 0);
        for (int i : res) cnt[cand[i].s + 1]++;
        for (int k = 0; k < S->n; ++k) cnt[k + 1] += cnt[k];
        for (int i : res) tmp[cnt[cand[i].s]++] = i;
        std::fill(cnt.begin(), cnt.begin() + R->n + 1, 0);
        for (int i : tmp) cnt[cand[i].r + 1]++;
        for (int k = 0; k < R->n; ++k) cnt[k + 1] += cnt[k];
        for (int i : tmp) res[cnt[cand[i].r]++] = i;
    } else {
        std::sort(res.begin(), res.end(), [&](int a, int b) {
            return cand[a].r != cand[b].r ? cand[a].r < cand[b].r : cand[a].s < cand[b].s;
        });
    }
    const int64_t n = (int64_t)res.size();
    out->n = n;
    out->r = (int32_t *)std::malloc(std::max<int64_t>(n, 1) * 4);
    out->s = (int32_t *)std::malloc(std::max<int64_t>(n, 1) * 4);
    if (ctx->cfg.want_dist) out->dist = (double *)std::malloc(std::max<int64_t>(n, 1) * 8);
    if (!out->r || !out->s || (ctx->cfg.want_dist && !out->dist)) {
        pj_pairs_free(out);
        return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "host result allocation");
    }
    for (int64_t k = 0; k < n; ++k) {
        out->r[k] = cand[res[k]].r;
        out->s[k] = cand[res[k]].s;
        if (out->dist) out->dist[k] = ps[res[k]].hit64 ? 0.0 : ps[res[k]].d64;
    }
    ctx->stats.peak_device_bytes = ctx->peak_bytes;
    if (ps.capacity() > (size_t(1) << 20)) {  // hold at most about 100 MB between joins
        std::vector<Cand>().swap(cand);
        std::vector<PairState>().swap(ps);
    }
    ctx->stats.t_total_ms = now_ms() - t0;
    return PJ_OK;
}

extern "C" pj_status pj_join_intersect(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, pj_pairs *out)
{
    return pj_join_within(ctx, R, S, 0.0, out);
}

namespace {

// One pruning round of Algorithm 6 (corrected) on the device for every query.
// Voxel-pair filtering (Section 3.2): Algorithm 1 bounds every voxel pair of
// the candidates in `idx` and takes the minima as the pairs' bounds;
// Algorithm 2 keeps the voxel pairs with lb_v <= ub_o (within-tau: also
// <= tau; a within pair that its voxel bounds decide keeps none) by count,
// scan and compaction.  The candidates are cut into chunks of at most
// kVpChunk voxel pairs so that the lb_v buffer has a fixed size (Algorithm
// 3); the chunks are enqueued back to back on the join stream with two
// alternating input and output sets.  The survivors stay on the device: a
// last kernel per chunk turns them into each candidate's 64 rows of 64 bits
// (R-major), which the refinement kernel reads; only the pairs' bounds
// return to the host, once.  On return every processed candidate's LB/UB
// include the voxel bounds and ctx->vmask points at the rows (a candidate
// that was not processed, or has no survivors because its bounds decided
// it, keeps every voxel pair).
constexpr int64_t kVpChunk = int64_t(1) << 26;

pj_status voxel_filter(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, const std::vector<Cand> &cand,
                       std::vector<PairState> &ps, const std::vector<int> &idx, float tau)
{
    ctx->vmask = nullptr;
    if (!R->has_vox || !S->has_vox || cand.empty()) return PJ_OK;
    const double t0 = now_ms();
    hipStream_t st = ctx->stream;
    for (int b = 0; b < 2; ++b)
        if (!ctx->ev_vcomp[b]) HIPTRY(ctx, hipEventCreateWithFlags(&ctx->ev_vcomp[b], hipEventDisableTiming));
    const int64_t nidx = (int64_t)idx.size();
    // rows of the processed candidates, and each candidate's row index (-1:
    // every voxel pair); under a cap that cannot hold them (and a chunk of
    // the smallest size) the filter is skipped and nothing is restricted
    const int64_t need = align256(nidx * kMaxVox * 8) + align256(cand.size() * 4) +
                         16 * kMaxVox * kMaxVox + 4 * align256(int64_t(1) << 12) + 64 * 1024;
    if (ctx->cfg.mem_cap_bytes > 0 && ctx->dev_bytes + need > ctx->cfg.mem_cap_bytes) return PJ_OK;
    PJTRY(ensure(ctx, ctx->b_vmask, std::max<int64_t>(nidx, 1) * kMaxVox * 8));
    PJTRY(ensure(ctx, ctx->b_vrow, cand.size() * 4));
    HIPTRY(ctx, hipMemsetAsync(ctx->b_vmask.p, 0xff, std::max<int64_t>(nidx, 1) * kMaxVox * 8, st));
    // the row map goes up from pinned memory, which the bounds come back
    // through at the end (the join stream is synchronised before that)
    const size_t tot_off = align256(std::max<int64_t>(nidx, 1) * 8);  // survivors per chunk after the bounds
    PJTRY(ensure_pinned(ctx, ctx->pin_vrow, std::max<size_t>(cand.size() * 4, tot_off + 8 * (size_t)(1 + cand.size()))));
    {
        int32_t *vrow = (int32_t *)ctx->pin_vrow.p;
        std::fill(vrow, vrow + cand.size(), -1);
        for (int64_t q = 0; q < nidx; ++q) vrow[idx[q]] = (int32_t)q;
        HIPTRY(ctx, hipMemcpyAsync(ctx->b_vrow.p, vrow, cand.size() * 4, hipMemcpyHostToDevice, st));
    }
    // voxel pairs per chunk: each costs 4 B of lb_v and 4 B of survivors in
    // each of the two output sets; under a cap, what is left after the pair
    // bounds and per-pair arrays (with room for one growth step)
    int64_t budget = kVpChunk;
    if (ctx->cfg.mem_cap_bytes > 0)
        budget = std::max<int64_t>(kMaxVox * kMaxVox,
                                   std::min<int64_t>(budget, (ctx->cfg.mem_cap_bytes - ctx->dev_bytes - 48 * nidx -
                                                              (int64_t(1) << 18)) / 24));
    // chunks of candidates (in idx order)
    std::vector<std::pair<size_t, size_t>> chunks;
    std::vector<int64_t> nvp(idx.size());
    {
        size_t c0 = 0;
        int64_t acc = 0;
        for (size_t q = 0; q < idx.size(); ++q) {
            const Cand &c = cand[idx[q]];
            nvp[q] = (int64_t)R->h_vcount[c.r] * S->h_vcount[c.s];
            if (q > c0 && (acc + nvp[q] > budget || q - c0 >= (size_t(1) << 20))) {
                chunks.push_back({c0, q});
                c0 = q;
                acc = 0;
            }
            acc += nvp[q];
        }
        if (c0 < idx.size()) chunks.push_back({c0, idx.size()});
    }
    const int nch = (int)chunks.size();
    int64_t max_np = 1, max_vp = 1, vp_total = 0;
    for (auto &ch : chunks) {
        max_np = std::max<int64_t>(max_np, (int64_t)(ch.second - ch.first));
        int64_t a = 0;
        for (size_t q = ch.first; q < ch.second; ++q) a += nvp[q];
        max_vp = std::max(max_vp, a);
        vp_total += a;
    }
    PJTRY(ensure(ctx, ctx->b_vplb, max_vp * 4));
    // pair bounds of every processed candidate (float lb, ub), read back once
    PJTRY(ensure(ctx, ctx->b_vpub, tot_off + 8 * (int64_t)nch));
    int64_t *dtot = (int64_t *)((char *)ctx->b_vpub.p + tot_off);  // survivors per chunk
    // per set: in = cr, cs (int32), vp_off (int64, np + 1); out = count
    // (int32), blk_off (int64, np + 1), survivors (uint32)
    const size_t in_bytes = align256(8 * max_np) + align256(8 * (max_np + 1));
    const size_t out_bytes = align256(4 * max_np) + align256(8 * (max_np + 1)) + align256(4 * max_vp);
    for (int b = 0; b < std::min(nch, 2); ++b) {
        PJTRY(ensure(ctx, ctx->vx_in[b], in_bytes));
        PJTRY(ensure(ctx, ctx->vx_out[b], out_bytes));
        PJTRY(ensure_pinned(ctx, ctx->pin_vin[b], in_bytes));
    }
    const VoxSide vr = R->vox(), vs = S->vox();
    float *op = ptr<float>(ctx->b_vpub);  // [nidx][2]
    for (int c = 0; c < nch; ++c) {
        const int b = c & 1;
        const size_t q0 = chunks[c].first, q1 = chunks[c].second;
        const int np = (int)(q1 - q0);
        // the set's pinned inputs are free once chunk c - 2 has run
        if (c >= 2) HIPTRY(ctx, hipEventSynchronize(ctx->ev_vcomp[b]));
        char *hin = (char *)ctx->pin_vin[b].p, *din = (char *)ctx->vx_in[b].p, *dout = (char *)ctx->vx_out[b].p;
        int32_t *hcr = (int32_t *)hin, *hcs = hcr + max_np;
        int64_t *hoff = (int64_t *)(hin + align256(8 * max_np));
        hoff[0] = 0;
        for (int q = 0; q < np; ++q) {
            hcr[q] = cand[idx[q0 + q]].r;
            hcs[q] = cand[idx[q0 + q]].s;
            hoff[q + 1] = hoff[q] + nvp[q0 + q];
        }
        HIPTRY(ctx, hipMemcpyAsync(din, hin, in_bytes, hipMemcpyHostToDevice, st));
        const int32_t *dcr = (const int32_t *)din, *dcs = dcr + max_np;
        const int64_t *doff = (const int64_t *)(din + align256(8 * max_np));
        int32_t *cnt = (int32_t *)dout;
        int64_t *boff = (int64_t *)(dout + align256(4 * max_np));
        uint32_t *vpairs = (uint32_t *)(dout + align256(4 * max_np) + align256(8 * (max_np + 1)));
        float *olb = op + q0, *oub = op + nidx + q0;
        HIPTRY(ctx, launch_vp_bound(dcr, dcs, doff, np, vr, vs, ptr<float>(ctx->b_vplb), olb, oub, st));
        HIPTRY(ctx, launch_vp_count(dcr, dcs, doff, np, vr, vs, ptr<float>(ctx->b_vplb), olb, oub, tau, cnt, st));
        HIPTRY(ctx, launch_scan_i32_to_i64(cnt, boff, boff + np, np, st));
        HIPTRY(ctx, hipMemcpyAsync(dtot + c, boff + np, 8, hipMemcpyDeviceToDevice, st));
        HIPTRY(ctx, launch_vp_write(dcr, dcs, doff, np, vr, vs, ptr<float>(ctx->b_vplb), olb, oub, tau, boff, vpairs,
                                    st));
        HIPTRY(ctx, launch_vp_rows((int)q0, np, boff, vpairs, ptr<unsigned long long>(ctx->b_vmask), st));
        HIPTRY(ctx, hipEventRecord(ctx->ev_vcomp[b], st));
    }
    // bounds and survivor counts in one copy (the row map upload, ahead on
    // the same stream, has read the pinned buffer by then)
    HIPTRY(ctx, hipMemcpyAsync(ctx->pin_vrow.p, op, tot_off + 8 * (size_t)nch, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    const float *hop = (const float *)ctx->pin_vrow.p;
    const int64_t *htot = (const int64_t *)((const char *)ctx->pin_vrow.p + tot_off);
    for (int c = 0; c < nch; ++c) ctx->stats.vp_kept += htot[c];
    for (int64_t q = 0; q < nidx; ++q) {
        PairState &p = ps[idx[q]];
        p.LB = std::max(p.LB, (double)hop[q]);
        p.UB = std::min(p.UB, (double)hop[nidx + q]);
    }
    if (ctx->cfg.mem_cap_bytes > 0) {
        // under a cap the chunk buffers go back before the LoD rounds
        for (DevBuf *x : {&ctx->b_vplb, &ctx->b_vpub, &ctx->vx_in[0], &ctx->vx_in[1], &ctx->vx_out[0], &ctx->vx_out[1]})
            x->release();
    }
    ctx->vmask = ptr<unsigned long long>(ctx->b_vmask);
    ctx->vrow = ptr<int32_t>(ctx->b_vrow);
    ctx->stats.vp_pairs += vp_total;
    ctx->stats.vp_chunks += nch;
    ctx->stats.t_voxel_ms += now_ms() - t0;
    return PJ_OK;
}

// Grid of the k-NN candidate kernels over S's anchors.  The cell edge is
// about the distance of an S anchor to its k-th nearest neighbour (from a
// sample: 128 anchors against up to 4096 others, scaled by the sampling
// density), so a query finds its k bounds within a few cell shells; at
// most 2^22 cells.
KnnGrid knn_grid_params(const pj_meshes *S, int k)
{
    const int64_t n = S->n;
    const float *a = S->h_anchor.data(), *b = S->h_box.data();
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, w[3] = {0, 0, 0}, M = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            const double x = a[3 * i + c];
            lo[c] = std::min(lo[c], x);
            hi[c] = std::max(hi[c], x);
            w[c] = std::max(w[c], std::max(x - (double)b[6 * i + c], (double)b[6 * i + 3 + c] - x));
            M = std::max(M, std::fabs(x));
        }
    double ext = 0.0;
    for (int c = 0; c < 3; ++c) ext = std::max(ext, hi[c] - lo[c]);
    ext = std::max(ext, 1e-6 * std::max(M, 1.0));
    // k-th neighbour distance on a sample
    const int64_t m = std::min<int64_t>(n, 4096), q = std::min<int64_t>(n, 128);
    std::vector<double> kd;
    std::vector<double> d(m);
    for (int64_t t = 0; t < q; ++t) {
        const int64_t i = t * n / q;
        for (int64_t j = 0; j < m; ++j) {
            const int64_t s = j * n / m;
            const double dx = a[3 * s] - a[3 * i], dy = a[3 * s + 1] - a[3 * i + 1], dz = a[3 * s + 2] - a[3 * i + 2];
            d[j] = std::sqrt(dx * dx + dy * dy + dz * dz);
        }
        const int64_t kk = std::min<int64_t>(m - 1, k);
        std::nth_element(d.begin(), d.begin() + kk, d.end());
        kd.push_back(d[kk]);
    }
    std::nth_element(kd.begin(), kd.begin() + kd.size() / 2, kd.end());
    double c = kd.empty() ? ext : kd[kd.size() / 2] * std::cbrt((double)m / (double)n);
    c = std::max(c, ext / 4096.0);
    auto cells = [&](double cc) {
        double t = 1.0;
        for (int a2 = 0; a2 < 3; ++a2) t *= std::max(1.0, std::ceil((hi[a2] - lo[a2]) / cc + 1e-9));
        return t;
    };
    while (cells(c) > double(1 << 22)) c *= 1.25;
    KnnGrid g;
    g.ox = (float)lo[0];
    g.oy = (float)lo[1];
    g.oz = (float)lo[2];
    g.c = (float)c;
    g.inv_c = (float)(1.0 / c);
    g.gx = (int)std::max(1.0, std::ceil((hi[0] - lo[0]) / c + 1e-9));
    g.gy = (int)std::max(1.0, std::ceil((hi[1] - lo[1]) / c + 1e-9));
    g.gz = (int)std::max(1.0, std::ceil((hi[2] - lo[2]) / c + 1e-9));
    g.wx = (float)w[0] * (1.0f + 0x1p-20f);
    g.wy = (float)w[1] * (1.0f + 0x1p-20f);
    g.wz = (float)w[2] * (1.0f + 0x1p-20f);
    g.M = (float)M;
    return g;
}

// The pruning rule on the host threads (the CPU side of the pruning
// ablation, cfg.knn_prune_host): the same decisions as k_knn_prune, from the
// same snapshot.
void knn_prune_host(pj_context *ctx, int nR, const std::vector<int64_t> &off, const std::vector<Cand> &cand,
                    const std::vector<double> &lb, const std::vector<double> &ub, const std::vector<int8_t> &sti,
                    std::vector<int8_t> &sto, const std::vector<int32_t> &kleft)
{
    host_for(ctx, nR, [&](int64_t r) {
        const int64_t o = off[r], N = off[r + 1] - o;
        const int kl = kleft[r];
        for (int64_t m = 0; m < N; ++m) {
            const int8_t st = sti[o + m];
            if (st != 0 || kl <= 0) {
                sto[o + m] = st != 0 ? st : 2;
                continue;
            }
            const double lbm = lb[o + m], ubm = ub[o + m];
            const int idm = cand[o + m].s;
            int maybe = 0, surely = 0;
            for (int64_t n = 0; n < N; ++n) {
                if (n == m || sti[o + n] != 0) continue;
                const double lbn = lb[o + n], ubn = ub[o + n];
                const int idn = cand[o + n].s;
                maybe += (ubm < lbn || (ubm == lbn && idm < idn)) ? 0 : 1;
                surely += (ubn < lbm || (ubn == lbm && idn < idm)) ? 1 : 0;
            }
            sto[o + m] = maybe < kl ? 1 : (surely >= kl ? 2 : 0);
        }
    });
}

pj_status knn_prune_round(pj_context *ctx, int nR, int k, const std::vector<int64_t> &off,
                          const std::vector<Cand> &cand, std::vector<PairState> &ps)
{
    const double t0 = now_ms();
    hipStream_t st = ctx->stream;
    const int64_t nc = (int64_t)cand.size();
    std::vector<double> lb(nc), ub(nc);
    std::vector<int8_t> sti(nc), sto(nc);
    std::vector<int32_t> kleft(nR, k);
    for (int64_t i = 0; i < nc; ++i) {
        lb[i] = ps[i].LB;
        ub[i] = ps[i].UB;
        sti[i] = ps[i].status;
        if (ps[i].status == ST_CONF) kleft[cand[i].r]--;
    }
    if (ctx->cfg.knn_prune_host) {
        knn_prune_host(ctx, nR, off, cand, lb, ub, sti, sto, kleft);
        for (int64_t i = 0; i < nc; ++i) ps[i].status = sto[i];
        ctx->stats.t_prune_ms += now_ms() - t0;
        return PJ_OK;
    }
    PJTRY(ensure(ctx, ctx->b_klb, nc * 8));
    PJTRY(ensure(ctx, ctx->b_kub, nc * 8));
    PJTRY(ensure(ctx, ctx->b_kst0, nc));
    PJTRY(ensure(ctx, ctx->b_kst1, nc));
    PJTRY(ensure(ctx, ctx->b_kleft, nR * 4));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_klb.p, lb.data(), nc * 8, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_kub.p, ub.data(), nc * 8, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_kst0.p, sti.data(), nc, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_kleft.p, kleft.data(), nR * 4, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, launch_knn_prune(nR, ptr<int64_t>(ctx->b_koff), ptr<double>(ctx->b_klb), ptr<double>(ctx->b_kub),
                                 ptr<int32_t>(ctx->b_cand_s), ptr<int8_t>(ctx->b_kst0), ptr<int8_t>(ctx->b_kst1),
                                 ptr<int32_t>(ctx->b_kleft), st));
    HIPTRY(ctx, hipMemcpyAsync(sto.data(), ctx->b_kst1.p, nc, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    for (int64_t i = 0; i < nc; ++i) ps[i].status = sto[i];
    ctx->stats.t_prune_ms += now_ms() - t0;
    return PJ_OK;
}

}  // namespace

extern "C" pj_status pj_join_knn(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int32_t k, pj_knn *out)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    if (!out) return fail(ctx, PJ_ERR_INVALID_ARG, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    PJTRY(check_pair_args(ctx, R, S));
    if (k < 1) return fail(ctx, PJ_ERR_INVALID_ARG, "k must be >= 1");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    begin_join(ctx);
    const double t0 = now_ms();
    const int nR = R->n, nS = S->n;
    out->n_r = nR;
    out->k = k;
    out->count = (int32_t *)std::calloc(std::max(nR, 1), 4);
    out->s = (int32_t *)std::malloc(std::max<int64_t>((int64_t)nR * k, 1) * 4);
    out->dist = (double *)std::malloc(std::max<int64_t>((int64_t)nR * k, 1) * 8);
    if (!out->count || !out->s || !out->dist) {
        pj_knn_free(out);
        return fail(ctx, PJ_ERR_OUT_OF_MEMORY, "host result allocation");
    }
    for (int64_t i = 0; i < (int64_t)nR * k; ++i) {
        out->s[i] = -1;
        out->dist[i] = NAN;
    }
    if (nR == 0 || nS == 0) {
        ctx->stats.t_total_ms = now_ms() - t0;
        return PJ_OK;
    }
    hipStream_t st = ctx->stream;
    // candidates: theta_r = k-th smallest anchor bound; s with box gap <= theta_r
    PJTRY(ensure(ctx, ctx->b_theta, nR * 4));
    PJTRY(ensure(ctx, ctx->b_blk, nR * 4));
    PJTRY(ensure(ctx, ctx->b_koff, (nR + 1) * 8));
    PJTRY(ensure(ctx, ctx->b_total, 16));
    // candidate generation through a grid over the S anchors, or all pairs
    // (filter_mode 1, or k above what the grid kernel keeps in registers)
    const bool use_grid = ctx->cfg.filter_mode != 1 && k <= kGridMaxK;
    KnnGrid grid;
    const pj_meshes::Grid *G = nullptr;
    if (use_grid) {
        PJTRY(set_grid(ctx, S, k, &G));
        grid = G->g;
        HIPTRY(ctx, launch_knn_theta_grid(R->d_anchor, nR, S->d_anchor, nS, k, grid, G->beg, G->items,
                                          ptr<float>(ctx->b_theta), st));
        HIPTRY(ctx, launch_knn_cand_grid(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, nS, ptr<float>(ctx->b_theta),
                                         grid, G->beg, G->items, ptr<int32_t>(ctx->b_blk), nullptr, nullptr, nullptr,
                                         nullptr, 0, st));
        ctx->stats.knn_grid_cells = G->ncell;
    } else {
        HIPTRY(ctx, launch_knn_theta(R->d_anchor, nR, S->d_anchor, nS, k, ptr<float>(ctx->b_theta), st));
        HIPTRY(ctx, launch_knn_cand(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, nS, ptr<float>(ctx->b_theta),
                                    ptr<int32_t>(ctx->b_blk), nullptr, nullptr, nullptr, nullptr, 0, st));
    }
    HIPTRY(ctx, launch_scan_i32_to_i64(ptr<int32_t>(ctx->b_blk), ptr<int64_t>(ctx->b_koff), ptr<int64_t>(ctx->b_total),
                                       nR, st));
    int64_t total = 0;
    HIPTRY(ctx, hipMemcpyAsync(&total, ctx->b_total.p, 8, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    if (total > INT32_MAX) return fail(ctx, PJ_ERR_UNSUPPORTED, "more than 2^31 k-NN candidates");
    HIPTRY(ctx, hipMemcpyAsync(ptr<int64_t>(ctx->b_koff) + nR, &total, 8, hipMemcpyHostToDevice, st));
    PJTRY(ensure(ctx, ctx->b_cand_s, std::max<int64_t>(total, 1) * 4));
    PJTRY(ensure(ctx, ctx->b_cand_lb, std::max<int64_t>(total, 1) * 4));
    PJTRY(ensure(ctx, ctx->b_cand_ub, std::max<int64_t>(total, 1) * 4));
    if (use_grid)
        HIPTRY(ctx, launch_knn_cand_grid(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, nS,
                                         ptr<float>(ctx->b_theta), grid, G->beg, G->items, nullptr,
                                         ptr<int64_t>(ctx->b_koff),
                                         ptr<int32_t>(ctx->b_cand_s), ptr<float>(ctx->b_cand_lb),
                                         ptr<float>(ctx->b_cand_ub), 1, st));
    else
        HIPTRY(ctx, launch_knn_cand(R->d_box, R->d_anchor, nR, S->d_box, S->d_anchor, nS, ptr<float>(ctx->b_theta),
                                    nullptr, ptr<int64_t>(ctx->b_koff), ptr<int32_t>(ctx->b_cand_s),
                                    ptr<float>(ctx->b_cand_lb), ptr<float>(ctx->b_cand_ub), 1, st));
    std::vector<int64_t> off(nR + 1);
    std::vector<int32_t> cs(total);
    std::vector<float> clb(total), cub(total);
    HIPTRY(ctx, hipMemcpyAsync(off.data(), ctx->b_koff.p, (nR + 1) * 8, hipMemcpyDeviceToHost, st));
    if (total) {
        HIPTRY(ctx, hipMemcpyAsync(cs.data(), ctx->b_cand_s.p, total * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(ctx, hipMemcpyAsync(clb.data(), ctx->b_cand_lb.p, total * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(ctx, hipMemcpyAsync(cub.data(), ctx->b_cand_ub.p, total * 4, hipMemcpyDeviceToHost, st));
    }
    HIPTRY(ctx, hipStreamSynchronize(st));
    std::vector<Cand> cand(total);
    std::vector<PairState> ps(total);
    for (int r = 0; r < nR; ++r)
        for (int64_t i = off[r]; i < off[r + 1]; ++i) {
            cand[i] = Cand{r, cs[i], clb[i], cub[i]};
            pair_frame(R, r, S, cs[i], ps[i]);
            ps[i].LB = clb[i];
            ps[i].UB = cub[i];
        }
    ctx->stats.candidates = total;
    const double t1 = now_ms();
    ctx->stats.t_filter_ms = t1 - t0;
    PJTRY(knn_prune_round(ctx, nR, k, off, cand, ps));
    if (ctx->cfg.voxels && ctx->cfg.schedule == PJ_SCHED_BATCHED) {
        // voxel-pair filtering of the undecided candidates (Section 3.2), then
        // the pruning rule on the tightened intervals
        std::vector<int> und;
        for (int64_t i = 0; i < total; ++i)
            if (ps[i].status == ST_UNDEC) und.push_back((int)i);
        PJTRY(voxel_filter(ctx, R, S, cand, ps, und, -1.0f));
        if (ctx->vmask) {
            PJTRY(knn_prune_round(ctx, nR, k, off, cand, ps));
            for (int i : und) ctx->stats.voxel_decided += ps[i].status != ST_UNDEC;
        }
    }
    const int L = R->L;
    // learned first LoD (the threshold feature of a candidate is its query's
    // theta_r, the k-th smallest anchor bound), and resolution logs of the
    // plain progressive order for training
    const bool learned = ctx->cfg.learned_skip && ctx->has_model && L == MLP_OUT && ctx->cfg.schedule == PJ_SCHED_BATCHED;
    std::vector<int> start(total, 0);
    std::vector<float> theta;
    if (learned || (ctx->cfg.log_path && L == MLP_OUT)) {
        theta.resize(nR);
        HIPTRY(ctx, hipMemcpyAsync(theta.data(), ctx->b_theta.p, (size_t)nR * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(ctx, hipStreamSynchronize(st));
        for (float &x : theta)
            if (!std::isfinite(x)) x = 1e30f;
    }
    for (int64_t i = 0; i < total; ++i) {
        ps[i].f_lb = ps[i].LB;
        ps[i].f_ub = ps[i].UB;
    }
    if (learned) PJTRY(learned_start(ctx, R, S, 0.0, cand, ps, start, &theta));
    // coarse LoD rounds on the undecided candidates
    const int TS = pick_tile_s(ctx);
    const bool plain = ctx->cfg.schedule == PJ_SCHED_PLAIN;
    const bool fp64 = plain || ctx->cfg.precision == PJ_PREC_FP64;
    TilePlan pl;
    // (FP32 schedule: the finest LoD is a round too; its FP32 minimum u also
    // bounds the exact recheck's collect threshold, u + 2 eps)
    for (int lod = 0; lod < (fp64 ? L - 1 : L); ++lod) {
        const bool fin_round = lod == L - 1;
        std::vector<int> act;
        bool any = false;
        for (int64_t i = 0; i < total; ++i)
            if (ps[i].status == ST_UNDEC) {
                any = true;
                if (start[i] <= lod) act.push_back((int)i);
            }
        if (!any) break;
        if (act.empty()) continue;
        ctx->stats.rounds++;
        if (fp64) {
            plan_tiles(R, S, act, cand, ps, lod, 0, 64, TS, !plain, pl);
            count_planned(ctx, R, S, lod, pl);
            std::vector<ItemOut64> o64;
            PJTRY(run_f64(ctx, R, S, pl, plain, o64));
            for (size_t q = 0; q < pl.items.size(); ++q) {
                PairState &p = ps[pl.items[q].cand];
                double e64 = std::ldexp(p.M, -40);
                p.LB = std::max(p.LB, bits_to_double(o64[q].lb) - e64);
                p.UB = std::min(p.UB, bits_to_double(o64[q].ub) + e64);
            }
        } else {
            PJTRY(choose_shape(ctx, R, S, act, cand, ps, lod, fin_round, -1.0f, false));
            plan_tiles(R, S, act, cand, ps, lod, fin_round, 64 * kP, ctx->cur.tile_s, true, pl,
                       tile_target(ctx, kPlanWPC));
            count_planned(ctx, R, S, lod, pl);
            std::vector<ItemOut> o32;
            PJTRY(run_f32(ctx, R, S, pl, -1.0f, false, o32, 0));
            for (size_t q = 0; q < pl.items.size(); ++q) {
                PairState &p = ps[pl.items[q].cand];
                const float u = bits_to_float(o32[q].ub);
                p.LB = std::max(p.LB, (double)bits_to_float(o32[q].lb) - p.eps);
                p.UB = std::min(p.UB, (double)u + p.eps);
                if (fin_round && std::isfinite(u)) p.thr = std::min(p.thr, up_float((double)u + 2.0 * (double)p.eps));
            }
        }
        std::vector<int8_t> before(total);
        for (int64_t i = 0; i < total; ++i) before[i] = ps[i].status;
        PJTRY(knn_prune_round(ctx, nR, k, off, cand, ps));
        for (int64_t i = 0; i < total; ++i)
            if (before[i] == ST_UNDEC && ps[i].status != ST_UNDEC) {
                ctx->stats.resolved_at_lod[lod]++;
                ps[i].res_lod = (int8_t)lod;
            }
    }
    ctx->stats.t_refine_ms = now_ms() - t1;
    // finest LoD: exact FP64 distances of every candidate still in play
    const double t2 = now_ms();
    std::vector<int> fin;
    for (int64_t i = 0; i < total; ++i)
        if (ps[i].status == ST_UNDEC || ps[i].status == ST_CONF) fin.push_back((int)i);
    ctx->stats.rounds++;
    if (plain) {
        plan_tiles(R, S, fin, cand, ps, L - 1, 1, 64, TS, false, pl);
        std::vector<ItemOut64> o64;
        PJTRY(run_f64(ctx, R, S, pl, true, o64));
        for (size_t q = 0; q < pl.items.size(); ++q) {
            PairState &p = ps[pl.items[q].cand];
            p.hit64 = o64[q].hit;
            p.d64 = p.hit64 ? 0.0 : bits_to_double(o64[q].lb);
        }
    } else {
        PJTRY(exact_finest(ctx, R, S, cand, ps, fin));
    }
    for (int i : fin) {
        ps[i].LB = ps[i].UB = ps[i].d64;
    }
    const int undecided_before = (int)std::count_if(fin.begin(), fin.end(), [&](int i) { return ps[i].status == ST_UNDEC; });
    for (int i : fin)
        if (ps[i].status == ST_UNDEC) ps[i].res_lod = (int8_t)(L - 1);
    PJTRY(knn_prune_round(ctx, nR, k, off, cand, ps));
    ctx->stats.resolved_at_lod[L - 1] += undecided_before;
    if (!learned && !theta.empty()) append_log(ctx, R, S, 0.0, cand, ps, &theta);
    ctx->stats.t_band_ms = now_ms() - t2;
    // results: confirmed candidates of each r ordered by (distance, id)
    for (int r = 0; r < nR; ++r) {
        std::vector<std::pair<double, int>> row;
        for (int64_t i = off[r]; i < off[r + 1]; ++i) {
            if (ps[i].status == ST_UNDEC) return fail(ctx, PJ_ERR_INTERNAL, "k-NN pruning left a candidate undecided");
            if (ps[i].status == ST_CONF) row.push_back({ps[i].d64, cand[i].s});
        }
        std::sort(row.begin(), row.end());
        const int want = std::min(k, nS);
        if ((int)row.size() != want) return fail(ctx, PJ_ERR_INTERNAL, "k-NN confirmed count differs from min(k, |S|)");
        out->count[r] = want;
        for (int q = 0; q < want; ++q) {
            out->s[(int64_t)r * k + q] = row[q].second;
            out->dist[(int64_t)r * k + q] = row[q].first;
        }
    }
    ctx->stats.peak_device_bytes = ctx->peak_bytes;
    ctx->stats.t_total_ms = now_ms() - t0;
    return PJ_OK;
}

extern "C" void pj_pairs_free(pj_pairs *p)
{
    if (!p) return;
    std::free(p->r);
    std::free(p->s);
    std::free(p->dist);
    std::memset(p, 0, sizeof(*p));
}

extern "C" void pj_knn_free(pj_knn *p)
{
    if (!p) return;
    std::free(p->count);
    std::free(p->s);
    std::free(p->dist);
    std::memset(p, 0, sizeof(*p));
}

// ===========================================================================
// inspection entry points
// ===========================================================================
extern "C" pj_status pj_facet_pairs(pj_context *ctx, const float *t1, const float *t2, int64_t n, int32_t precision,
                                    double *d, double *d_hi, int8_t *hit)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && (!t1 || !t2 || !d || !d_hi || !hit))) return fail(ctx, PJ_ERR_INVALID_ARG, "bad argument");
    if (precision != PJ_PREC_FP32_BAND && precision != PJ_PREC_FP64) return fail(ctx, PJ_ERR_INVALID_ARG, "precision");
    if (n == 0) return PJ_OK;
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t st = ctx->stream;
    PJTRY(ensure(ctx, ctx->b_tmp0, n * 36));
    PJTRY(ensure(ctx, ctx->b_tmp1, n * 36));
    PJTRY(ensure(ctx, ctx->b_tmp2, n * 16));
    PJTRY(ensure(ctx, ctx->b_tmp3, n));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_tmp0.p, t1, n * 36, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(ctx->b_tmp1.p, t2, n * 36, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, launch_facet_pairs(ptr<float>(ctx->b_tmp0), ptr<float>(ctx->b_tmp1), n, precision,
                                   ptr<double>(ctx->b_tmp2), ptr<double>(ctx->b_tmp2) + n, ptr<int8_t>(ctx->b_tmp3),
                                   st));
    HIPTRY(ctx, hipMemcpyAsync(d, ctx->b_tmp2.p, n * 8, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipMemcpyAsync(d_hi, ptr<double>(ctx->b_tmp2) + n, n * 8, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipMemcpyAsync(hit, ctx->b_tmp3.p, n, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    return PJ_OK;
}

extern "C" pj_status pj_pair_bounds(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int64_t n,
                                    const int32_t *r, const int32_t *s, int32_t lod, double *lb, double *ub,
                                    int8_t *hit)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    PJTRY(check_pair_args(ctx, R, S));
    if (n < 0 || (n > 0 && (!r || !s || !lb || !ub || !hit))) return fail(ctx, PJ_ERR_INVALID_ARG, "bad argument");
    if (n == 0) return PJ_OK;
    if (lod < 0 || lod >= R->L) return fail(ctx, PJ_ERR_INVALID_ARG, "lod out of range");
    for (int64_t i = 0; i < n; ++i)
        if (r[i] < 0 || r[i] >= R->n || s[i] < 0 || s[i] >= S->n) return fail(ctx, PJ_ERR_INVALID_ARG, "object id");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    ctx->vmask = nullptr;  // every facet pair counts here
    std::vector<Cand> cand(n);
    std::vector<PairState> ps(n);
    std::vector<int> act(n);
    for (int64_t i = 0; i < n; ++i) {
        cand[i] = Cand{r[i], s[i], 0.0f, INFINITY};
        pair_frame(R, r[i], S, s[i], ps[i]);
        act[i] = (int)i;
    }
    const bool plain = ctx->cfg.schedule == PJ_SCHED_PLAIN;
    const bool fp64 = plain || ctx->cfg.precision == PJ_PREC_FP64;
    const bool finest = lod == R->L - 1;
    TilePlan pl;
    for (int64_t i = 0; i < n; ++i) {
        lb[i] = INFINITY;
        ub[i] = INFINITY;
        hit[i] = 0;
    }
    if (fp64) {
        plan_tiles(R, S, act, cand, ps, lod, finest, 64, pick_tile_s(ctx), !plain, pl);
        std::vector<ItemOut64> out;
        PJTRY(run_f64(ctx, R, S, pl, plain, out));
        for (size_t k = 0; k < pl.items.size(); ++k) {
            int c = pl.items[k].cand;
            lb[c] = bits_to_double(out[k].lb);
            ub[c] = bits_to_double(out[k].ub);
            hit[c] = (int8_t)out[k].hit;
        }
    } else {
        plan_tiles(R, S, act, cand, ps, lod, finest, 64 * kP, pick_tile_s(ctx), true, pl,
                   tile_target(ctx, kPlanWPC));
        std::vector<ItemOut> out;
        PJTRY(run_f32(ctx, R, S, pl, -1.0f, false, out, 0));
        for (size_t k = 0; k < pl.items.size(); ++k) {
            int c = pl.items[k].cand;
            lb[c] = bits_to_float(out[k].lb);
            ub[c] = bits_to_float(out[k].ub);
            hit[c] = (int8_t)out[k].hit;
        }
    }
    return PJ_OK;
}

// Allocation-free variant of pj_pair_bounds: the FP32 batched path with
// its work lists in this device's fixed scratch array instead of the
// context's grow-only buffers; host arrays move with plain (pageable)
// copies, and the round launches directly (no graph, no pinned staging).
extern "C" pj_status pj_pair_bounds_noalloc(pj_context *ctx, const pj_meshes *R, const pj_meshes *S, int64_t n,
                                            const int32_t *r, const int32_t *s, int32_t lod, double *lb, double *ub,
                                            int8_t *hit)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    PJTRY(check_pair_args(ctx, R, S));
    if (n < 0 || (n > 0 && (!r || !s || !lb || !ub || !hit))) return fail(ctx, PJ_ERR_INVALID_ARG, "bad argument");
    if (n > kNoAllocMaxPairs)
        return fail(ctx, PJ_ERR_INVALID_ARG, "more than " + std::to_string(kNoAllocMaxPairs) +
                                                 " pairs for the allocation-free entry point");
    if (ctx->cfg.precision != PJ_PREC_FP32_BAND || ctx->cfg.schedule != PJ_SCHED_BATCHED)
        return fail(ctx, PJ_ERR_UNSUPPORTED, "the allocation-free entry point runs the FP32 batched path only");
    if (R->host || S->host)
        return fail(ctx, PJ_ERR_UNSUPPORTED, "the allocation-free entry point needs device-resident mesh sets");
    if (n == 0) return PJ_OK;
    if (lod < 0 || lod >= R->L) return fail(ctx, PJ_ERR_INVALID_ARG, "lod out of range");
    for (int64_t i = 0; i < n; ++i)
        if (r[i] < 0 || r[i] >= R->n || s[i] < 0 || s[i] >= S->n) return fail(ctx, PJ_ERR_INVALID_ARG, "object id");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    if (!ctx->scratch) return hipfail(ctx, ctx->scratch_err, "device scratch address");
    std::vector<Cand> cand(n);
    std::vector<PairState> ps(n);
    std::vector<int> act(n);
    for (int64_t i = 0; i < n; ++i) {
        cand[i] = Cand{r[i], s[i], 0.0f, INFINITY};
        pair_frame(R, r[i], S, s[i], ps[i]);
        act[i] = (int)i;
        lb[i] = INFINITY;
        ub[i] = INFINITY;
        hit[i] = 0;
    }
    const int wpc = std::min(ctx->cfg.waves_per_cu > 0 ? ctx->cfg.waves_per_cu : ctx->cur.wpc,
                             kNoAllocMaxGrid / std::max(ctx->num_cu, 1));
    const int grid = ctx->num_cu * wpc;
    if (grid < 1 || grid > kNoAllocMaxGrid) return fail(ctx, PJ_ERR_UNSUPPORTED, "persistent grid beyond the scratch slots");
    // whole-A-side tiles; B ranges lengthened until the tiles fit (one tile
    // per item always does)
    // (the tile-count hint is capped too: a round of few pairs shortens its B
    // ranges only until it has about a quarter of the hint in claimable units)
    TilePlan pl;
    int TS = pick_tile_s(ctx);
    const int64_t hint = std::min<int64_t>(tile_target(ctx, wpc), kNoAllocMaxTiles / 2);
    for (int tries = 0;; ++tries) {
        plan_tiles(R, S, act, cand, ps, lod, lod == R->L - 1, 64 * kP, TS, true, pl, hint);
        if ((int64_t)pl.tiles.size() <= kNoAllocMaxTiles) break;
        if (tries >= 40) return fail(ctx, PJ_ERR_INTERNAL, "no tile plan fits the scratch array");
        TS = TS >= (1 << 29) ? TS : TS * 2;
    }
    const int ni = (int)pl.items.size(), nt = (int)pl.tiles.size();
    if (ni == 0 || nt == 0) return PJ_OK;
    // scratch layout: items | tiles | results | counter block | slots, cursors
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    char *base = (char *)ctx->scratch;
    const size_t o_items = 0, o_tiles = al(o_items + sizeof(Item) * kNoAllocMaxPairs),
                 o_out = al(o_tiles + sizeof(Tile) * kNoAllocMaxTiles), o_ctr = al(o_out + sizeof(ItemOut) * kNoAllocMaxPairs),
                 o_sched = al(o_ctr + 64), o_end = o_sched + 4 * (size_t)(kNoAllocMaxGrid + kNoAllocMaxTiles);
    static_assert(sizeof(Item) * kNoAllocMaxPairs + sizeof(Tile) * kNoAllocMaxTiles + sizeof(ItemOut) * kNoAllocMaxPairs +
                          64 + 4 * (size_t)(kNoAllocMaxGrid + kNoAllocMaxTiles) + 5 * 256 <=
                      kScratchBytes,
                  "scratch layout");
    if (o_end > kScratchBytes) return fail(ctx, PJ_ERR_INTERNAL, "scratch layout");
    hipStream_t st = ctx->stream;
    int32_t hc[16] = {0};  // [1] tiles, [2..5] counters, [6] items, [10] next tile to take
    hc[1] = nt;
    hc[6] = ni;
    int32_t *dctr = (int32_t *)(base + o_ctr);
    HIPTRY(ctx, hipMemcpyAsync(base + o_items, pl.items.data(), ni * sizeof(Item), hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(base + o_tiles, pl.tiles.data(), nt * sizeof(Tile), hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(dctr, hc, sizeof(hc), hipMemcpyHostToDevice, st));
    RefineArgs a;
    std::memset(&a, 0, sizeof(a));
    a.R = R->dev();
    a.S = S->dev();
    a.items = (const Item *)(base + o_items);
    a.tiles = (const Tile *)(base + o_tiles);
    a.ntiles = dctr + 1;
    a.tile_next = dctr + 10;
    a.wave_slot = (int32_t *)(base + o_sched);
    a.tile_cur = a.wave_slot + grid;
    a.out = (ItemOut *)(base + o_out);
    a.pairs_done = reinterpret_cast<unsigned long long *>(dctr + 2);
    a.chunks_culled = reinterpret_cast<unsigned long long *>(dctr + 4);
    a.tau = -1.0f;
    a.early = 0;
    a.cull = ctx->cfg.tile_cull ? 1 : 0;
    PJTRY(launch_round(ctx, a, dctr, ni, nt, wpc, false, st));
    std::vector<ItemOut> out(ni);
    HIPTRY(ctx, hipMemcpyAsync(out.data(), a.out, ni * sizeof(ItemOut), hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    for (int k = 0; k < ni; ++k) {
        const int c = pl.items[k].cand;
        lb[c] = bits_to_float(out[k].lb);
        ub[c] = bits_to_float(out[k].ub);
        hit[c] = (int8_t)out[k].hit;
    }
    return PJ_OK;
}

extern "C" pj_status pj_mlp_eval(pj_context *ctx, const float *params, const float *x, const int32_t *y, int64_t n,
                                 float *logits, float *loss, float *grads)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    if (!params || n < 0 || n > (1 << 24) || (n > 0 && (!x || !logits)) || (y && (!loss || !grads)))
        return fail(ctx, PJ_ERR_INVALID_ARG, "bad argument");
    if (n == 0) return PJ_OK;
    for (int64_t i = 0; y && i < n; ++i)
        if (y[i] < 0 || y[i] >= MLP_OUT) return fail(ctx, PJ_ERR_INVALID_ARG, "label out of range");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t st = ctx->stream;
    const size_t fx = (size_t)n * MLP_IN * 4, fl = (size_t)n * MLP_OUT * 4;
    const size_t scratch = ((size_t)4 * n * MLP_H + (size_t)n * MLP_OUT) * 4;
    PJTRY(ensure(ctx, ctx->b_tmp0, fx + fl + (size_t)n * 8 + MLP_NPARAM * 8));
    PJTRY(ensure(ctx, ctx->b_tmp1, scratch));
    char *base = (char *)ctx->b_tmp0.p;
    float *dx = (float *)base, *dlog = (float *)(base + fx), *dloss = (float *)(base + fx + fl);
    int32_t *dy = (int32_t *)(base + fx + fl + (size_t)n * 4);
    float *dpar = (float *)(base + fx + fl + (size_t)n * 8), *dgr = dpar + MLP_NPARAM;
    HIPTRY(ctx, hipMemcpyAsync(dx, x, fx, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemcpyAsync(dpar, params, MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    if (y) HIPTRY(ctx, hipMemcpyAsync(dy, y, (size_t)n * 4, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, launch_mlp_fwd_bwd(dpar, dx, y ? dy : nullptr, (int)n, dlog, dloss, dgr, ptr<float>(ctx->b_tmp1), st));
    HIPTRY(ctx, hipMemcpyAsync(logits, dlog, fl, hipMemcpyDeviceToHost, st));
    std::vector<float> lp(y ? n : 0);
    if (y) {
        HIPTRY(ctx, hipMemcpyAsync(lp.data(), dloss, (size_t)n * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(ctx, hipMemcpyAsync(grads, dgr, MLP_NPARAM * 4, hipMemcpyDeviceToHost, st));
    }
    HIPTRY(ctx, hipStreamSynchronize(st));
    if (y) {
        double acc = 0.0;
        for (float v : lp) acc += v;
        *loss = (float)(acc / n);
    }
    return PJ_OK;
}

extern "C" pj_status pj_train_lod_model(pj_context *ctx, const char *log_path, const char *model_out,
                                        const pj_train_opts *opts, float *final_loss)
{
    if (!ctx) return PJ_ERR_INVALID_ARG;
    if (!log_path || !model_out) return fail(ctx, PJ_ERR_INVALID_ARG, "NULL path");
    pj_train_opts o = {30, 1024, 3e-3f, 0};
    if (opts) o = *opts;
    if (o.epochs < 1 || o.batch < 1 || !(o.lr > 0.0f)) return fail(ctx, PJ_ERR_INVALID_ARG, "bad training options");
    FILE *fp = std::fopen(log_path, "rb");
    if (!fp) return fail(ctx, PJ_ERR_INVALID_ARG, "cannot open the resolution log");
    std::vector<LogRec> recs;
    LogRec rec;
    while (std::fread(&rec, sizeof(rec), 1, fp) == 1)
        if (rec.n_lods == MLP_OUT && rec.label >= 0 && rec.label < MLP_OUT) recs.push_back(rec);
    std::fclose(fp);
    const int64_t n = (int64_t)recs.size();
    if (n == 0) return fail(ctx, PJ_ERR_INVALID_ARG, "the resolution log holds no usable records");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t st = ctx->stream;
    ModelFile h;
    std::memcpy(h.magic, "PJLM", 4);
    h.version = 1;
    h.n_in = MLP_IN;
    h.n_h = MLP_H;
    h.n_out = MLP_OUT;
    for (int j = 0; j < MLP_IN; ++j) {
        double m = 0.0, v = 0.0;
        for (const LogRec &r : recs) m += r.f[j];
        m /= n;
        for (const LogRec &r : recs) v += (r.f[j] - m) * (r.f[j] - m);
        h.mean[j] = (float)m;
        h.stdv[j] = (float)std::max(std::sqrt(v / n), 1e-6);
    }
    // deterministic initialisation (He-scaled uniform) from the seed
    std::vector<float> par(MLP_NPARAM, 0.0f);
    uint64_t sd = o.seed * 6364136223846793005ull + 1442695040888963407ull;
    auto uni = [&]() {
        sd = sd * 6364136223846793005ull + 1442695040888963407ull;
        return ((sd >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
    };
    const int lay[3][2] = {{MLP_IN, MLP_H}, {MLP_H, MLP_H}, {MLP_H, MLP_OUT}};
    int off = 0;
    for (int l = 0; l < 3; ++l) {
        const double a = std::sqrt(6.0 / lay[l][0]);
        for (int q = 0; q < lay[l][0] * lay[l][1]; ++q) par[off + q] = (float)(a * uni());
        off += lay[l][0] * lay[l][1] + lay[l][1];
    }
    const int B = (int)std::min<int64_t>(o.batch, n);
    const size_t scratch = ((size_t)4 * B * MLP_H + (size_t)B * MLP_OUT) * 4;
    PJTRY(ensure(ctx, ctx->b_tmp0, (size_t)n * MLP_IN * 4 + (size_t)n * 4));
    PJTRY(ensure(ctx, ctx->b_tmp1, scratch));
    PJTRY(ensure(ctx, ctx->b_tmp2, (size_t)MLP_NPARAM * 4 * 4 + (size_t)B * (MLP_OUT + 1) * 4));
    float *dx = ptr<float>(ctx->b_tmp0);
    int32_t *dy = reinterpret_cast<int32_t *>(dx + (size_t)n * MLP_IN);
    float *dpar = ptr<float>(ctx->b_tmp2), *dm = dpar + MLP_NPARAM, *dv = dm + MLP_NPARAM, *dg = dv + MLP_NPARAM;
    float *dlog = dg + MLP_NPARAM, *dloss = dlog + (size_t)B * MLP_OUT;
    HIPTRY(ctx, hipMemcpyAsync(dpar, par.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice, st));
    HIPTRY(ctx, hipMemsetAsync(dm, 0, MLP_NPARAM * 8, st));
    std::vector<float> xs((size_t)n * MLP_IN);
    std::vector<int32_t> ys(n);
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    int step = 0;
    double last = 0.0;
    for (int ep = 0; ep < o.epochs; ++ep) {
        for (int64_t i = n - 1; i > 0; --i) {  // Fisher-Yates with the same generator
            int64_t j = (int64_t)((uni() * 0.5 + 0.5) * (i + 1));
            if (j > i) j = i;
            std::swap(perm[i], perm[j]);
        }
        for (int64_t i = 0; i < n; ++i) {
            const LogRec &r = recs[perm[i]];
            for (int j = 0; j < MLP_IN; ++j) xs[(size_t)i * MLP_IN + j] = (r.f[j] - h.mean[j]) / h.stdv[j];
            ys[i] = r.label;
        }
        HIPTRY(ctx, hipMemcpyAsync(dx, xs.data(), xs.size() * 4, hipMemcpyHostToDevice, st));
        HIPTRY(ctx, hipMemcpyAsync(dy, ys.data(), ys.size() * 4, hipMemcpyHostToDevice, st));
        double ep_loss = 0.0;
        int64_t seen = 0;
        std::vector<float> lp(B);
        for (int64_t b0 = 0; b0 + B <= n; b0 += B) {
            HIPTRY(ctx, launch_mlp_fwd_bwd(dpar, dx + b0 * MLP_IN, dy + b0, B, dlog, dloss, dg, ptr<float>(ctx->b_tmp1),
                                           st));
            HIPTRY(ctx, launch_mlp_adam(dpar, dm, dv, dg, ++step, o.lr, 0.9f, 0.999f, 1e-8f, st));
            if (ep == o.epochs - 1) {
                HIPTRY(ctx, hipMemcpyAsync(lp.data(), dloss, (size_t)B * 4, hipMemcpyDeviceToHost, st));
                HIPTRY(ctx, hipStreamSynchronize(st));
                for (float v : lp) ep_loss += v;
                seen += B;
            }
        }
        if (ep == o.epochs - 1 && seen) last = ep_loss / seen;
    }
    HIPTRY(ctx, hipMemcpyAsync(par.data(), dpar, MLP_NPARAM * 4, hipMemcpyDeviceToHost, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    FILE *wf = std::fopen(model_out, "wb");
    if (!wf) return fail(ctx, PJ_ERR_INVALID_ARG, "cannot write the model file");
    bool ok = std::fwrite(&h, sizeof(h), 1, wf) == 1 && std::fwrite(par.data(), 4, MLP_NPARAM, wf) == (size_t)MLP_NPARAM;
    ok = (std::fclose(wf) == 0) && ok;
    if (!ok) return fail(ctx, PJ_ERR_INTERNAL, "short write of the model file");
    if (final_loss) *final_loss = (float)last;
    ctx->model = par;
    std::memcpy(ctx->feat_mean, h.mean, sizeof(h.mean));
    std::memcpy(ctx->feat_std, h.stdv, sizeof(h.stdv));
    ctx->has_model = true;
    ctx->model_dev = nullptr;
    return PJ_OK;
}

extern "C" pj_status pj_probe_fma(pj_context *ctx, int32_t fp64, double *gflops)
{
    if (!ctx || !gflops) return PJ_ERR_INVALID_ARG;
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    const int blocks = ctx->num_cu * 16, iters = 1 << 16;
    PJTRY(ensure(ctx, ctx->b_tmp0, (size_t)blocks * 256 * 8));
    hipStream_t st = ctx->stream;
    HIPTRY(ctx, launch_fma_probe(fp64, ctx->b_tmp0.p, blocks, 64, st));  // warm-up
    HIPTRY(ctx, hipEventRecord(ctx->ev0, st));
    HIPTRY(ctx, launch_fma_probe(fp64, ctx->b_tmp0.p, blocks, iters, st));
    HIPTRY(ctx, hipEventRecord(ctx->ev1, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    float ms = 0;
    HIPTRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    *gflops = (double)blocks * 256 * iters * 8 * 2 / (ms * 1e-3) / 1e9;
    return PJ_OK;
}

extern "C" pj_status pj_probe_copy(pj_context *ctx, int64_t nbytes, double *gbps)
{
    if (!ctx || !gbps || nbytes <= 0 || nbytes % 16) return fail(ctx, PJ_ERR_INVALID_ARG, "nbytes must be a positive multiple of 16");
    HIPTRY(ctx, hipSetDevice(ctx->cfg.device));
    PJTRY(ensure(ctx, ctx->b_tmp0, nbytes));
    PJTRY(ensure(ctx, ctx->b_tmp1, nbytes));
    hipStream_t st = ctx->stream;
    const int blocks = ctx->num_cu * 8;
    HIPTRY(ctx, hipMemsetAsync(ctx->b_tmp0.p, 0, nbytes, st));
    HIPTRY(ctx, launch_copy_probe(ctx->b_tmp0.p, ctx->b_tmp1.p, nbytes, blocks, st));  // warm-up
    HIPTRY(ctx, hipEventRecord(ctx->ev0, st));
    HIPTRY(ctx, launch_copy_probe(ctx->b_tmp0.p, ctx->b_tmp1.p, nbytes, blocks, st));
    HIPTRY(ctx, hipEventRecord(ctx->ev1, st));
    HIPTRY(ctx, hipStreamSynchronize(st));
    float ms = 0;
    HIPTRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    *gbps = 2.0 * (double)nbytes / (ms * 1e-3) / 1e9;
    return PJ_OK;
}
