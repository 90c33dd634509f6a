// mpcd_engine.hip -- host runtime of libmpcd.so: contexts, box slots,
// device tables, the per-step launch sequence (eager or replayed from a
// captured hipGraph), per-kernel timing, and the C ABI of include/mpcd.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "mpcd.h"
#include "mpcd_dev.h"
#include "mpcd_launch.h"

using namespace mpcd;

#define HIPCHK(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "libmpcd: %s failed: %s (%s:%d)\n", #expr,      \
                    hipGetErrorString(e_), __FILE__, __LINE__);             \
            return MPCD_EDEVICE;                                            \
        }                                                                   \
    } while (0)

namespace {

enum Kern {
    K_MARK, K_ZERO, K_COUNT, K_SCAN, K_SCATTER, K_FLIP, K_BRICK_STEP, K_CELL_ROTATE, K_BOX_FINISH, K_NUM
};
const char* const kKernName[K_NUM] = {
    "mark_holes", "zero_counts", "count", "scan", "scatter", "flip", "brick_step", "cell_rotate",
    "box_finish"};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Slot {
    bool live = false;
    mpcd_box_desc desc{};
    void* mem = nullptr;
    size_t bytes = 0;
    BoxDev dev{};
    int64_t ptiles = 0, ctiles = 0;
    int32_t ntile = 0;               // particle tiles of kPartTile slots
    long long* part = nullptr;       // ntile x kNumDiag partials of the per-box kernels
    double mass_total = 0.0;         // sum of the per-particle masses (MPCD_PARTICLE_MASS)
};

// Pinned staging buffer of an asynchronous upload; reusable once the copy
// that reads it (recorded by `done`) has run.
struct Upload {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

// A replaced step graph: destroyed once the launches queued before the
// replacement (recorded by `done`) have run.
struct Retired {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace

struct mpcd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mpcd_alloc_fn alloc = nullptr;
    mpcd_free_fn free = nullptr;
    void* user = nullptr;
    int64_t budget = 0, used = 0;
    int32_t binning = MPCD_BIN_AUTO;
    int32_t brick[3] = {0, 0, 0};
    bool pending_rebucket = false;
    int* host_flag = nullptr;        // pinned: set by the device when a brick box needs re-bucketing
    int* host_flag_dev = nullptr;    // its device address
    bool tuning = false;             // this context is an autotuner trial context
    std::map<uint64_t, std::pair<int32_t, std::array<int32_t, 3>>> tuned;   // shape class -> choice
    std::vector<std::pair<std::string, double>> tune_log;                  // last trial timings
    bool use_graph = false;
    int max_slots = 4096;
    std::vector<Slot> slots;

    // device tables
    Tables T;
    void* tab_mem = nullptr;         // boxes + state (fixed size, max_slots)
    void* tile_mem = nullptr;        // tiles, active, partials, tilesum
    size_t tile_cap = 0;
    bool dirty = true;
    bool any_brick = false, any_sort = false;

    // graph of one step
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<Retired> retired;

    // host-to-device uploads are stream-ordered through pinned staging
    std::vector<Upload> uploads;

    // profiling
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double prof_ms[K_NUM] = {};
    int64_t prof_n[K_NUM] = {};

    // host copies handed out by mpcd_observe
    std::vector<double> vacf_host;
    std::vector<float> stage;
    std::vector<int32_t> stage_pid;
};

namespace {

// Registers a brick workgroup needs for buckets of `mean` particles on
// average: the mean plus four Poisson standard deviations (larger buckets
// run in a second chunk).
int64_t bucket_need(double mean) { return (int64_t)std::ceil(mean + 4.0 * std::sqrt(mean) + 16.0); }

void* ctx_alloc(mpcd_ctx* c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (c->alloc) return c->alloc(bytes, c->user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void ctx_free(mpcd_ctx* c, void* p)
{
    if (!p) return;
    if (c->free)
        c->free(p, c->user);
    else
        (void)hipFree(p);
}

// Destroy the retired graphs whose queued launches have run (all of them
// with `wait`, after the stream has drained).
void purge_retired(mpcd_ctx* c, bool wait)
{
    size_t keep = 0;
    for (size_t i = 0; i < c->retired.size(); ++i) {
        Retired& r = c->retired[i];
        if (wait || hipEventQuery(r.done) == hipSuccess) {
            if (r.exec) (void)hipGraphExecDestroy(r.exec);
            if (r.graph) (void)hipGraphDestroy(r.graph);
            (void)hipEventDestroy(r.done);
        } else {
            c->retired[keep++] = r;
        }
    }
    c->retired.resize(keep);
}

// Take the current step graph out of use.  Launches of it may still be
// queued on the stream, so it is destroyed later (purge_retired).
int drop_graph(mpcd_ctx* c)
{
    purge_retired(c, false);
    if (!c->graph && !c->graph_exec) return MPCD_OK;
    Retired r{c->graph, c->graph_exec, nullptr};
    c->graph = nullptr;
    c->graph_exec = nullptr;
    if (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r.done, c->stream) != hipSuccess) {
        // no event: wait for the stream instead
        if (r.done) (void)hipEventDestroy(r.done);
        (void)hipStreamSynchronize(c->stream);
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        return MPCD_EDEVICE;
    }
    c->retired.push_back(r);
    return MPCD_OK;
}

// Copy `bytes` host bytes to device address `dst` in stream order: the
// bytes are staged in pinned memory at once (the caller may reuse `src` on
// return) and the copy runs after the work already queued on the stream.
int upload(mpcd_ctx* c, void* dst, const void* src, size_t bytes)
{
    if (bytes == 0) return MPCD_OK;
    constexpr size_t kMaxUploads = 1024;
    Upload* u = nullptr;
    for (Upload& x : c->uploads)
        if (x.cap >= bytes && hipEventQuery(x.done) == hipSuccess) {
            u = &x;
            break;
        }
    if (!u && c->uploads.size() >= kMaxUploads) {
        // all buffers busy or small: wait for the oldest copy, grow its buffer
        u = &c->uploads.front();
        for (Upload& x : c->uploads)
            if (x.cap >= bytes) {
                u = &x;
                break;
            }
        HIPCHK(hipEventSynchronize(u->done));
    }
    if (!u) {
        c->uploads.emplace_back();
        u = &c->uploads.back();
        HIPCHK(hipEventCreateWithFlags(&u->done, hipEventDisableTiming));
    }
    if (u->cap < bytes) {
        if (u->p) HIPCHK(hipHostFree(u->p));
        u->p = nullptr;
        u->cap = 0;
        size_t cap = 4096;
        while (cap < bytes) cap *= 2;
        HIPCHK(hipHostMalloc(&u->p, cap, hipHostMallocDefault));
        u->cap = cap;
    }
    memcpy(u->p, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, u->p, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipEventRecord(u->done, c->stream));
    return MPCD_OK;
}

// Layout of one box's device allocation.
struct Layout {
    size_t off_p[2][6], off_v0, off_pid[2], off_m[2], off_cell, off_rank, off_perm, off_cstart, off_un, off_uam,
        off_esc[2], off_ecnt[2], off_eflag, off_bstart, off_bsize[2], off_vacf, off_part, total;
};

int ntile_of(int64_t nslot) { return (int)std::max<int64_t>(1, (nslot + kPartTile - 1) / kPartTile); }

Layout box_layout(int64_t n, int64_t nslot, int64_t ncell, bool vacf, int vacf_cap, bool brick, const BrickGeom& g,
                  bool masses, bool am, bool ids)
{
    Layout L{};
    size_t o = 0;
    const size_t pf = align256((size_t)nslot * 4);
    for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 6; ++d) { L.off_p[b][d] = o; o += pf; }
    L.off_v0 = o;
    if (vacf) o += align256((size_t)n * 16);
    for (int b = 0; b < 2; ++b) {
        L.off_pid[b] = o;
        if (ids) o += pf;
    }
    for (int b = 0; b < 2; ++b) {
        L.off_m[b] = o;
        if (masses) o += pf;
    }
    L.off_cell = o; o += pf;
    L.off_rank = o; o += pf;
    L.off_perm = o; o += (!brick && !am) ? pf : 0;
    L.off_cstart = o; o += align256((size_t)(ncell + 1) * 4);
    const size_t nbk = brick ? (size_t)g.nbrick : 0;
    L.off_un = o; o += brick ? align256((size_t)ncell * sizeof(CellRot)) : 0;
    L.off_uam = o; o += brick && am ? align256((size_t)ncell * sizeof(CellAm)) : 0;
    for (int b = 0; b < 2; ++b) { L.off_esc[b] = o; o += brick ? align256((size_t)ncell * sizeof(CellAcc)) : 0; }
    for (int b = 0; b < 2; ++b) { L.off_ecnt[b] = o; o += brick && masses ? align256((size_t)ncell * 4) : 0; }
    L.off_eflag = o; o += align256(2 * nbk * 4);
    L.off_bstart = o; o += align256((nbk + 2) * 4);
    for (int b = 0; b < 2; ++b) { L.off_bsize[b] = o; o += align256((nbk + 1) * 4); }
    L.off_vacf = o; o += align256((size_t)std::max(vacf_cap, 1) * 8);
    L.off_part = o; o += align256((size_t)ntile_of(nslot) * kNumDiag * 8);
    L.total = o;
    return L;
}

int validate_desc(const mpcd_box_desc* d)
{
    if (!d) return MPCD_EINVAL;
    int64_t C = 1;
    for (int i = 0; i < 3; ++i) {
        if (d->L[i] < 1 || d->L[i] > 4096) return MPCD_EINVAL;
        C *= d->L[i];
    }
    if (C >= ((int64_t)1 << 31)) return MPCD_EINVAL;
    if (!(d->a > 0.0) || !isfinite(d->a)) return MPCD_EINVAL;
    if (d->n_particles < 0 || d->n_particles >= ((int64_t)1 << 31)) return MPCD_EINVAL;
    if (!(d->dt > 0.0) || !isfinite(d->dt)) return MPCD_EINVAL;
    if (!isfinite(d->alpha)) return MPCD_EINVAL;
    if (!(d->mass > 0.0) || !isfinite(d->mass)) return MPCD_EINVAL;
    if (d->n_steps < 0) return MPCD_EINVAL;
    if (d->flags & ~(MPCD_INIT_MAXWELL | MPCD_INIT_EXTERNAL | MPCD_TRACK_VACF | MPCD_PARTICLE_MASS |
                     MPCD_CONSERVE_L | MPCD_UNORDERED))
        return MPCD_EINVAL;
    // boxes without particle ids can neither follow a particle's VACF nor
    // take masses indexed by particle
    if ((d->flags & MPCD_UNORDERED) && (d->flags & (MPCD_TRACK_VACF | MPCD_PARTICLE_MASS))) return MPCD_EINVAL;
    // range of the exact fixed-point sums (velocity limit kVelocityLimit,
    // masses in [kMassMin, kMassMax], cells of the angular-momentum rule at
    // most 16 long so that its position moments stay in range)
    if ((d->flags & MPCD_PARTICLE_MASS) && !(d->mass >= kMassMin && d->mass <= kMassMax)) return MPCD_EINVAL;
    if ((d->flags & MPCD_CONSERVE_L) && !(d->a <= 16.0)) return MPCD_EINVAL;
    const uint32_t init = d->flags & (MPCD_INIT_MAXWELL | MPCD_INIT_EXTERNAL);
    if (init != MPCD_INIT_MAXWELL && init != MPCD_INIT_EXTERNAL) return MPCD_EINVAL;
    if ((d->flags & MPCD_INIT_MAXWELL) && (!(d->kT > 0.0) || !isfinite(d->kT))) return MPCD_EINVAL;
    // Maxwellian draws stay far inside the velocity limit: thermal speed <= 16
    if ((d->flags & MPCD_INIT_MAXWELL) && !(d->kT / d->mass <= 256.0)) return MPCD_EINVAL;
    if ((d->flags & MPCD_TRACK_VACF) && d->vacf_stride < 1) return MPCD_EINVAL;
    if (d->vacf_capacity < 0) return MPCD_EINVAL;
    for (int i = 0; i < 3; ++i)
        if ((double)d->L[i] * d->a > 1e7) return MPCD_EINVAL;
    return MPCD_OK;
}

int vacf_capacity(const mpcd_box_desc* d)
{
    if (!(d->flags & MPCD_TRACK_VACF)) return 1;
    if (d->vacf_capacity > 0) return d->vacf_capacity;
    if (d->n_steps > 0) return (int)std::min<int64_t>(d->n_steps / d->vacf_stride + 1, 1 << 24);
    return 1024;
}

// Rebuild the device tables (tiles, active list, descriptors) for the live
// slots.  The uploads are stream-ordered, so work already queued still reads
// the old tables; the step graph is replaced.
int rebuild_tables(mpcd_ctx* c)
{
    {
        int rc = drop_graph(c);
        if (rc) return rc;
    }
    std::vector<Tile> pt, ct, bt;
    std::vector<int32_t> active;
    c->any_brick = c->any_sort = false;
    int max_bvol = 0;
    size_t brick_lds = 0;
    bool brick_am = false, brick_wide = false, brick_ids = false;
    int64_t max_bucket = 0;
    bool brick_mass = false;
    int n_brick_boxes = 0, brick_box = -1;
    for (int s = 0; s < (int)c->slots.size(); ++s) {
        Slot& sl = c->slots[s];
        if (!sl.live) continue;
        active.push_back(s);
        BoxDev& b = sl.dev;
        b.ptile0 = (int32_t)pt.size();
        for (int64_t i = 0; i < b.nslot; i += kPartTile)
            pt.push_back(Tile{s, 0, i, std::min<int64_t>(b.nslot, i + kPartTile)});
        b.ptile1 = (int32_t)pt.size();
        b.ctile0 = (int32_t)ct.size();
        for (int64_t i = 0; i < b.ncell; i += kCellTile)
            ct.push_back(Tile{s, 0, i, std::min<int64_t>(b.ncell, i + kCellTile)});
        b.ctile1 = (int32_t)ct.size();
        b.btile0 = (int32_t)bt.size();
        if (b.binning == MPCD_BIN_ATOMIC)
            for (int64_t i = 0; i < b.nbrick; ++i) bt.push_back(Tile{s, 0, i, i + 1});
        b.btile1 = (int32_t)bt.size();
        if (b.binning == MPCD_BIN_SORT) {
            c->any_sort = true;
        } else {
            c->any_brick = true;
            n_brick_boxes += 1;
            brick_box = s;
            max_bvol = std::max(max_bvol, b.bmax[0] * b.bmax[1] * b.bmax[2]);
            // a full brick's bucket, with a 4-sigma Poisson margin, fits one chunk
            max_bucket = std::max<int64_t>(max_bucket, bucket_need((double)b.n * b.bmax[0] * b.bmax[1] * b.bmax[2] /
                                                                   (double)b.ncell));
            brick_mass |= b.m[0] != nullptr;
            brick_am |= b.conserve_l != 0;
            brick_wide |= b.nslot >= ((int64_t)1 << 30);   // byte offsets beyond 32 bits
            brick_ids |= b.pid[0] != nullptr;
            brick_lds = std::max(brick_lds, (size_t)b.bmax[0] * b.bmax[1] * b.bmax[2] *
                                                (b.conserve_l ? kAmCellBytes : kBrickCellBytes));
        }
    }
    const size_t need = align256(pt.size() * sizeof(Tile) + 256) + align256(ct.size() * sizeof(Tile) + 256) +
                        align256(bt.size() * sizeof(Tile) + 256) + align256(active.size() * 4 + 256) +
                        align256(ct.size() * 4 + 256);
    if (need > c->tile_cap) {
        void* m = ctx_alloc(c, need * 5 / 4);
        if (!m) return MPCD_ENOMEM;
        ctx_free(c, c->tile_mem);
        c->tile_mem = m;
        c->tile_cap = need * 5 / 4;
    }
    char* base = (char*)c->tile_mem;
    size_t o = 0;
    c->T.ptiles = (Tile*)(base + o); o += align256(pt.size() * sizeof(Tile) + 256);
    c->T.ctiles = (Tile*)(base + o); o += align256(ct.size() * sizeof(Tile) + 256);
    c->T.btiles = (Tile*)(base + o); o += align256(bt.size() * sizeof(Tile) + 256);
    c->T.active = (int32_t*)(base + o); o += align256(active.size() * 4 + 256);
    c->T.tilesum = (uint32_t*)(base + o);
    c->T.nptiles = (int)pt.size();
    c->T.nctiles = (int)ct.size();
    c->T.nbtiles = (int)bt.size();
    c->T.brick_box = n_brick_boxes == 1 ? brick_box : -1;
    c->T.nactive = (int)active.size();
    c->T.max_bvol = max_bvol;
    c->T.brick_shape = brick_shape_for(max_bucket);
    c->T.brick_mass = brick_mass;
    c->T.brick_am = brick_am;
    c->T.brick_wide = brick_wide;
    c->T.brick_ids = brick_ids;
    c->T.brick_lds = brick_lds;
    c->T.host_flag = c->host_flag_dev;
    // one upload for the tile lists (laid out as on the device) and one for
    // the box descriptors of every slot in use
    const size_t tiles_bytes = (size_t)((char*)c->T.tilesum - base);
    std::vector<char> host(tiles_bytes, 0);
    auto put = [&](void* dev, const void* src, size_t bytes) {
        if (bytes) memcpy(host.data() + ((char*)dev - base), src, bytes);
    };
    put(c->T.ptiles, pt.data(), pt.size() * sizeof(Tile));
    put(c->T.ctiles, ct.data(), ct.size() * sizeof(Tile));
    put(c->T.btiles, bt.data(), bt.size() * sizeof(Tile));
    put(c->T.active, active.data(), active.size() * 4);
    int rc = upload(c, base, host.data(), tiles_bytes);
    if (rc) return rc;
    if (!c->slots.empty()) {
        std::vector<BoxDev> devs(c->slots.size());
        for (size_t s = 0; s < c->slots.size(); ++s) devs[s] = c->slots[s].dev;
        rc = upload(c, c->T.boxes, devs.data(), devs.size() * sizeof(BoxDev));
        if (rc) return rc;
    }
    c->dirty = false;
    return MPCD_OK;
}

hipEvent_t get_event(mpcd_ctx* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int harvest(mpcd_ctx* c)
{
    if (c->pending.empty()) return MPCD_OK;
    HIPCHK(hipEventSynchronize(c->pending.back().second.second));
    for (auto& p : c->pending) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        c->prof_ms[p.first] += ms;
        c->prof_n[p.first] += 1;
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    c->pending.clear();
    return MPCD_OK;
}

template <class F>
int timed(mpcd_ctx* c, int k, F&& launch)
{
    if (!c->profiling) {
        launch();
        return MPCD_OK;
    }
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return MPCD_EDEVICE;
    HIPCHK(hipEventRecord(a, c->stream));
    launch();
    HIPCHK(hipEventRecord(b, c->stream));
    c->pending.push_back({k, {a, b}});
    return MPCD_OK;
}

// The launch sequence of one step for every live box.  with_sort adds the
// counting sort that re-buckets brick boxes flagged for it (fresh state, or
// a bucket that overflowed).
int enqueue_step(mpcd_ctx* c, bool with_sort)
{
    const Tables& T = c->T;
    hipStream_t s = c->stream;
    int rc = MPCD_OK;
#define STEP_K(id, call)                                       \
    do {                                                       \
        rc = timed(c, id, [&] { call; });                      \
        if (rc) return rc;                                     \
    } while (0)
    if (c->any_sort || with_sort) {
        if (with_sort && c->any_brick) {
            STEP_K(K_MARK, launch_mark_holes(T.ptiles, T.nptiles, T, 0, s); launch_rebucket_clear(T, s));
        }
        STEP_K(K_ZERO, launch_zero_counts(T, s));
        STEP_K(K_COUNT, launch_count(T, s));
        STEP_K(K_SCAN, launch_scan(T, s));
        STEP_K(K_SCATTER, launch_scatter(T, s));
        STEP_K(K_FLIP, launch_flip(T, s));
    }
    if (c->any_brick) STEP_K(K_BRICK_STEP, launch_brick_step(T, s));
    if (c->any_sort) STEP_K(K_CELL_ROTATE, launch_cell_rotate(T, s));
    STEP_K(K_BOX_FINISH, launch_box_finish(T, s));
#undef STEP_K
    HIPCHK(hipGetLastError());
    return MPCD_OK;
}

int capture_graph(mpcd_ctx* c)
{
    int rc0 = drop_graph(c);
    if (rc0) return rc0;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_step(c, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    HIPCHK(e);
    c->graph = g;
    HIPCHK(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    return MPCD_OK;
}

Slot* live_slot(mpcd_ctx* c, int32_t slot)
{
    if (!c || slot < 0 || slot >= (int)c->slots.size() || !c->slots[slot].live) return nullptr;
    return &c->slots[slot];
}

// Mark the holes of brick box s's current buffer (pid -1), so that passes
// over all its slots see only particles.
void mark_holes(mpcd_ctx* c, int32_t s)
{
    const Slot& sl = c->slots[s];
    if (sl.dev.binning != MPCD_BIN_ATOMIC) return;
    launch_mark_holes_box(c->T, s, sl.ntile, c->stream);
}

// Bucket description of a brick box whose particles sit in slots [0, n) of
// buffer `parity` in no particular order (all in bucket 0, the rest of the
// buffer an empty overflow bucket), with no pending escape sums; the next
// step re-buckets it.  Stream-ordered.
int set_compact_layout(mpcd_ctx* c, int32_t s, int parity)
{
    const Slot& sl = c->slots[s];
    const BoxDev& b = sl.dev;
    if (b.binning != MPCD_BIN_ATOMIC) return MPCD_OK;
    const size_t nbk = (size_t)b.nbrick;
    std::vector<uint32_t> start(nbk + 2, (uint32_t)b.n), size(nbk + 1, 0u);
    start[0] = 0u;
    start[nbk + 1] = (uint32_t)b.nslot;
    size[0] = (uint32_t)b.n;
    int rc = upload(c, b.bstart, start.data(), start.size() * 4);
    if (!rc) rc = upload(c, b.bsize[parity], size.data(), size.size() * 4);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(b.bsize[parity ^ 1], 0, (nbk + 1) * 4, c->stream));
    for (int k = 0; k < 2; ++k) HIPCHK(hipMemsetAsync(b.esc[k], 0, (size_t)b.ncell * sizeof(CellAcc), c->stream));
    for (int k = 0; k < 2; ++k)
        if (b.ecnt[k]) HIPCHK(hipMemsetAsync(b.ecnt[k], 0, (size_t)b.ncell * 4, c->stream));
    HIPCHK(hipMemsetAsync(b.eflag, 0, 2 * nbk * 4, c->stream));
    return MPCD_OK;
}

// Write a fresh BoxState for slot s (stream-ordered).
int reset_state(mpcd_ctx* c, int32_t s, int64_t step, int parity)
{
    Slot& sl = c->slots[s];
    BoxState st{};
    st.k = step;
    st.remaining = sl.desc.n_steps > 0 ? std::max<int64_t>(sl.desc.n_steps - step, 0) : -1;
    st.vacf_origin = step;
    st.parity = parity;
    st.vacf_len = 0;
    st.status = 0;
    st.rebucket = (sl.dev.binning == MPCD_BIN_ATOMIC) ? 1 : 0;
    st.adj[3] = 1.0f;
    if (st.rebucket) c->pending_rebucket = true;
    return upload(c, &c->T.state[s], &st, sizeof(BoxState));
}

// Diagnostics of the current state into the box state (exact sums, status);
// with new_origin also v0 <- v (if tracked) and VACF sample 0.  Queued on
// the stream; nothing is read back here.
int take_snapshot(mpcd_ctx* c, int32_t s, bool new_origin = true)
{
    Slot& sl = c->slots[s];
    mark_holes(c, s);
    launch_snapshot(c->T, s, sl.ntile, new_origin ? 1 : 0, sl.part, c->stream);
    launch_box_stats(c->T, s, sl.ntile, sl.part, kStatsSnapshot | (new_origin ? kStatsOrigin : 0), 0.0, 0.0,
                     c->stream);
    HIPCHK(hipGetLastError());
    return MPCD_OK;
}

// Maxwell-Boltzmann initial state at temperature kT: uniform positions and
// Gaussian velocities, then the mean velocity removed and the velocities
// rescaled to the exact temperature.  All on the device.
int init_maxwell(mpcd_ctx* c, int32_t s)
{
    Slot& sl = c->slots[s];
    const double vs = sqrt(sl.desc.kT / sl.desc.mass);
    launch_init_maxwell(c->T, s, sl.ntile, (float)vs, sl.part, c->stream);
    launch_box_stats(c->T, s, sl.ntile, sl.part, kStatsCentre, sl.desc.kT, sl.desc.mass, c->stream);
    launch_init_adjust(c->T, s, sl.ntile, sl.part, c->stream);
    launch_box_stats(c->T, s, sl.ntile, sl.part, kStatsScale, sl.desc.kT, sl.desc.mass, c->stream);
    launch_init_adjust(c->T, s, sl.ntile, sl.part, c->stream);
    HIPCHK(hipGetLastError());
    return MPCD_OK;
}

}  // namespace

// the descriptor check, for the host leg (mpcd_host.hip)
int mpcd::validate_box_desc(const mpcd_box_desc* d) { return validate_desc(d); }

// ==========================================================================
// Autotuner: picks the binning (brick or sort) and the brick shape.  Boxes
// below 2^21 cells, and boxes whose buffers reach 2^30 slots, take the shape
// the density rule gives; for the others a class of boxes is timed once on
// short trial runs of a proxy box of the same density and time step (at most
// 128^3 cells) in a private context on the same stream, and a candidate
// replaces the rule's shape only when clearly faster.  Results do not depend
// on the choice (cell sums are exact), only the speed does.

static uint64_t shape_class(const mpcd_box_desc* d)
{
    const double C = (double)d->L[0] * d->L[1] * d->L[2];
    const int lc = (int)std::floor(std::log2(std::max(1.0, C)));
    const double dens = std::max(1e-3, (double)d->n_particles / C);
    const int rho = (int)std::lround(std::min(255.0, std::max(0.0, 2.0 * std::log2(dens) + 20.0)));
    const double vth = d->kT > 0 ? std::sqrt(d->kT / d->mass) : 1.0;
    const int step = (int)std::min(15.0, std::floor(8.0 * d->dt * vth / d->a));   // free path / cell
    const uint64_t rule = (d->flags & MPCD_CONSERVE_L) ? 1 : 0;   // angular-momentum rule
    const uint64_t ids = (d->flags & MPCD_UNORDERED) ? 0 : 1;     // particle ids travel
    return (ids << 33) | (rule << 32) | ((uint64_t)lc << 16) | ((uint64_t)rho << 4) | (uint64_t)step;
}

static int trial_ms(mpcd_ctx* parent, const mpcd_box_desc* proxy, int32_t binning, const int32_t brick[3],
             double* ms)
{
    mpcd_options o{};
    o.binning = binning;
    for (int k = 0; k < 3; ++k) o.brick[k] = brick[k];
    o.stream = parent->stream;
    o.alloc = parent->alloc;
    o.free = parent->free;
    o.user = parent->user;
    o.device = parent->device;
    o.max_slots = 1;
    mpcd_ctx* t = nullptr;
    int rc = mpcd_create(&o, &t);
    if (rc) return rc;
    t->tuning = true;
    int32_t slot = -1;
    rc = mpcd_admit(t, proxy, &slot);
    if (!rc) rc = mpcd_step(t, 3);   // bucket + warm up
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = MPCD_EDEVICE;
    // the faster of two timed runs of `reps` steps
    for (int round = 0; round < 2 && !rc; ++round) {
        const int reps = 8;
        (void)hipEventRecord(e0, t->stream);
        rc = mpcd_step(t, reps);
        (void)hipEventRecord(e1, t->stream);
        float f = 0.0f;
        if (!rc && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&f, e0, e1) == hipSuccess)
            *ms = round == 0 ? f / reps : std::min(*ms, (double)f / reps);
        else if (!rc)
            rc = MPCD_EDEVICE;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    mpcd_destroy(t);
    return rc;
}

// Brick shapes by volume; the step's cost depends mostly on the particles
// per brick, so the shape follows the density: the largest brick whose
// expected bucket (with its Poisson margin) fits kRuleBucket particles, the
// registers of a 256 x 8 workgroup in one chunk.  Larger bricks mean fewer
// particles crossing brick faces and fewer workgroups; measured on 256^3
// boxes they beat the next smaller brick whenever their bucket fits
// (density 7.1: 8x8x4 bricks 13.8 ps per particle-step against 17.0 for
// 8x4x4; density 12: 8x4x4 14.2 against 15.0 for 4x4x4), and a 512-box
// ensemble runs 5 % faster than with a 1536-particle limit.
constexpr int64_t kRuleBucket = 2048;
static const int32_t kRuleShapes[][3] = {{2, 2, 2}, {4, 2, 2}, {4, 4, 2}, {4, 4, 4}, {8, 4, 4},
                                         {8, 8, 4}, {8, 8, 8}, {16, 8, 8}};
constexpr int kNumRuleShapes = (int)(sizeof(kRuleShapes) / sizeof(kRuleShapes[0]));

static int rule_volume(int i) { return kRuleShapes[i][0] * kRuleShapes[i][1] * kRuleShapes[i][2]; }

// angular-momentum boxes: bricks of at most kMaxAmBrickCells cells
static bool rule_allowed(int i, bool am) { return !am || rule_volume(i) <= kMaxAmBrickCells; }

static int rule_shape(double density, bool am)
{
    const int64_t fit = kRuleBucket;
    int best = 0;
    for (int i = 0; i < kNumRuleShapes; ++i)
        if (rule_allowed(i, am) && bucket_need(rule_volume(i) * density) <= fit) best = i;
    return best;
}

static int autotune(mpcd_ctx* c, const mpcd_box_desc* d, int32_t* binning, int32_t brick[3])
{
    const double C = (double)d->L[0] * d->L[1] * d->L[2];
    const double density = (double)d->n_particles / C;
    const bool am = (d->flags & MPCD_CONSERVE_L) != 0;
    const int r = rule_shape(density, am);
    // defaults, also used inside trial contexts, for empty and for small boxes
    *binning = MPCD_BIN_ATOMIC;
    for (int k = 0; k < 3; ++k) brick[k] = kRuleShapes[r][k];
    if (c->tuning || d->n_particles == 0 || C < (double)(1 << 21)) return MPCD_OK;
    // boxes whose buffers need 64-bit offsets run a different instance than
    // any proxy: the rule decides
    if (brick_slots(d->n_particles, brick_geometry(d->L, brick).nbrick) >= ((int64_t)1 << 30)) return MPCD_OK;
    const uint64_t key = shape_class(d);
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        *binning = it->second.first;
        for (int k = 0; k < 3; ++k) brick[k] = it->second.second[k];
        return MPCD_OK;
    }
    // large boxes: time the rule's shape, its neighbours and sort binning on
    // a proxy box of the same density and time step (at most 128^3 cells)
    mpcd_box_desc p = *d;
    double cells = 1.0;
    for (int k = 0; k < 3; ++k) {
        p.L[k] = std::min(d->L[k], 128);
        cells *= p.L[k];
    }
    p.n_particles = std::max<int64_t>(1, std::llround(density * cells));
    p.flags = MPCD_INIT_MAXWELL | (d->flags & (MPCD_CONSERVE_L | MPCD_PARTICLE_MASS | MPCD_UNORDERED));
    if (!(p.kT > 0.0) || !(p.kT / p.mass <= 256.0)) p.kT = p.mass;   // thermal speed 1
    p.n_steps = 0;
    p.vacf_stride = 0;
    p.vacf_capacity = 0;
    struct Cand { int32_t bin; int32_t b[3]; std::string name; };
    std::vector<Cand> cands;
    for (int i = std::max(0, r - 1); i <= std::min(kNumRuleShapes - 1, r + 1); ++i) {
        if (!rule_allowed(i, am)) continue;
        const int32_t* sh = kRuleShapes[i];
        cands.push_back({MPCD_BIN_ATOMIC, {sh[0], sh[1], sh[2]},
                         "brick" + std::to_string(sh[0]) + "x" + std::to_string(sh[1]) + "x" + std::to_string(sh[2])});
    }
    cands.push_back({MPCD_BIN_SORT, {0, 0, 0}, "sort"});
    c->tune_log.clear();
    // the rule's shape stays unless another candidate is at least 10% faster
    // on the proxy (trial timings carry noise, and the proxy's ranking of
    // close candidates does not always carry over to the full box)
    double best = 1e300, rule_ms = 1e300;
    std::vector<double> ms_of(cands.size(), 1e300);
    for (size_t i = 0; i < cands.size(); ++i) {
        const Cand& cd = cands[i];
        double ms = 0.0;
        const int rc = trial_ms(c, &p, cd.bin, cd.b, &ms);
        if (rc == MPCD_EDEVICE) return rc;
        if (rc) continue;   // e.g. over memory: skip the candidate
        c->tune_log.push_back({cd.name, ms});
        ms_of[i] = ms;
        if (cd.bin == MPCD_BIN_ATOMIC && cd.b[0] == kRuleShapes[r][0] && cd.b[1] == kRuleShapes[r][1] &&
            cd.b[2] == kRuleShapes[r][2])
            rule_ms = ms;
    }
    for (size_t i = 0; i < cands.size(); ++i)
        best = std::min(best, ms_of[i]);
    if (best * 1.10 >= rule_ms) best = rule_ms;   // keep the rule (already in *binning / brick)
    else
        for (size_t i = 0; i < cands.size(); ++i)
            if (ms_of[i] == best) {
                *binning = cands[i].bin;
                for (int k = 0; k < 3; ++k) brick[k] = cands[i].b[k];
                break;
            }
    c->tuned[key] = {*binning, {brick[0], brick[1], brick[2]}};
    return MPCD_OK;
}

// ==========================================================================
// C ABI

extern "C" {

int mpcd_abi_version(void) { return MPCD_ABI_VERSION; }

const char* mpcd_strerror(int status)
{
    switch (status) {
        case MPCD_OK: return "ok";
        case MPCD_EINVAL: return "invalid argument";
        case MPCD_ENOMEM: return "device memory budget exceeded or allocation failed";
        case MPCD_EDEVICE: return "HIP runtime error";
        case MPCD_EBUSY: return "no free slot";
        case MPCD_ESTATE: return "non-finite state detected";
        case MPCD_ENOTFOUND: return "slot not live";
        default: return "unknown status";
    }
}

int mpcd_create(const mpcd_options* opt, mpcd_ctx** out)
{
    if (!out) return MPCD_EINVAL;
    *out = nullptr;
    mpcd_options o{};
    if (opt) o = *opt;
    if (o.binning < 0 || o.binning > 2 || o.hbm_budget < 0 || o.max_slots < 0) return MPCD_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!brick_edge_ok(o.brick[d])) return MPCD_EINVAL;
    if (o.block != 0) return MPCD_EINVAL;
    if ((o.alloc == nullptr) != (o.free == nullptr)) return MPCD_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MPCD_EDEVICE;
    if (o.device < 0 || o.device >= ndev) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(o.device));
    mpcd_ctx* c = new mpcd_ctx();
    c->device = o.device;
    c->alloc = o.alloc;
    c->free = o.free;
    c->user = o.user;
    c->budget = o.hbm_budget;
    c->binning = o.binning;
    for (int d = 0; d < 3; ++d) c->brick[d] = o.brick[d];
    c->use_graph = o.use_graph != 0;
    c->max_slots = o.max_slots > 0 ? o.max_slots : 4096;
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return MPCD_EDEVICE;
        }
        c->own_stream = true;
    }
    const size_t tab = align256(sizeof(BoxDev) * c->max_slots) + align256(sizeof(BoxState) * c->max_slots) +
                       align256(sizeof(long long) * kAccLanes * 3 * c->max_slots);
    c->tab_mem = ctx_alloc(c, tab);
    if (!c->tab_mem) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return MPCD_ENOMEM;
    }
    if (hipHostMalloc((void**)&c->host_flag, sizeof(int), hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&c->host_flag_dev, c->host_flag, 0) != hipSuccess) {
        if (c->host_flag) (void)hipHostFree(c->host_flag);
        ctx_free(c, c->tab_mem);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return MPCD_EDEVICE;
    }
    *c->host_flag = 0;
    c->T.boxes = (BoxDev*)c->tab_mem;
    c->T.state = (BoxState*)((char*)c->tab_mem + align256(sizeof(BoxDev) * c->max_slots));
    c->T.dacc = (long long*)((char*)c->T.state + align256(sizeof(BoxState) * c->max_slots));
    if (hipMemset(c->T.dacc, 0, sizeof(long long) * kAccLanes * 3 * c->max_slots) != hipSuccess) {
        ctx_free(c, c->tab_mem);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        (void)hipHostFree(c->host_flag);
        delete c;
        return MPCD_EDEVICE;
    }
    *out = c;
    return MPCD_OK;
}

int mpcd_admit(mpcd_ctx* c, const mpcd_box_desc* d, int32_t* slot)
{
    if (!c || !slot) return MPCD_EINVAL;
    int rc = validate_desc(d);
    if (rc) return rc;
    int s = -1;
    for (int i = 0; i < (int)c->slots.size(); ++i)
        if (!c->slots[i].live) { s = i; break; }
    if (s < 0) {
        if ((int)c->slots.size() >= c->max_slots) return MPCD_EBUSY;
        s = (int)c->slots.size();
    }
    const bool vacf = (d->flags & MPCD_TRACK_VACF) != 0;
    const int64_t ncell = (int64_t)d->L[0] * d->L[1] * d->L[2];
    const int cap = vacf_capacity(d);
    int32_t binning = c->binning;
    int32_t want[3] = {c->brick[0], c->brick[1], c->brick[2]};
    if (binning == MPCD_BIN_AUTO) {
        rc = autotune(c, d, &binning, want);
        if (rc) return rc;
    }
    BrickGeom g = brick_geometry(d->L, want);
    const bool am = (d->flags & MPCD_CONSERVE_L) != 0;
    if (binning == MPCD_BIN_ATOMIC && g.bvol > (am ? kMaxAmBrickCells : kMaxBrickCells)) return MPCD_EINVAL;
    // bucket starts are 32-bit: beyond 2^32 slots the box uses the counting sort
    if (binning == MPCD_BIN_ATOMIC && brick_slots(d->n_particles, g.nbrick) >= ((int64_t)1 << 32))
        binning = MPCD_BIN_SORT;
    const bool brick = binning == MPCD_BIN_ATOMIC;
    const int64_t nslot = brick ? brick_slots(d->n_particles, g.nbrick) : d->n_particles;
    const bool masses = (d->flags & MPCD_PARTICLE_MASS) != 0;
    const bool ids = (d->flags & MPCD_UNORDERED) == 0;
    const Layout L = box_layout(d->n_particles, nslot, ncell, vacf, cap, brick, g, masses, am, ids);
    if (c->budget > 0 && c->used + (int64_t)L.total > c->budget) return MPCD_ENOMEM;
    HIPCHK(hipSetDevice(c->device));
    void* mem = ctx_alloc(c, L.total);
    if (!mem) return MPCD_ENOMEM;

    Slot sl;
    sl.live = true;
    sl.desc = *d;
    sl.mem = mem;
    sl.bytes = L.total;
    sl.ntile = ntile_of(nslot);
    sl.part = (long long*)((char*)mem + L.off_part);
    BoxDev& b = sl.dev;
    char* m = (char*)mem;
    for (int p = 0; p < 2; ++p) {
        for (int k = 0; k < 6; ++k) b.p[p][k] = (float*)(m + L.off_p[p][k]);
        b.pid[p] = ids ? (int32_t*)(m + L.off_pid[p]) : nullptr;
        b.m[p] = masses ? (float*)(m + L.off_m[p]) : nullptr;
    }
    b.v0 = vacf ? (float4*)(m + L.off_v0) : nullptr;
    b.cell = (uint32_t*)(m + L.off_cell);
    b.rank = (uint32_t*)(m + L.off_rank);
    b.perm = (!brick && !am) ? (uint32_t*)(m + L.off_perm) : nullptr;
    b.cstart = (uint32_t*)(m + L.off_cstart);
    b.un = brick ? (CellRot*)(m + L.off_un) : nullptr;
    b.uam = brick && am ? (CellAm*)(m + L.off_uam) : nullptr;
    for (int p = 0; p < 2; ++p) {
        b.esc[p] = brick ? (CellAcc*)(m + L.off_esc[p]) : nullptr;
        b.ecnt[p] = brick && masses ? (uint32_t*)(m + L.off_ecnt[p]) : nullptr;
        b.bsize[p] = brick ? (uint32_t*)(m + L.off_bsize[p]) : nullptr;
    }
    b.eflag = brick ? (uint32_t*)(m + L.off_eflag) : nullptr;
    b.bstart = brick ? (uint32_t*)(m + L.off_bstart) : nullptr;
    for (int k = 0; k < 3; ++k) {
        b.nb[k] = brick ? g.nb[k] : 1;
        b.bshift[k] = brick ? g.shift[k] : 0;
        b.bmax[k] = brick ? g.bmax[k] : d->L[k];
        b.sshift[k] = kSortBlockShift;
    }
    b.nbrick = brick ? g.nbrick : 0;
    b.nslot = nslot;
    b.vacf = (double*)(m + L.off_vacf);
    b.n = d->n_particles;
    b.ncell = ncell;
    for (int k = 0; k < 3; ++k) {
        b.L[k] = d->L[k];
        b.len[k] = (float)(d->L[k] * d->a);
    }
    b.vacf_stride = vacf ? d->vacf_stride : 0;
    b.vacf_cap = cap;
    b.binning = binning;
    b.conserve_l = (d->flags & MPCD_CONSERVE_L) ? 1 : 0;
    b.a = (float)d->a;
    b.inv_a = (float)(1.0 / d->a);
    b.dt = (float)d->dt;
    b.ca = cos(d->alpha);
    b.sa = sin(d->alpha);
    b.mass = (float)d->mass;
    b.key0 = (uint32_t)(d->seed & 0xffffffffu);
    b.key1 = (uint32_t)(d->seed >> 32);
    if (s == (int)c->slots.size())
        c->slots.push_back(sl);
    else
        c->slots[s] = sl;

    // Everything below is queued on the stream (nothing waits for the steps
    // in flight); the box joins the step tables at the next mpcd_step.  Only
    // its own descriptor is needed by the per-box kernels now.
    auto undo = [&](int code) {
        c->slots[s].live = false;
        ctx_free(c, mem);
        return code;
    };
    c->dirty = true;
    rc = upload(c, &c->T.boxes[s], &c->slots[s].dev, sizeof(BoxDev));
    if (rc) return undo(rc);
    // zeroed cell accumulators and a defined particle state
    Slot& S = c->slots[s];
    if (brick) {
        if (hipMemsetAsync(S.dev.un, 0, ncell * sizeof(CellRot), c->stream) != hipSuccess)
            return undo(MPCD_EDEVICE);
        rc = set_compact_layout(c, s, 0);
        if (rc) return undo(rc);
    }
    rc = reset_state(c, s, 0, 0);
    if (rc) return undo(rc);
    if (masses) {
        launch_fill_f32(S.dev.m[0], S.dev.n, (float)d->mass, c->stream);
        S.mass_total = (double)(float)d->mass * (double)S.dev.n;
    }
    if (d->flags & MPCD_INIT_MAXWELL) {
        rc = init_maxwell(c, s);
    } else {
        for (int k = 0; k < 6; ++k)
            if (hipMemsetAsync(S.dev.p[0][k], 0, (size_t)S.dev.nslot * 4, c->stream) != hipSuccess)
                return undo(MPCD_EDEVICE);
        if (S.dev.pid[0]) launch_fill_iota(S.dev.pid[0], S.dev.n, c->stream);
    }
    if (rc) return undo(rc);
    rc = take_snapshot(c, s);
    if (rc) return undo(rc);
    c->used += (int64_t)L.total;
    *slot = s;
    return MPCD_OK;
}

int mpcd_step(mpcd_ctx* c, int32_t n)
{
    if (!c || n < 0) return MPCD_EINVAL;
    if (n == 0) return MPCD_OK;
    HIPCHK(hipSetDevice(c->device));
    if (c->dirty) {
        int rc = rebuild_tables(c);
        if (rc) return rc;
    }
    if (c->T.nactive == 0) return MPCD_OK;
    // a bucket overflowed in an earlier step: the boxes concerned carry the
    // rebucket flag; re-bucket them in the next step
    if (__atomic_exchange_n(c->host_flag, 0, __ATOMIC_ACQ_REL) != 0) c->pending_rebucket = true;
    if (c->pending_rebucket) {   // bucket fresh brick boxes, then one eager step
        int rc = enqueue_step(c, true);
        if (rc) return rc;
        c->pending_rebucket = false;
        if (--n == 0) return MPCD_OK;
    }
    const bool graph = c->use_graph && !c->profiling;
    if (graph && !c->graph_exec) {
        int rc = capture_graph(c);
        if (rc) return rc;
    }
    for (int i = 0; i < n; ++i) {
        if (graph) {
            HIPCHK(hipGraphLaunch(c->graph_exec, c->stream));
        } else {
            int rc = enqueue_step(c, false);
            if (rc) return rc;
            if (c->pending.size() > 4096) {
                rc = harvest(c);
                if (rc) return rc;
            }
        }
    }
    return MPCD_OK;
}

int mpcd_observe(mpcd_ctx* c, int32_t slot, mpcd_observables* out)
{
    if (!c || !out) return MPCD_EINVAL;
    Slot* sl = live_slot(c, slot);
    if (!sl) return MPCD_ENOTFOUND;
    HIPCHK(hipSetDevice(c->device));
    // momentum and energy of the current state (exact sums over the box)
    int rc = take_snapshot(c, slot, false);
    if (rc) return rc;
    BoxState st;
    HIPCHK(hipMemcpyAsync(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->vacf_host.assign((size_t)std::max(st.vacf_len, 0), 0.0);
    if (st.vacf_len > 0)
        HIPCHK(hipMemcpy(c->vacf_host.data(), sl->dev.vacf, (size_t)st.vacf_len * 8, hipMemcpyDeviceToHost));
    // the kernels sum m v and m v^2 with m = 1 for equal masses
    const bool masses = sl->dev.m[0] != nullptr;
    const double m = masses ? 1.0 : sl->desc.mass;
    const int64_t n = sl->dev.n;
    const double M = masses ? sl->mass_total : sl->desc.mass * (double)n;
    memset(out, 0, sizeof(*out));
    out->step = st.k;
    for (int d = 0; d < 3; ++d) out->P[d] = m * st.diag[d];
    out->E_kin = 0.5 * m * st.diag[3];
    out->mass_total = M;
    if (n > 1 && M > 0) {
        const double P2 = out->P[0] * out->P[0] + out->P[1] * out->P[1] + out->P[2] * out->P[2];
        out->T = (m * st.diag[3] - P2 / M) / (3.0 * (double)(n - 1));
    }
    out->status = st.status ? MPCD_ESTATE : MPCD_OK;
    out->vacf_len = st.vacf_len;
    out->vacf = c->vacf_host.empty() ? nullptr : c->vacf_host.data();
    out->n_particles = n;
    out->binning = sl->dev.binning;
    for (int d = 0; d < 3; ++d) out->brick[d] = sl->dev.binning == MPCD_BIN_ATOMIC ? sl->dev.bmax[d] : 0;
    out->overflow_steps = st.overflow_steps;
    out->rebuckets = st.rebuckets;
    return out->status;
}

int mpcd_get_state(mpcd_ctx* c, int32_t slot, float* xyzv, int64_t* step)
{
    Slot* sl = live_slot(c, slot);
    if (!c || !xyzv) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    HIPCHK(hipSetDevice(c->device));
    BoxState st;
    HIPCHK(hipMemcpyAsync(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = sl->dev.n, ns = sl->dev.nslot;
    mark_holes(c, slot);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stage.resize((size_t)ns);
    c->stage_pid.resize((size_t)ns);
    if (n > 0 && sl->dev.pid[st.parity]) {   // particle-id order
        HIPCHK(hipMemcpy(c->stage_pid.data(), sl->dev.pid[st.parity], (size_t)ns * 4, hipMemcpyDeviceToHost));
        int64_t seen = 0;
        for (int64_t i = 0; i < ns; ++i) {
            const int32_t id = c->stage_pid[i];
            if (id >= n) return MPCD_ESTATE;
            seen += id >= 0;
        }
        if (seen != n) return MPCD_ESTATE;
        for (int d = 0; d < 6; ++d) {
            HIPCHK(hipMemcpy(c->stage.data(), sl->dev.p[st.parity][d], (size_t)ns * 4, hipMemcpyDeviceToHost));
            float* dst = xyzv + (size_t)d * n;
            for (int64_t i = 0; i < ns; ++i) {
                const int32_t id = c->stage_pid[i];
                if (id >= 0) dst[id] = c->stage[i];
            }
        }
    } else if (n > 0) {   // no ids: storage order, holes (x = -1) left out
        std::vector<int64_t> live;
        live.reserve((size_t)n);
        HIPCHK(hipMemcpy(c->stage.data(), sl->dev.p[st.parity][0], (size_t)ns * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < ns; ++i)
            if (!(c->stage[i] < 0.0f)) live.push_back(i);
        if ((int64_t)live.size() != n) return MPCD_ESTATE;
        for (int d = 0; d < 6; ++d) {
            if (d > 0)
                HIPCHK(hipMemcpy(c->stage.data(), sl->dev.p[st.parity][d], (size_t)ns * 4, hipMemcpyDeviceToHost));
            float* dst = xyzv + (size_t)d * n;
            for (int64_t j = 0; j < n; ++j) dst[j] = c->stage[live[j]];
        }
    }
    if (step) *step = st.k;
    return MPCD_OK;
}

int mpcd_set_state(mpcd_ctx* c, int32_t slot, const float* xyzv, int64_t step)
{
    Slot* sl = live_slot(c, slot);
    if (!c || !xyzv || step < 0) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    const int64_t n = sl->dev.n;
    for (int d = 0; d < 3; ++d) {
        const float len = sl->dev.len[d];
        const float* p = xyzv + (size_t)d * n;
        for (int64_t i = 0; i < n; ++i)
            if (!(p[i] >= 0.0f && p[i] < len)) return MPCD_EINVAL;
    }
    for (int64_t i = 3 * n; i < 6 * n; ++i)
        if (!isfinite(xyzv[i])) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (n > 0 && sl->dev.m[0]) {   // masses back into particle-id order, in buffer 0
        BoxState st;
        HIPCHK(hipMemcpy(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost));
        const int par = st.parity;
        mark_holes(c, slot);
        launch_permute_f32(sl->dev.m[par ^ 1], sl->dev.m[par], sl->dev.pid[par], sl->dev.nslot, n, 1, c->stream);
        if (par == 0)
            HIPCHK(hipMemcpyAsync(sl->dev.m[0], sl->dev.m[1], (size_t)n * 4, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    if (n > 0) {
        for (int d = 0; d < 6; ++d)
            HIPCHK(hipMemcpy(sl->dev.p[0][d], xyzv + (size_t)d * n, (size_t)n * 4, hipMemcpyHostToDevice));
        if (sl->dev.pid[0]) launch_fill_iota(sl->dev.pid[0], n, c->stream);
        HIPCHK(hipGetLastError());
    }
    {
        int rc = set_compact_layout(c, slot, 0);
        if (rc) return rc;
    }
    int rc = reset_state(c, slot, step, 0);
    if (rc) return rc;
    rc = take_snapshot(c, slot);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));
    return MPCD_OK;
}

int mpcd_set_mass(mpcd_ctx* c, int32_t slot, const float* mass)
{
    Slot* sl = live_slot(c, slot);
    if (!c || !mass) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    if (!sl->dev.m[0]) return MPCD_EINVAL;
    const int64_t n = sl->dev.n;
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(mass[i] >= kMassMin && mass[i] <= kMassMax)) return MPCD_EINVAL;
        total += mass[i];
    }
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (n > 0) {
        BoxState st;
        HIPCHK(hipMemcpy(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost));
        const int par = st.parity;
        // stage the id-ordered masses in the idle buffer, then gather by id
        mark_holes(c, slot);
        HIPCHK(hipMemcpyAsync(sl->dev.m[par ^ 1], mass, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
        launch_permute_f32(sl->dev.m[par], sl->dev.m[par ^ 1], sl->dev.pid[par], sl->dev.nslot, n, 0, c->stream);
        HIPCHK(hipGetLastError());
    }
    sl->mass_total = total;
    int rc = take_snapshot(c, slot, false);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));
    return MPCD_OK;
}

int mpcd_get_mass(mpcd_ctx* c, int32_t slot, float* mass)
{
    Slot* sl = live_slot(c, slot);
    if (!c || !mass) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    if (!sl->dev.m[0]) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    BoxState st;
    HIPCHK(hipMemcpyAsync(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = sl->dev.n, ns = sl->dev.nslot;
    if (n == 0) return MPCD_OK;
    mark_holes(c, slot);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stage.resize((size_t)ns);
    c->stage_pid.resize((size_t)ns);
    HIPCHK(hipMemcpy(c->stage_pid.data(), sl->dev.pid[st.parity], (size_t)ns * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(c->stage.data(), sl->dev.m[st.parity], (size_t)ns * 4, hipMemcpyDeviceToHost));
    int64_t seen = 0;
    for (int64_t i = 0; i < ns; ++i) {
        const int32_t id = c->stage_pid[i];
        if (id >= n) return MPCD_ESTATE;
        if (id >= 0) {
            mass[id] = c->stage[i];
            ++seen;
        }
    }
    return seen == n ? MPCD_OK : MPCD_ESTATE;
}

int mpcd_get_vacf(mpcd_ctx* c, int32_t slot, float* v0, int64_t* origin, double* samples, int32_t max,
                  int32_t* len)
{
    Slot* sl = live_slot(c, slot);
    if (!c || max < 0 || (max > 0 && !samples)) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    if (sl->dev.vacf_stride <= 0) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    BoxState st;
    HIPCHK(hipMemcpyAsync(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = sl->dev.n;
    if (v0 && n > 0) {
        std::vector<float> rec((size_t)n * 4);
        HIPCHK(hipMemcpy(rec.data(), sl->dev.v0, (size_t)n * 16, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) v0[(size_t)d * n + i] = rec[(size_t)i * 4 + d];
    }
    const int32_t k = std::min<int32_t>(std::max(st.vacf_len, 0), max);
    if (k > 0) HIPCHK(hipMemcpy(samples, sl->dev.vacf, (size_t)k * 8, hipMemcpyDeviceToHost));
    if (origin) *origin = st.vacf_origin;
    if (len) *len = st.vacf_len;
    return MPCD_OK;
}

int mpcd_set_vacf(mpcd_ctx* c, int32_t slot, const float* v0, int64_t origin, const double* samples, int32_t len)
{
    Slot* sl = live_slot(c, slot);
    if (!c || !v0 || !samples) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    const BoxDev& b = sl->dev;
    if (b.vacf_stride <= 0 || len < 1 || len > b.vacf_cap || origin < 0) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    BoxState st;
    HIPCHK(hipMemcpyAsync(&st, &c->T.state[slot], sizeof(BoxState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    // sample j belongs to step origin + j stride: a series that reaches the
    // box's current step holds exactly this many samples
    if (origin > st.k || (st.k - origin) / b.vacf_stride + 1 != len) return MPCD_EINVAL;
    const int64_t n = b.n;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!isfinite(v0[i])) return MPCD_EINVAL;
    for (int32_t j = 0; j < len; ++j)
        if (!isfinite(samples[j])) return MPCD_EINVAL;
    if (n > 0) {
        std::vector<float> rec((size_t)n * 4, 0.0f);
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) rec[(size_t)i * 4 + d] = v0[(size_t)d * n + i];
        HIPCHK(hipMemcpy(b.v0, rec.data(), (size_t)n * 16, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(b.vacf, samples, (size_t)len * 8, hipMemcpyHostToDevice));
    st.vacf_origin = origin;
    st.vacf_len = len;
    HIPCHK(hipMemcpy(&c->T.state[slot], &st, sizeof(BoxState), hipMemcpyHostToDevice));
    return MPCD_OK;
}

int mpcd_moments(const float* vx, const float* vy, const float* vz, const float* mass, int64_t n, double* out,
                 void* stream)
{
    if (!out || n < 0 || (n > 0 && (!vx || !vy || !vz))) return MPCD_EINVAL;
    if (n > ((int64_t)INT32_MAX) * kPartTile) return MPCD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t ntile = std::max<int64_t>(1, (n + kPartTile - 1) / kPartTile);
    long long* part = nullptr;
    HIPCHK(hipMalloc((void**)&part, (size_t)ntile * kNumDiag * sizeof(long long)));
    launch_moments(vx, vy, vz, mass, n, part, out, s);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);   // the workspace is freed once the kernels have run
    (void)hipFree(part);
    if (e1 != hipSuccess || e2 != hipSuccess) return MPCD_EDEVICE;
    return MPCD_OK;
}

// Workspace of mpcd_moments_noalloc: the partials of at most
// kMomentsMaxTiles particle tiles (n <= 2^28 particles; 3.5 MiB), one copy
// per GPU, held until the process ends.  Host code never uses the array's
// name as an address: each device's address comes from hipGetSymbolAddress,
// taken once per device with that device current.
constexpr int64_t kMomentsMaxTiles = 65536;
static __device__ __align__(256) long long scratch[kMomentsMaxTiles * kNumDiag];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
long long* scratch_ptr[kMaxDevices] = {};

// scratch's address on the current device (looked up on its first use there)
int scratch_address(long long** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MPCD_EDEVICE;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return MPCD_EDEVICE;
        scratch_ptr[dev] = (long long*)p;
    }
    *out = scratch_ptr[dev];
    return MPCD_OK;
}
}  // namespace

int mpcd_moments_noalloc(const float* vx, const float* vy, const float* vz, const float* mass, int64_t n,
                         double* out, void* stream)
{
    if (!out || n < 0 || (n > 0 && (!vx || !vy || !vz))) return MPCD_EINVAL;
    if (n > kMomentsMaxTiles * kPartTile) return MPCD_EINVAL;
    long long* part = nullptr;
    const int rc = scratch_address(&part);
    if (rc) return rc;
    launch_moments(vx, vy, vz, mass, n, part, out, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return MPCD_OK;
}

int mpcd_hbm_copy(const void* src, void* dst, size_t bytes, int32_t blocks, void* stream)
{
    if (!src || !dst || blocks < 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15)) return MPCD_EINVAL;
    if (bytes == 0) return MPCD_OK;
    launch_hbm_copy(src, dst, (int64_t)(bytes / 16), blocks > 0 ? blocks : 8192, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return MPCD_OK;
}

int mpcd_release(mpcd_ctx* c, int32_t slot)
{
    Slot* sl = live_slot(c, slot);
    if (!c) return MPCD_EINVAL;
    if (!sl) return MPCD_ENOTFOUND;
    HIPCHK(hipSetDevice(c->device));
    // Steps already queued may still read this box: the caller's allocator
    // is stream-ordered (its memory is reused only by later work on the
    // stream) and hipFree waits for the device, so the memory can go now.
    // The tables are rebuilt before the next step.
    ctx_free(c, sl->mem);
    c->used -= (int64_t)sl->bytes;
    sl->live = false;
    sl->mem = nullptr;
    c->dirty = true;
    return MPCD_OK;
}

int mpcd_profile(mpcd_ctx* c, int32_t enable)
{
    if (!c) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    int rc = harvest(c);
    if (rc) return rc;
    if (enable) {
        for (int k = 0; k < K_NUM; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_n[k] = 0;
        }
    }
    c->profiling = enable != 0;
    return MPCD_OK;
}

int mpcd_kernel_stats(mpcd_ctx* c, mpcd_kernel_stat* out, int32_t max, int32_t* count)
{
    if (!c || !count || max < 0 || (max > 0 && !out)) return MPCD_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    int rc = harvest(c);
    if (rc) return rc;
    int n = 0;
    for (int k = 0; k < K_NUM; ++k) {
        if (c->prof_n[k] == 0) continue;
        if (n < max) {
            out[n].name = kKernName[k];
            out[n].launches = c->prof_n[k];
            out[n].total_ms = c->prof_ms[k];
        }
        ++n;
    }
    *count = n;
    return MPCD_OK;
}

void mpcd_destroy(mpcd_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)harvest(c);
    (void)drop_graph(c);
    purge_retired(c, true);
    for (Upload& u : c->uploads) {
        if (u.p) (void)hipHostFree(u.p);
        if (u.done) (void)hipEventDestroy(u.done);
    }
    for (auto& sl : c->slots)
        if (sl.live) ctx_free(c, sl.mem);
    ctx_free(c, c->tile_mem);
    ctx_free(c, c->tab_mem);
    if (c->host_flag) (void)hipHostFree(c->host_flag);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
