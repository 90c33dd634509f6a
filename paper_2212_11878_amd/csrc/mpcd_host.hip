// mpcd_host.hip -- the SRD step of one box on the host's cores (host code
// only): the CPU leg of hybrid CPU+GPU execution (paper Sec. 3.2 and Sec. 4,
// Fig. 2f, where some ranks of a run compute on CPU cores next to the GPUs).
//
// The method is the GPU path's: streaming with the periodic fold, the random
// grid shift s_k and the per-cell rotation axes from the same Philox4x32-10
// streams keyed by the seed, exact 64-bit fixed-point cell sums, the cell's
// collision map built in FP64 (cell_rotation) and applied in FP32
// (apply_rotation).  Binning is a counting sort by collision cell each step
// (the GPU's SORT binning): stream and key every particle, count per cell,
// scan, scatter into cell order, then collide every cell's contiguous run.
// The arithmetic helpers are the ones the kernels use (mpcd_dev.h); only the
// axis goes through the host's sinf/cosf/sqrtf instead of the device
// library, so a host axis can differ from the GPU's in the last bit.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <system_error>
#include <thread>
#include <vector>

#include "mpcd.h"
#include "mpcd_dev.h"
#include "mpcd_launch.h"

namespace mpcd {
namespace {

// Rotation axis of canonical cell c at step k: the recipe of cell_axis
// (z uniform in [-1, 1), azimuth uniform, one Newton step on the inverse
// norm) with the host's math library.
float3 host_cell_axis(const BoxDev& b, long long k, uint32_t c)
{
    const uint4 q = philox4x32_10(
        make_uint4((uint32_t)k, c, (uint32_t)((unsigned long long)k >> 32), 1u), b.key0, b.key1);
    const float z = 2.0f * unit24(q.x) - 1.0f;
    const float phi = 6.2831853071795864769f * unit24(q.y);
    const float sp = sinf(phi), cp = cosf(phi);
    const float rho = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    const float nx = rho * cp, ny = rho * sp, nz = z;
    const float nn = nx * nx + ny * ny + nz * nz;
    float r = 1.0f / sqrtf(nn);
    r = r * (1.5f - 0.5f * nn * r * r);
    return make_float3(nx * r, ny * r, nz * r);
}

// A barrier for the threads of one call (sense-reversing, spinning with
// yields: phases are short and the team is at most the machine's cores).
class Barrier {
public:
    explicit Barrier(int n) : n_(n) {}
    void wait()
    {
        const int gen = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
            count_.store(0, std::memory_order_relaxed);
            gen_.store(gen + 1, std::memory_order_release);
            return;
        }
        while (gen_.load(std::memory_order_acquire) == gen) std::this_thread::yield();
    }

private:
    const int n_;
    std::atomic<int> count_{0};
    std::atomic<int> gen_{0};
};

// [begin, end) of part t of n items split over T parts
inline void part_of(int64_t n, int t, int T, int64_t* b, int64_t* e)
{
    *b = n * t / T;
    *e = n * (t + 1) / T;
}

struct HostBox {
    BoxDev b;                      // descriptor fields the helpers read (no device pointers)
    int64_t n = 0, ncell = 0;
    float* in[6];                  // current particle arrays
    float* out[6];                 // the other buffer
    float* m_in = nullptr;
    float* m_out = nullptr;
    int32_t* id_in = nullptr;
    int32_t* id_out = nullptr;
    std::vector<uint32_t> key;     // collision cell of each particle (this step)
    std::unique_ptr<std::atomic<uint32_t>[]> cnt;   // per cell: count, then the scatter cursor
    std::vector<uint32_t> start;   // per cell: first slot in cell order (ncell + 1)
    std::vector<int64_t> part;     // per thread: particles counted in its cell range
    std::atomic<int64_t> bad{0};   // range violations
};

// One SRD step by thread t of T (all threads call it; barriers inside).
void step_part(HostBox& h, long long k, int t, int T, Barrier& bar)
{
    const BoxDev& b = h.b;
    int64_t pb, pe, cb, ce;
    part_of(h.n, t, T, &pb, &pe);
    part_of(h.ncell, t, T, &cb, &ce);
    const float3 sh = grid_shift(b, k);
    // 1. stream, key, count
    for (int64_t c = cb; c < ce; ++c) h.cnt[c].store(0, std::memory_order_relaxed);
    bar.wait();
    for (int64_t i = pb; i < pe; ++i) {
        const float x = fold(fmaf(h.in[3][i], b.dt, h.in[0][i]), b.len[0]);
        const float y = fold(fmaf(h.in[4][i], b.dt, h.in[1][i]), b.len[1]);
        const float z = fold(fmaf(h.in[5][i], b.dt, h.in[2][i]), b.len[2]);
        h.in[0][i] = x;
        h.in[1][i] = y;
        h.in[2][i] = z;
        const int ix = axis_cell(x, sh.x, b.inv_a, b.L[0]);
        const int iy = axis_cell(y, sh.y, b.inv_a, b.L[1]);
        const int iz = axis_cell(z, sh.z, b.inv_a, b.L[2]);
        const uint32_t c = (uint32_t)ix + (uint32_t)b.L[0] * ((uint32_t)iy + (uint32_t)b.L[1] * (uint32_t)iz);
        h.key[i] = c;
        h.cnt[c].fetch_add(1, std::memory_order_relaxed);
    }
    bar.wait();
    // 2. exclusive scan of the counts: per-thread sums, then local prefixes
    int64_t s = 0;
    for (int64_t c = cb; c < ce; ++c) s += h.cnt[c].load(std::memory_order_relaxed);
    h.part[t] = s;
    bar.wait();
    int64_t run = 0;
    for (int q = 0; q < t; ++q) run += h.part[q];
    for (int64_t c = cb; c < ce; ++c) {
        const uint32_t n = h.cnt[c].load(std::memory_order_relaxed);
        h.start[c] = (uint32_t)run;
        h.cnt[c].store((uint32_t)run, std::memory_order_relaxed);   // scatter cursor
        run += n;
    }
    if (t == T - 1) h.start[h.ncell] = (uint32_t)h.n;
    bar.wait();
    // 3. scatter into cell order (the order inside a cell is free: the sums
    // are exact)
    for (int64_t i = pb; i < pe; ++i) {
        const uint32_t j = h.cnt[h.key[i]].fetch_add(1, std::memory_order_relaxed);
        for (int d = 0; d < 6; ++d) h.out[d][j] = h.in[d][i];
        if (h.m_in) h.m_out[j] = h.m_in[i];
        if (h.id_in) h.id_out[j] = h.id_in[i];
    }
    bar.wait();
    // 4. collide every cell of this thread's range
    int64_t bad = 0;
    for (int64_t c = cb; c < ce; ++c) {
        const uint32_t beg = h.start[c], end = h.start[c + 1];
        if (beg == end) continue;
        if (end - beg >= kMaxCellCount) ++bad;   // the cell's sums may have wrapped
        unsigned long long sx = 0, sy = 0, sz = 0, sw = 0;
        for (uint32_t j = beg; j < end; ++j) {
            const float mj = h.m_out ? h.m_out[j] : 1.0f;
            sx += to_fixed(mj * h.out[3][j]);
            sy += to_fixed(mj * h.out[4][j]);
            sz += to_fixed(mj * h.out[5][j]);
            sw += to_fixed(mj);
        }
        double uc[3];
        fixed_mean3(sx, sy, sz, sw, uc);
        const CellRot cr = cell_rotation(uc[0], uc[1], uc[2], host_cell_axis(b, k, (uint32_t)c), b.ca, b.sa);
        for (uint32_t j = beg; j < end; ++j) {
            const float3 v = apply_rotation(cr, h.out[3][j], h.out[4][j], h.out[5][j]);
            h.out[3][j] = v.x;
            h.out[4][j] = v.y;
            h.out[5][j] = v.z;
            if (!in_range(v)) ++bad;
        }
    }
    if (bad) h.bad.fetch_add(bad, std::memory_order_relaxed);
    bar.wait();
    // the sorted buffer becomes the state
    if (t == 0) {
        for (int d = 0; d < 6; ++d) std::swap(h.in[d], h.out[d]);
        std::swap(h.m_in, h.m_out);
        std::swap(h.id_in, h.id_out);
    }
    bar.wait();
}

}  // namespace
}  // namespace mpcd

using namespace mpcd;

namespace {

int host_step(const mpcd_box_desc* desc, float* xyzv, float* mass, int32_t* pid, int64_t step, int32_t n_steps,
              int32_t threads)
{
    int rc = validate_box_desc(desc);
    if (rc) return rc;
    if (step < 0 || n_steps < 0 || threads < 0) return MPCD_EINVAL;
    // the angular-momentum rule and the VACF record are kept by contexts only
    if (desc->flags & (MPCD_CONSERVE_L | MPCD_TRACK_VACF)) return MPCD_EINVAL;
    const int64_t n = desc->n_particles;
    if (n > 0 && !xyzv) return MPCD_EINVAL;
    if ((desc->flags & MPCD_PARTICLE_MASS) && n > 0 && !mass) return MPCD_EINVAL;
    if (!(desc->flags & MPCD_PARTICLE_MASS) && mass) return MPCD_EINVAL;
    HostBox h;
    BoxDev& b = h.b;
    std::memset(&b, 0, sizeof(b));
    for (int d = 0; d < 3; ++d) {
        b.L[d] = desc->L[d];
        b.len[d] = (float)(desc->L[d] * desc->a);
    }
    b.a = (float)desc->a;
    b.inv_a = (float)(1.0 / desc->a);
    b.dt = (float)desc->dt;
    b.ca = cos(desc->alpha);
    b.sa = sin(desc->alpha);
    b.mass = (float)desc->mass;
    b.key0 = (uint32_t)(desc->seed & 0xffffffffu);
    b.key1 = (uint32_t)(desc->seed >> 32);
    h.n = n;
    h.ncell = (int64_t)desc->L[0] * desc->L[1] * desc->L[2];
    // the state the GPU path accepts (mpcd_set_state, mpcd_set_mass)
    for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) {
            const float x = xyzv[(size_t)d * n + i];
            if (!(x >= 0.0f && x < b.len[d])) return MPCD_EINVAL;
        }
    int64_t out_of_range = 0;   // velocities beyond the exact sums' range: flagged, as on the GPU
    for (int64_t i = 3 * n; i < 6 * n; ++i) {
        if (!std::isfinite(xyzv[i])) return MPCD_EINVAL;
        if (!(fabsf(xyzv[i]) < kVelocityLimit)) ++out_of_range;
    }
    if (mass)
        for (int64_t i = 0; i < n; ++i)
            if (!(mass[i] >= kMassMin && mass[i] <= kMassMax)) return MPCD_EINVAL;
    if (n_steps == 0 || n == 0) return MPCD_OK;

    int T = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    T = (int)std::max<int64_t>(1, std::min<int64_t>(T, std::max<int64_t>(1, h.ncell / 64)));
    std::vector<float> other((size_t)6 * n);
    std::vector<float> m_other(mass ? (size_t)n : 0);
    std::vector<int32_t> id_other(pid ? (size_t)n : 0);
    for (int d = 0; d < 6; ++d) {
        h.in[d] = xyzv + (size_t)d * n;
        h.out[d] = other.data() + (size_t)d * n;
    }
    h.m_in = mass;
    h.m_out = mass ? m_other.data() : nullptr;
    h.id_in = pid;
    h.id_out = pid ? id_other.data() : nullptr;
    h.key.resize((size_t)n);
    h.cnt.reset(new std::atomic<uint32_t>[(size_t)h.ncell]);
    h.start.resize((size_t)h.ncell + 1);
    h.part.assign((size_t)T, 0);
    h.bad.store(out_of_range);

    Barrier bar(T);
    std::atomic<int> go{0};   // the team starts together (1), or not at all (-1)
    auto work = [&](int t) {
        int g;
        while ((g = go.load(std::memory_order_acquire)) == 0) std::this_thread::yield();
        if (g < 0) return;
        for (int32_t q = 0; q < n_steps; ++q) step_part(h, (long long)(step + q), t, T, bar);
    };
    std::vector<std::thread> team;
    team.reserve((size_t)T);
    try {
        for (int t = 1; t < T; ++t) team.emplace_back(work, t);
    } catch (...) {   // a thread could not start: release the others, leave the state untouched
        go.store(-1, std::memory_order_release);
        for (auto& th : team) th.join();
        throw;
    }
    go.store(1, std::memory_order_release);
    work(0);
    for (auto& th : team) th.join();
    // the state ends in the caller's arrays
    if (h.in[0] != xyzv) {
        std::memcpy(xyzv, h.in[0], sizeof(float) * (size_t)6 * n);
        if (mass) std::memcpy(mass, h.m_in, sizeof(float) * (size_t)n);
        if (pid) std::memcpy(pid, h.id_in, sizeof(int32_t) * (size_t)n);
    }
    return h.bad.load() ? MPCD_ESTATE : MPCD_OK;
}

}  // namespace

extern "C" int mpcd_host_step(const mpcd_box_desc* desc, float* xyzv, float* mass, int32_t* pid, int64_t step,
                              int32_t n_steps, int32_t threads)
{
    try {
        return host_step(desc, xyzv, mass, pid, step, n_steps, threads);
    } catch (const std::bad_alloc&) {   // work buffers
        return MPCD_ENOMEM;
    } catch (const std::system_error&) {   // a thread could not start
        return MPCD_EDEVICE;
    }
}
