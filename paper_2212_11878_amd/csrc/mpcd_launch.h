// mpcd_launch.h -- host-side launchers of the SRD kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpcd.h"
#include "mpcd_dev.h"

namespace mpcd {

// Device tables describing the live boxes; every kernel reads its box's
// descriptor and step counter from here, so a captured graph stays valid
// until the tables are rebuilt.
struct Tables {
    BoxDev* boxes = nullptr;     // indexed by slot
    BoxState* state = nullptr;   // indexed by slot
    Tile* ptiles = nullptr;      // slot tiles of all live boxes
    Tile* ctiles = nullptr;      // cell tiles of all live boxes
    Tile* btiles = nullptr;      // brick tiles (begin = brick index) of brick boxes
    int32_t* active = nullptr;   // live slots
    long long* dacc = nullptr;        // per slot: kAccLanes x (VACF high, VACF low, violations)
    uint32_t* tilesum = nullptr; // per cell tile
    int nptiles = 0, nctiles = 0, nbtiles = 0, nactive = 0;
    int32_t brick_box = -1;        // the slot of the only brick box (its bricks are the brick tiles in
                                   // order), or -1
    int max_bvol = 0;              // largest brick of the live boxes (cells)
    int brick_shape = 0;           // launch shape of the brick step (brick_shape_for)
    bool brick_mass = false;       // some brick box carries per-particle masses
    bool brick_am = false;         // some brick box uses the angular-momentum rule
    bool brick_wide = false;       // some brick box has buffers of 2^30 slots or more
    bool brick_ids = false;        // some brick box keeps particle ids
    size_t brick_lds = 0;          // LDS bytes of the largest brick record
    int* host_flag = nullptr;      // host-visible: a brick box asks for re-bucketing
};

void launch_brick_step(const Tables& T, hipStream_t s);
int brick_shape_for(int64_t bucket);   // launch shape whose workgroup holds `bucket` particles
int brick_shape_threads(int shape);
int brick_shape_slots(int shape);
void launch_mark_holes(const Tile* tiles, int ntiles, const Tables& T, int all, hipStream_t s);
void launch_rebucket_clear(const Tables& T, hipStream_t s);
void launch_box_finish(const Tables& T, hipStream_t s);
void launch_zero_counts(const Tables& T, hipStream_t s);
void launch_count(const Tables& T, hipStream_t s);
void launch_scan(const Tables& T, hipStream_t s);
void launch_scatter(const Tables& T, hipStream_t s);
void launch_flip(const Tables& T, hipStream_t s);
void launch_cell_rotate(const Tables& T, hipStream_t s);

// per-box launches over ntile = ceil(nslot / kPartTile) particle tiles of
// box `box`; `part` receives ntile x kNumDiag exact partials
void launch_init_maxwell(const Tables& T, int32_t box, int ntile, float vscale, long long* part, hipStream_t s);
void launch_init_adjust(const Tables& T, int32_t box, int ntile, long long* part, hipStream_t s);
void launch_snapshot(const Tables& T, int32_t box, int ntile, int set_v0, long long* part, hipStream_t s);
// modes of launch_box_stats
enum { kStatsCentre = 0, kStatsScale = 1, kStatsSnapshot = 2, kStatsOrigin = 4 };
void launch_box_stats(const Tables& T, int32_t box, int ntile, long long* part, int mode, double kT,
                      double mass, hipStream_t s);   // consumes the partials
void launch_mark_holes_box(const Tables& T, int32_t box, int ntile, hipStream_t s);
void launch_fill_iota(int32_t* p, int64_t n, hipStream_t s);
void launch_fill_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
void launch_hbm_copy(const void* src, void* dst, int64_t n16, int blocks, hipStream_t s);

// mpcd_admit's check of a box descriptor (MPCD_OK or MPCD_EINVAL)
int validate_box_desc(const mpcd_box_desc* d);
// exact momentum and energy of caller arrays: ceil(n / kPartTile) x kNumDiag
// partials in `partials` (scratch), the five results in out (device)
void launch_moments(const float* vx, const float* vy, const float* vz, const float* m, int64_t n,
                    long long* partials, double* out, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
void launch_permute_f32(float* dst, const float* src, const int32_t* pid, int64_t nslot, int64_t n, int scatter,
                        hipStream_t s);

}  // namespace mpcd
