// Internal declarations of batches (several independent instances of up to
// four element kinds advanced by one persistent kernel).  Not public ABI.
#pragma once

#include "djtled_internal.h"

namespace dj {

constexpr int KMAXB = 128;  // work items (chunks) per workgroup: the kernel's LDS list

// Device view of one element kind of a batch (a multi-instance context plus
// the load set of its instances).
struct BatchKind {
    DevTopo tp;                     // n_chunks == 0: kind absent
    const uint32_t *flags = nullptr;  // topology flags | BC mask | FLAG_RU
    const void *ru = nullptr;       // 3 planes over copies (targets), or null
    const void *rate = nullptr;     // per copy signed ramp rate, or null
    void *ubuf[3] = {nullptr, nullptr, nullptr};
    void *part = nullptr;
    const void *ab = nullptr;       // per copy (A, B') side by side
    const void *rq = nullptr;       // per copy (target x, y, z, ramp rate), or null (no loads)
};

struct BatchDev {
    BatchKind k[4];
    const int32_t *work = nullptr;  // kind << 28 | chunk; item j belongs to workgroup j % grid
    int32_t n_items = 0;
    int32_t n_steps = 0;
    int32_t first_launch = 0;       // records start time stamps
    int64_t *clock = nullptr;       // [0] step index n of u^n, [1] buffer holding u^n
    uint32_t *bar = nullptr;        // (grid + 16) x 32 flags
    int32_t *status = nullptr;      // as StepArgs::status; [2] = kind << 28 | element
    uint64_t *tstamp = nullptr;     // per workgroup: start (first launch), end (every launch)
};

bool batch_variant_ok(int prec, int v);
// ab[2l..2l+1] = (A_l, B'_l); with ru: rq[4l..4l+3] = (ru_x, ru_y, ru_z, rate_l or 0)
hipError_t launch_pack_copy_pairs(int prec, int n_copies, const void *acoef, const void *bpc, const void *ru,
                                  const void *rate, void *ab, void *rq, hipStream_t s);
int batch_geometry(int v);  // the step-kernel variant whose chunk geometry batch variant v uses
#ifdef DJ_INSTR
hipError_t instr_set(uint64_t *p);  // instrumented build: the sub-phase counter array
#endif
hipError_t batch_occupancy(int prec, int v, int *blocks_per_cu, size_t *lds, int *block);
hipError_t launch_batch_step(const BatchDev &bd, int prec, int v, int grid, hipStream_t s);
hipError_t launch_batch_reset(uint32_t *bar, int n_sync, int32_t *status, bool clear_status, hipStream_t s);
hipError_t launch_gather_canon(const BatchKind &kd, int prec, int cur, void *u_cur, void *u_prev, hipStream_t s);
hipError_t launch_scatter_state(const BatchKind &kd, int prec, int cur, const void *u_cur, const void *u_prev,
                                hipStream_t s);

}  // namespace dj
