// Templates of the single-mesh DJ-TLED step kernels for gfx950 (MI355X): the
// persistent multi-step kernel and its several-load-cases twin, the force
// entry point's kernels, the average-nodal-pressure force pass, and their
// launchers for every (model, variant) of one (precision, element type).
// Each djtled_inst_*.hip translation unit instantiates one (precision,
// element type, form) through run_ops, so the variants build in parallel.
#pragma once

#include "djtled_device.h"

namespace dj {

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC>
__global__ void __launch_bounds__(BLOCK) k_forces_elem(DevTopo tp, StepPtrs<T> sp) {
    using C = Chunk<T, NE, MODEL, BLOCK, EPT, MC>;
    extern __shared__ __align__(16) unsigned char smem[];
    PhaseOut po{0.0, 0.0, 0, -1};
    const ChunkDesc ch = tp.chunks[blockIdx.x];
    C::template element_phase<0>(tp, ch, sp, smem, po);
}

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC>
__global__ void __launch_bounds__(BLOCK) k_forces_shared(DevTopo tp, StepPtrs<T> sp) {
    using C = Chunk<T, NE, MODEL, BLOCK, EPT, MC>;
    PhaseOut po{0.0, 0.0, 0, -1};
    const ChunkDesc ch = tp.chunks[blockIdx.x];
    C::template shared_batch<0, 1>(tp, &ch, 1, 0, sp, po);
}

// The persistent multi-step kernel: n_steps x {element phase of every owned
// chunk -> grid barrier -> shared-node phase}, one barrier per step (plus one
// on residual-check steps).  All workgroups take every decision from values
// published before a common barrier, so they leave the loop together.

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC, int WPE>
__global__ void __launch_bounds__(BLOCK, WPE) k_step(DevTopo tp, StepArgs a) {
    using C = Chunk<T, NE, MODEL, BLOCK, EPT, MC>;
    constexpr int KB = 4;  // chunks per shared-phase batch
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sred[2 * (BLOCK / 64)];
    __shared__ int s_flag;
    __shared__ ChunkDesc s_ch[KMAX];
    const int64_t L = tp.n_copies;
    const int64_t NPART = tp.n_part;
    const uint32_t G = gridDim.x;
    const int nmine = int(blockIdx.x) < tp.n_chunks ? (tp.n_chunks - int(blockIdx.x) + int(G) - 1) / int(G) : 0;
    for (int k = threadIdx.x; k < min(nmine, KMAX); k += BLOCK) s_ch[k] = tp.chunks[blockIdx.x + k * G];
    __syncthreads();
    // The workgroup's chunk descriptors: all in LDS when they fit, otherwise
    // in windows of KMAX refilled as the loops below advance (large meshes).
    auto window = [&](int w0) {
        const int wn = min(KMAX, nmine - w0);
        if (nmine > KMAX) {
            __syncthreads();  // no thread still reads the previous window
            for (int k = threadIdx.x; k < wn; k += BLOCK) s_ch[k] = tp.chunks[blockIdx.x + (w0 + k) * G];
            __syncthreads();
        }
        return wn;
    };
    uint32_t epoch = 0;  // the flags are cleared before every launch
    T *const ub0 = static_cast<T *>(a.ubuf[0]), *const ub1 = static_cast<T *>(a.ubuf[1]),
            *const ub2 = static_cast<T *>(a.ubuf[2]);
    auto ub = [&](int i) { return i == 0 ? ub0 : (i == 1 ? ub1 : ub2); };  // no runtime-indexed array
    T *part = static_cast<T *>(a.part);
    const T *ru = static_cast<const T *>(a.ru);
    int cur = a.cur0;
    int done = 0;
    int code = DJ_OK;
    int s = 0;
    for (s = 0; s < a.n_steps; s++) {
        const int nxt = (cur + 1) % 3, prv = (cur + 2) % 3;
        const int64_t n = a.step0 + s;
        const bool check = a.relax && (s % a.check_every) == 0 && ramp_value(a.ramp, double(n) * a.dt, a.t_ramp) >= 1.0;
        StepPtrs<T> sp;
        for (int k = 0; k < 3; k++) {
            sp.uc[k] = ub(cur) + k * L;
            sp.up[k] = ub(prv) + k * L;
            sp.un[k] = ub(nxt) + k * L;

            sp.ru[k] = ru ? ru + k * L : nullptr;
        }
        for (int k = 0; k < 3; k++) sp.pp[k] = part + ((s & 1) * 3 + k) * NPART;
        sp.flags = a.flags;
        sp.acoef = static_cast<const T *>(tp.acoef);
        sp.bprime = T(a.bprime);
        sp.sval = T(ramp_value(a.ramp, double(n + 1) * a.dt, a.t_ramp));
        sp.want_res = check;
        sp.fout = nullptr;
        sp.bpc = nullptr;
        sp.rrate = nullptr;
        sp.n1 = T(n + 1);
        sp.pn = nullptr;
        PhaseOut po{0.0, 0.0, 0, -1};
        if constexpr (C::ANPM) {
            // Average nodal pressure (Sec. 7): a J pass over every chunk, its own
            // grid barrier, the nodal pressures of the shared copies, then the
            // force pass below with each element's pressure the mean of its
            // nodes' pressures.  The J partial sums are single-buffered: they
            // are read before the force barrier and written after it.
            T *jpart = static_cast<T *>(a.anp_jpart);
            const T *cn = static_cast<const T *>(a.anp_c);
            T *pnb = static_cast<T *>(a.anp_p);
            for (int w0 = 0; w0 < nmine; w0 += KMAX) {
                const int wn = window(w0);
                for (int k = 0; k < wn; k++) C::anp_j_phase(tp, s_ch[k], sp, jpart, cn, pnb, smem);
            }
            if (!grid_barrier(a.bar, G, epoch, a.status)) {
                code = DJ_ERR_BARRIER;
                break;
            }
            for (int w0 = 0; w0 < nmine; w0 += KMAX) {
                const int wn = window(w0);
                for (int k = 0; k < wn; k++) C::anp_j_shared(tp, s_ch[k], sp, jpart, cn, pnb);
            }
            __syncthreads();  // pressures written above by one thread are scattered by another
            sp.pn = pnb;
        }
        // The copy data of chunk k + 1 is loaded while chunk k is summed and
        // updated; the element data of chunk k is in flight during its
        // scatter.  (Element data loaded one chunk ahead, or across the step
        // boundary, measured slower: it does not fit the register budget of
        // two waves per SIMD, or it competes with the shared phase's loads.)
        // Variants built for three waves per SIMD keep the plain order.
        for (int w0 = 0; w0 < nmine; w0 += KMAX) {
            const int wn = window(w0);
            if constexpr (WPE >= 3) {
                for (int k = 0; k < wn; k++) C::template element_phase<1>(tp, s_ch[k], sp, smem, po);
            } else {
                typename C::CopyRegs cp;
                C::template load_copies<1>(tp, s_ch[0], sp, cp);
                for (int k = 0; k < wn; k++) {
                    typename C::ElemRegs er;
                    C::load_elems(tp, s_ch[k], er);
                    C::template process<1, true>(tp, s_ch[k], sp, smem, po, er, cp, [&]() {
                        if (k + 1 < wn) C::template load_copies<1>(tp, s_ch[k + 1], sp, cp);
                    });
                }
            }
        }
        // round A of the first batch of shared copies, in flight during the barrier
        const int wn0 = nmine > 0 ? window(0) : 0;
        SharedRegs<T, KB> sr;
        C::template shared_load<1, KB>(tp, s_ch, min(KB, wn0), 0, sp, sr);
        // Errors of step s go to the error word of parity s & 1, which nobody
        // writes again before every workgroup has read it after this barrier.
        int32_t *errw = &a.status[5 + (s & 1)];
        if (po.bad) {
            if (atomicCAS(errw, 0, po.bad) == 0) {  // first reporter names the element
                a.status[2] = po.bad_elem;
                a.status[3] = s;
            }
        }
        if (!grid_barrier(a.bar, G, epoch, a.status)) {
            code = DJ_ERR_BARRIER;
            break;
        }
        if (threadIdx.x == 0) s_flag = ld_dev(errw);
        __syncthreads();
        if (s_flag != 0) {
            code = s_flag;
            break;
        }
        C::template shared_finish<1, KB>(tp, sr, sp, po);
        for (int w0 = 0; w0 < nmine; w0 += KMAX) {
            const int wn = w0 == 0 ? wn0 : window(w0);
            for (int k0 = 0; k0 < wn; k0 += KB)
                C::template shared_batch<1, KB>(tp, s_ch + k0, min(KB, wn - k0), (w0 == 0 && k0 == 0) ? 1 : 0, sp, po);
        }
        if (po.bad) publish_late_error(a.status, s, po.bad, po.bad_elem, s);
        if (check) {
            double x = po.num, y = po.den;
            block_sum2<BLOCK>(x, y, sred);
            double *red = a.red + size_t(s & 1) * 2 * G;
            if (threadIdx.x == 0) {
                st_dev(&red[2 * blockIdx.x], x);
                st_dev(&red[2 * blockIdx.x + 1], y);
            }
            if (!grid_barrier(a.bar, G, epoch, a.status)) {
                code = DJ_ERR_BARRIER;
                break;
            }
            // every workgroup reduces all partials in the same order
            double sx = 0, sy = 0;
            for (uint32_t g = threadIdx.x; g < G; g += BLOCK) {
                sx += ld_dev(&red[2 * g]);
                sy += ld_dev(&red[2 * g + 1]);
            }
            block_sum2<BLOCK>(sx, sy, sred);
            if (threadIdx.x == 0) {
                // no reaction force (e.g. prescribed values not yet applied): undefined, not converged
                const double r = sy > 0.0 ? sqrt(sx) / sqrt(sy) : INFINITY;
                s_flag = (r <= a.tol) ? 1 : 0;
                if (blockIdx.x == 0) *a.res_out = r;
            }
            __syncthreads();
            if (s_flag) {
                code = DJ_CONVERGED;
                break;  // u^n is the converged state; u^{n+1} is discarded
            }
        }
        // shared copies written above by one thread are read by another in the
        // next step's scatter (and in the final write-out)
        __syncthreads();
        cur = nxt;
        done = s + 1;
    }
    __syncthreads();
    if (code == DJ_ERR_BARRIER) return;  // status[4] is set; the caller's state is left untouched
    if (code != DJ_OK && code != DJ_CONVERGED) done = s;  // the failing step is not completed
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.status[0] = code;
        a.status[1] = done;
    }
    // write the final state (canonical copies) to the caller arrays
    const int prv = (cur + 2) % 3;
    T *oc = static_cast<T *>(a.u_out_cur);
    T *op = static_cast<T *>(a.u_out_prev);
    for (int w0 = 0; w0 < nmine; w0 += KMAX) {
        const int wn = window(w0);
        for (int k = 0; k < wn; k++) {
            const ChunkDesc ch = s_ch[k];
            for (int i = threadIdx.x; i < ch.copy_count; i += BLOCK) {
                const int l = ch.copy_begin + i;
                if (!(tp.flags[l] & FLAG_CANON)) continue;
                const int nd = tp.cnode[l];
#pragma unroll
                for (int c3 = 0; c3 < 3; c3++) {
                    oc[3 * nd + c3] = ub(cur)[c3 * L + l];
                    op[3 * nd + c3] = ub(prv)[c3 * L + l];
                }
            }
        }
    }
}

// The same step for a.nrhs load cases per launch (djtled_step_multi): per
// step, the element phase of every case, one grid barrier, the shared phase
// of every case.  A separate kernel: the case loops, even with one case,
// measured 3-13 % slower than k_step.  The element data is reloaded per case:
// holding it in registers across the cases of a chunk overflowed the budget
// of two waves per SIMD, and staging it in LDS by direct loads measured
// 15-25 % slower per case.
template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC, int WPE>
__global__ void __launch_bounds__(BLOCK, WPE) k_step_multi(DevTopo tp, StepArgs a) {
    using C = Chunk<T, NE, MODEL, BLOCK, EPT, MC>;
    constexpr int KB = 4;  // chunks per shared-phase batch
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sred[2 * (BLOCK / 64)];
    __shared__ double s_res[2 * MAX_RHS];  // this workgroup's residual sums per load case (R > 1)
    __shared__ int s_flag;
    __shared__ ChunkDesc s_ch[KMAX];
    const int64_t L = tp.n_copies;
    const int64_t NPART = tp.n_part;
    const uint32_t G = gridDim.x;
    const int R = a.nrhs;
    const int nmine = int(blockIdx.x) < tp.n_chunks ? (tp.n_chunks - int(blockIdx.x) + int(G) - 1) / int(G) : 0;
    for (int k = threadIdx.x; k < nmine; k += BLOCK) s_ch[k] = tp.chunks[blockIdx.x + k * G];
    __syncthreads();
    uint32_t epoch = 0;  // the flags are cleared before every launch
    T *const ub0 = static_cast<T *>(a.ubuf[0]), *const ub1 = static_cast<T *>(a.ubuf[1]),
            *const ub2 = static_cast<T *>(a.ubuf[2]);
    auto ub = [&](int i) { return i == 0 ? ub0 : (i == 1 ? ub1 : ub2); };  // no runtime-indexed array
    T *part = static_cast<T *>(a.part);
    int cur = a.cur0;
    int done = 0;
    int code = DJ_OK;
    int s = 0;
    for (s = 0; s < a.n_steps; s++) {
        const int nxt = (cur + 1) % 3, prv = (cur + 2) % 3;
        const int64_t n = a.step0 + s;
        bool check = a.relax && (s % a.check_every) == 0;
        check = check && ramp_value(a.ramp, double(n) * a.dt, a.t_ramp) >= 1.0;
        const T sval = T(ramp_value(a.ramp, double(n + 1) * a.dt, a.t_ramp));
        // pointers of load case r: its u planes and partials follow those of r - 1
        auto make_sp = [&](int r) {
            StepPtrs<T> sp;
            const int64_t uo = int64_t(r) * 3 * L;
            const T *ru = a.ru ? static_cast<const T *>(a.ru) + uo : nullptr;
            for (int k = 0; k < 3; k++) {
                sp.uc[k] = ub(cur) + uo + k * L;
                sp.up[k] = ub(prv) + uo + k * L;
                sp.un[k] = ub(nxt) + uo + k * L;
                sp.ru[k] = ru ? ru + k * L : nullptr;
            }
            for (int k = 0; k < 3; k++) sp.pp[k] = part + ((int64_t(r) * 2 + (s & 1)) * 3 + k) * NPART;
            sp.flags = a.flags + int64_t(r) * L;
            sp.acoef = static_cast<const T *>(tp.acoef);
            sp.bprime = T(a.bprime);
            sp.sval = sval;
            sp.want_res = check;
            sp.fout = nullptr;
            sp.bpc = nullptr;
            sp.rrate = nullptr;
            sp.n1 = T(n + 1);
            sp.pn = nullptr;
            return sp;
        };
        PhaseOut po{0.0, 0.0, 0, -1};
        int bad_rhs = -1;
        if (check && R > 1 && threadIdx.x < 2 * R) s_res[threadIdx.x] = 0.0;
        // with several load cases, each case's residual sums are reduced after
        // its part of a chunk (one case: once per step, below)
        auto after_case = [&](int r) {
            if (po.bad && bad_rhs < 0) bad_rhs = r;
            if (check && R > 1) {
                double x = po.num, y = po.den;
                block_sum2<BLOCK>(x, y, sred);
                if (threadIdx.x == 0) {
                    s_res[2 * r] += x;
                    s_res[2 * r + 1] += y;
                }
                po.num = po.den = 0.0;
            }
        };
        // Element phase: each chunk's element data (planes and slot positions)
        // is loaded once and kept in registers while every case runs the
        // chunk (scatter, forces, sums, update of its own copies), so the
        // element stream is shared by the cases.  The copy data of the next
        // (chunk, case) is loaded while the current one is summed and updated.
        // Variants built for three waves per SIMD keep the plain order.
        if constexpr (WPE >= 3) {
            for (int r = 0; r < R; r++) {
                const StepPtrs<T> sp = make_sp(r);
                for (int k = 0; k < nmine; k++) C::template element_phase<1>(tp, s_ch[k], sp, smem, po);
                after_case(r);
            }
        } else {
            typename C::CopyRegs cp;
            if (nmine > 0) C::template load_copies<1>(tp, s_ch[0], make_sp(0), cp);
            for (int k = 0; k < nmine; k++) {
                typename C::ElemRegs er;
                C::load_elems(tp, s_ch[k], er);
                for (int r = 0; r < R; r++) {
                    C::template process<1, true>(tp, s_ch[k], make_sp(r), smem, po, er, cp, [&]() {
                        if (r + 1 < R) C::template load_copies<1>(tp, s_ch[k], make_sp(r + 1), cp);
                        else if (k + 1 < nmine) C::template load_copies<1>(tp, s_ch[k + 1], make_sp(0), cp);
                    });
                    after_case(r);
                }
            }
        }
        // round A of the first batch of shared copies (case 0), in flight during the barrier
        SharedRegs<T, KB> sr;
        C::template shared_load<1, KB>(tp, s_ch, min(KB, nmine), 0, make_sp(0), sr);
        // Errors of step s go to the error word of parity s & 1, which nobody
        // writes again before every workgroup has read it after this barrier.
        int32_t *errw = &a.status[5 + (s & 1)];
        if (po.bad) {
            if (atomicCAS(errw, 0, po.bad) == 0) {  // first reporter names the element and the case
                a.status[2] = po.bad_elem;
                a.status[3] = s;
                a.status[7] = max(bad_rhs, 0);
            }
        }
        if (!grid_barrier(a.bar, G, epoch, a.status)) {
            code = DJ_ERR_BARRIER;
            break;
        }
        if (threadIdx.x == 0) s_flag = ld_dev(errw);
        __syncthreads();
        if (s_flag != 0) {
            code = s_flag;
            break;
        }
        {
            const StepPtrs<T> sp = make_sp(0);
            C::template shared_finish<1, KB>(tp, sr, sp, po);
            for (int k0 = 0; k0 < nmine; k0 += KB)
                C::template shared_batch<1, KB>(tp, s_ch + k0, min(KB, nmine - k0), k0 == 0 ? 1 : 0, sp, po);
            after_case(0);
        }
        for (int r = 1; r < R; r++) {  // the other cases: round A after the barrier
            const StepPtrs<T> sp = make_sp(r);
            for (int k0 = 0; k0 < nmine; k0 += KB)
                C::template shared_batch<1, KB>(tp, s_ch + k0, min(KB, nmine - k0), 0, sp, po);
            after_case(r);
        }
        if (po.bad) publish_late_error(a.status, s, po.bad, po.bad_elem, s, max(bad_rhs, 0));
        if (check) {
            // per workgroup and case: (|F - R|^2 over free, |F|^2 over constrained) components
            double *red = a.red + size_t(s & 1) * 2 * G * R;
            if (R == 1) {
                double x = po.num, y = po.den;
                block_sum2<BLOCK>(x, y, sred);
                if (threadIdx.x == 0) {
                    st_dev(&red[2 * blockIdx.x], x);
                    st_dev(&red[2 * blockIdx.x + 1], y);
                }
            } else {
                __syncthreads();
                if (threadIdx.x < 2 * R) st_dev(&red[2 * size_t(blockIdx.x) * R + threadIdx.x], s_res[threadIdx.x]);
            }
            if (!grid_barrier(a.bar, G, epoch, a.status)) {
                code = DJ_ERR_BARRIER;
                break;
            }
            // every workgroup reduces all partials in the same order; the run
            // stops when every case has converged
            int conv = 1;
            for (int r = 0; r < R; r++) {
                double sx = 0, sy = 0;
                for (uint32_t g = threadIdx.x; g < G; g += BLOCK) {
                    sx += ld_dev(&red[2 * (size_t(g) * R + r)]);
                    sy += ld_dev(&red[2 * (size_t(g) * R + r) + 1]);
                }
                block_sum2<BLOCK>(sx, sy, sred);
                if (threadIdx.x == 0) {
                    const double res = sy > 0.0 ? sqrt(sx) / sqrt(sy) : INFINITY;
                    conv &= (res <= a.tol) ? 1 : 0;
                    if (blockIdx.x == 0) a.res_out[r] = res;
                }
            }
            if (threadIdx.x == 0) s_flag = conv;
            __syncthreads();
            if (s_flag) {
                code = DJ_CONVERGED;
                break;  // u^n is the converged state; u^{n+1} is discarded
            }
        }
        // shared copies written above by one thread are read by another in the
        // next step's scatter (and in the final write-out)
        __syncthreads();
        cur = nxt;
        done = s + 1;
    }
    __syncthreads();
    if (code == DJ_ERR_BARRIER) return;  // status[4] is set; the caller's state is left untouched
    if (code != DJ_OK && code != DJ_CONVERGED) done = s;  // the failing step is not completed
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.status[0] = code;
        a.status[1] = done;
    }
    // write the final state (canonical copies) of every case to the caller arrays
    const int prv = (cur + 2) % 3;
    for (int r = 0; r < R; r++) {
        T *oc = static_cast<T *>(a.u_out_cur) + int64_t(r) * a.out_stride;
        T *op = static_cast<T *>(a.u_out_prev) + int64_t(r) * a.out_stride;
        const int64_t uo = int64_t(r) * 3 * L;
        for (int k = 0; k < nmine; k++) {
            const ChunkDesc ch = s_ch[k];
            for (int i = threadIdx.x; i < ch.copy_count; i += BLOCK) {
                const int l = ch.copy_begin + i;
                if (!(tp.flags[l] & FLAG_CANON)) continue;
                const int nd = tp.cnode[l];
#pragma unroll
                for (int c3 = 0; c3 < 3; c3++) {
                    oc[3 * nd + c3] = ub(cur)[uo + c3 * L + l];
                    op[3 * nd + c3] = ub(prv)[uo + c3 * L + l];
                }
            }
        }
    }
}

// clears the barrier flags and the status words before a persistent launch
// (a kernel rather than a memset, so that the sequence can be graph-captured)
static __global__ void k_reset_sync(uint32_t *sync, int n_sync, int32_t *status) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_sync; i += gridDim.x * blockDim.x) sync[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x < 8) status[threadIdx.x] = threadIdx.x == 2 ? -1 : 0;
}

// ---------------------------------------------------------------------------
// Dispatch over (precision, element type, model, variant)
// ---------------------------------------------------------------------------

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC, int WPE>
struct Inst {
    using C = Chunk<T, NE, MODEL, BLOCK, EPT, MC>;
    // several load cases per launch: FP32, Jacobian form, two-wave variants
    static constexpr bool has_multi() {
        return sizeof(T) == 4 && (MODEL & (DJ_FORM_TLED | DJ_FORM_ANP)) == 0 && WPE < 3;
    }
    // dynamic LDS of the step kernel (a fourth slot plane for the average nodal pressure)
    static constexpr size_t STEP_LDS = C::ANPM ? C::LDS_ANP : C::LDS;
    static hipError_t occ(int *bpc, size_t *lds) {
        *lds = STEP_LDS;
        const void *kern = reinterpret_cast<const void *>(&k_step<T, NE, MODEL, BLOCK, EPT, MC, WPE>);
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(STEP_LDS));
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_step<T, NE, MODEL, BLOCK, EPT, MC, WPE>, BLOCK,
                                                            STEP_LDS);
    }
    // workgroups per CU of the several-cases kernel; 0: not built
    static hipError_t occ_multi(int *bpc) {
        *bpc = 0;
        if constexpr (has_multi()) {
            const void *kern = reinterpret_cast<const void *>(&k_step_multi<T, NE, MODEL, BLOCK, EPT, MC, WPE>);
            hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(C::LDS));
            if (e != hipSuccess) return e;
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_step_multi<T, NE, MODEL, BLOCK, EPT, MC, WPE>,
                                                                BLOCK, C::LDS);
        }
        return hipSuccess;
    }
    // ubuf0: 3 x n_copies u planes, part: 3 x max(n_part, 1) partial sums
    static hipError_t forces(Ctx &c, const void *u, void *f, void *ubuf0, void *part_buf, hipStream_t s) {
        const int L = c.topo.n_copies, B = 256;
        T *u0 = static_cast<T *>(ubuf0);
        hipLaunchKernelGGL(k_scatter_in<T>, dim3((L + B - 1) / B), dim3(B), 0, s, c.topo.cnode, L,
                           static_cast<const T *>(u), static_cast<const T *>(nullptr), u0, static_cast<T *>(nullptr));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        StepPtrs<T> sp{};
        T *part = static_cast<T *>(part_buf);
        for (int k = 0; k < 3; k++) {
            sp.uc[k] = u0 + int64_t(k) * L;
            sp.up[k] = nullptr;
            sp.un[k] = nullptr;
            sp.ru[k] = nullptr;
        }
        for (int k = 0; k < 3; k++) sp.pp[k] = part + int64_t(k) * std::max(c.topo.n_part, 1);
        sp.flags = c.topo.flags;
        sp.acoef = static_cast<const T *>(c.d_acoef);
        sp.bprime = T(0);
        sp.sval = T(0);
        sp.want_res = false;
        sp.fout = static_cast<T *>(f);
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_forces_elem<T, NE, MODEL, BLOCK, EPT, MC>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(C::LDS));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_forces_elem<T, NE, MODEL, BLOCK, EPT, MC>), dim3(c.topo.n_chunks), dim3(BLOCK), C::LDS,
                           s, c.topo, sp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_forces_shared<T, NE, MODEL, BLOCK, EPT, MC>), dim3(c.topo.n_chunks), dim3(BLOCK), 0, s,
                           c.topo, sp);
        return hipGetLastError();
    }
    // u_cur_in / u_prev_in: a.nrhs x n_nodes x 3 each
    static hipError_t step(Ctx &c, const StepArgs &a, const void *u_cur_in, const void *u_prev_in, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
        const int L = c.topo.n_copies, B = 256;
        const int n_sync = (c.grid + N_RELEASE) * FLAG_STRIDE;
        hipLaunchKernelGGL(k_reset_sync, dim3((n_sync + 255) / 256), dim3(256), 0, s, c.d_bar, n_sync, c.d_status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        for (int r = 0; r < a.nrhs; r++) {
            T *dcur = static_cast<T *>(a.ubuf[a.cur0]) + int64_t(r) * 3 * L;
            T *dprev = static_cast<T *>(a.ubuf[(a.cur0 + 2) % 3]) + int64_t(r) * 3 * L;
            hipLaunchKernelGGL(k_scatter_in<T>, dim3((L + B - 1) / B), dim3(B), 0, s, c.topo.cnode, L,
                               static_cast<const T *>(u_cur_in) + r * a.out_stride,
                               static_cast<const T *>(u_prev_in) + r * a.out_stride, dcur, dprev);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        DevTopo tp = c.topo;
        StepArgs aa = a;
        void *args[] = {&tp, &aa};
        const void *kern = reinterpret_cast<const void *>(&k_step<T, NE, MODEL, BLOCK, EPT, MC, WPE>);
        if (a.nrhs > 1) {
            if constexpr (has_multi()) kern = reinterpret_cast<const void *>(&k_step_multi<T, NE, MODEL, BLOCK, EPT, MC, WPE>);
            else return hipErrorInvalidValue;
        }
        const size_t lds = a.nrhs > 1 ? C::LDS : STEP_LDS;
        e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
        e = hipLaunchCooperativeKernel(kern, dim3(c.grid), dim3(BLOCK), args, lds, s);
        if (e != hipSuccess) return e;
        if (ev1) e = hipEventRecord(ev1, s);
        return e;
    }
};

template <typename T, int NE, int MODEL, int V>
using InstV = Inst<T, NE, MODEL, var_table<T, NE>()[V].block, var_table<T, NE>()[V].ept, var_table<T, NE>()[V].mcopy,
                  var_table<T, NE>()[V].wpe>;

// The three-waves-per-SIMD variants (4, 5) are built for the neo-Hookean and
// transversely isotropic models only; the others have too little register room.
template <typename T, int NE, int MODEL, typename F>
static hipError_t with_variant(int v, F &&f) {
    switch (v) {
        case 0: return f(InstV<T, NE, MODEL, 0>());
        case 1: return f(InstV<T, NE, MODEL, 1>());
        case 2: return f(InstV<T, NE, MODEL, 2>());
        case 3: return f(InstV<T, NE, MODEL, 3>());
        default: break;
    }
    if constexpr (MODEL == DJ_NH || MODEL == DJ_TI) {
        if (v == 4) return f(InstV<T, NE, MODEL, 4>());
        if (v == 5) return f(InstV<T, NE, MODEL, 5>());
    }
    return hipErrorInvalidValue;
}

template <typename T, int NE, int FORM = 0, typename F>
static hipError_t with_model(int model, int v, F &&f) {
    switch (model) {
        case DJ_NH: return with_variant<T, NE, DJ_NH | FORM>(v, f);
        case DJ_TI: return with_variant<T, NE, DJ_TI | FORM>(v, f);
        case DJ_OT: return with_variant<T, NE, DJ_OT | FORM>(v, f);
        case DJ_MR: return with_variant<T, NE, DJ_MR | FORM>(v, f);
        default: return hipErrorInvalidValue;
    }
}

// ---- average nodal pressure: element J (FP64), nodal pressures, element planes
template <typename T, int NE>
__global__ void k_anp_je(const int32_t *__restrict__ enode, const int32_t *__restrict__ nperm, int E,
                         const T *__restrict__ u, const double *__restrict__ jinv64, double *__restrict__ Je) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double du[NE][3];
    int n0 = nperm[enode[int64_t(NE) * e]];
    for (int a = 0; a < NE; a++) {
        const int n = nperm[enode[int64_t(NE) * e + a]];
        for (int k = 0; k < 3; k++) du[a][k] = double(u[3 * int64_t(n) + k]) - double(u[3 * int64_t(n0) + k]);
    }
    double dJ[3][3];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) {
            double s = 0.0;
            if (NE == 4) {
                s = du[i + 1][k];
            } else {
                for (int a = 1; a < 8; a++) s += h8s(a, i) * du[a][k];
                s *= 0.125;
            }
            dJ[i][k] = s;
        }
    const double *Ji = jinv64 + 9 * int64_t(e);
    double A[3][3];  // I + D, D = 0J^-1 dJ
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++)
            A[i][k] = (i == k ? 1.0 : 0.0) + Ji[3 * i] * dJ[0][k] + Ji[3 * i + 1] * dJ[1][k] + Ji[3 * i + 2] * dJ[2][k];
    Je[e] = det3d(A);  // Eq. 12
}

// per internal node: V_n, J_n, kappa_n over its elements (ascending), pressure kappa_n (J_n - 1)
template <int NE>
__global__ void k_anp_node(const int32_t *__restrict__ off, const int32_t *__restrict__ lst, int N,
                           const double *__restrict__ V64, const double *__restrict__ Je,
                           const double *__restrict__ kappa, double *__restrict__ Pn) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double v = 0.0, vj = 0.0, vk = 0.0;
    for (int j = off[n]; j < off[n + 1]; j++) {
        const int e = lst[j];
        const double w = V64[e] / NE;
        v += w;
        vj += w * Je[e];
        vk += w * kappa[e];
    }
    Pn[n] = v > 0.0 ? (vk / v) * (vj / v - 1.0) : 0.0;
}

// the kappa 0V plane of a copy of the element planes <- mean nodal pressure x 0V
template <typename T, int NE>
__global__ void k_anp_plane(const int32_t *__restrict__ enode, int E, const double *__restrict__ Pn,
                            const double *__restrict__ V64, T *__restrict__ plane) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int a = 0; a < NE; a++) s += Pn[enode[int64_t(NE) * e + a]];
    plane[e] = T(s / NE * V64[e]);
}

template <typename T, int NE>
static hipError_t forces_anp_t(Ctx &c, const void *u, void *f, hipStream_t s) {
    const int B = 256, E = c.n_elems, N = c.n_nodes;
    hipLaunchKernelGGL((k_anp_je<T, NE>), dim3((E + B - 1) / B), dim3(B), 0, s, c.d_enode, c.d_node_perm, E,
                       static_cast<const T *>(u), c.d_jinv64, c.d_anp_je);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_anp_node<NE>, dim3((N + B - 1) / B), dim3(B), 0, s, c.d_ne_off, c.d_ne_list, N, c.d_V64,
                       c.d_anp_je, c.d_kappa64, c.d_anp_pn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int NP = n_planes(NE, c.model);
    const size_t bytes = size_t(NP) * c.topo.estride * sizeof(T);
    if ((e = hipMemcpyAsync(c.d_anp_planes, c.d_elem, bytes, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    T *kplane = static_cast<T *>(c.d_anp_planes) + int64_t(Planes<NE, DJ_NH>::KAV) * c.topo.estride;
    hipLaunchKernelGGL((k_anp_plane<T, NE>), dim3((E + B - 1) / B), dim3(B), 0, s, c.d_enode, E, c.d_anp_pn,
                       c.d_V64, kplane);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the standard force pass over the modified planes
    const void *saved = c.topo.elem;
    c.topo.elem = c.d_anp_planes;
    auto run = [&](auto inst) { return decltype(inst)::forces(c, u, f, c.d_ubuf[0], c.d_part, s); };
    e = c.model == DJ_NH ? with_variant<T, NE, DJ_NH | DJ_FORM_ANP>(c.variant, run)
                         : with_variant<T, NE, DJ_TI | DJ_FORM_ANP>(c.variant, run);
    c.topo.elem = saved;
    return e;
}

// One operation of the single-mesh launchers, for one (precision, element
// type, form); dispatched at run time over (model, variant).
template <typename T, int NE, int FORM>
hipError_t run_ops(const OpArgs &o) {
    if (o.op == Op::FORCES_ANP) {
        if constexpr (FORM == 0) return forces_anp_t<T, NE>(*o.c, o.u, o.f, o.s);
        return hipErrorInvalidValue;
    }
    auto run = [&](auto inst) -> hipError_t {
        using I = decltype(inst);
        switch (o.op) {
            case Op::OCC: return I::occ(o.bpc, o.lds);
            case Op::OCC_MULTI: return I::occ_multi(o.bpc);
            case Op::FORCES:
                return o.ubuf0 ? I::forces(*o.c, o.u, o.f, o.ubuf0, o.part, o.s)
                               : I::forces(*o.c, o.u, o.f, o.c->d_ubuf[0], o.c->d_part, o.s);
            case Op::STEP: return I::step(*o.c, *o.a, o.u_cur_in, o.u_prev_in, o.s, o.ev0, o.ev1);
            default: return hipErrorInvalidValue;
        }
    };
    if constexpr (FORM == 0) {
        // the average-nodal-pressure step (neo-Hookean and transversely isotropic)
        if (o.anp) {
            if (o.op == Op::FORCES || o.op == Op::OCC_MULTI) return hipErrorInvalidValue;
            if (o.model == DJ_NH) return with_variant<T, NE, DJ_NH | DJ_FORM_ANP>(o.variant, run);
            if (o.model == DJ_TI) return with_variant<T, NE, DJ_TI | DJ_FORM_ANP>(o.variant, run);
            return hipErrorInvalidValue;
        }
    }
    return with_model<T, NE, FORM>(o.model, o.variant, run);
}

}  // namespace dj
