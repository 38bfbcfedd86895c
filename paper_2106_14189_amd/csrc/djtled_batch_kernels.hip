// Batched DJ-TLED: many independent meshes (instances) of up to four element
// kinds -- (T4 | H8) x (neo-Hookean | transversely isotropic) -- advanced
// together by ONE persistent kernel with one grid barrier per step.
//
// Each kind is a multi-instance context (its instances' elements and node
// copies side by side, every instance with its own time step, damping and
// ramp through per-copy coefficients).  The batch's work list holds every
// chunk of every kind, sorted by kind and dealt round-robin to the resident
// workgroups, so each workgroup sees a similar mix and its chunks of one kind
// are consecutive.  A workgroup runs the element phase of each of its chunks
// with the element code of the chunk's kind, then after the barrier the
// shared-node phase in batches of chunks of one kind.
//
// The step index and the current state buffer live in device memory and are
// advanced by the kernel, so a captured graph of launches can be replayed.
#include "djtled_device.h"
#include "djtled_batch.h"

namespace dj {

namespace {

// Batch variant V: 0..3 use the step-kernel tables' variants 0..3 for every
// kind; V + 4 is the same with the element data staged in LDS by prefetch.
// 8 trades registers for occupancy: the chunk geometry of variant 2 (512
// threads) compiled for 4 waves per SIMD, i.e. two workgroups per compute
// unit (its registers spill), with the element phase in plain order.
template <typename T, int V>
struct Kinds {
    static constexpr int VB = V < 8 ? (V & 3) : 2;
    static constexpr bool PF = V >= 4 && V < 8;
    static constexpr int WPE = V < 8 ? 1 : 4;                 // minimum waves per SIMD
    static constexpr bool PIPE = sizeof(T) == 4 && V < 8;     // software-pipelined element phase
    static constexpr Variant v4 = var_table<T, 4>()[VB];
    static constexpr Variant v8 = var_table<T, 8>()[VB];
    static_assert(v4.block == v8.block, "one block size for all element kinds");
    static constexpr int BLOCK = v4.block;
    template <int K>
    using C = Chunk<T, (K >= 2 ? 8 : 4), (K & 1) ? DJ_TI : DJ_NH, BLOCK, (K >= 2 ? v8.ept : v4.ept),
                    (K >= 2 ? v8.mcopy : v4.mcopy), true, PF>;
    static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
    static constexpr size_t LDS = mx(mx(C<0>::LDS, C<1>::LDS), mx(C<2>::LDS, C<3>::LDS));
};

template <typename F>
__device__ __forceinline__ void on_kind(int kind, F &&f) {
    switch (kind) {
        case 0: f(std::integral_constant<int, 0>()); break;
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        default: f(std::integral_constant<int, 3>()); break;
    }
}

template <typename T>
__device__ __forceinline__ StepPtrs<T> kind_ptrs(const BatchKind &kd, int cur, int prv, int nxt, int s, int64_t n) {
    StepPtrs<T> sp;
    const int64_t L = kd.tp.n_copies;
    const T *u0 = static_cast<const T *>(kd.ubuf[0]), *u1 = static_cast<const T *>(kd.ubuf[1]),
            *u2 = static_cast<const T *>(kd.ubuf[2]);
    const T *uc = cur == 0 ? u0 : (cur == 1 ? u1 : u2);
    const T *up = prv == 0 ? u0 : (prv == 1 ? u1 : u2);
    T *un = const_cast<T *>(nxt == 0 ? u0 : (nxt == 1 ? u1 : u2));
    // copy-major state: component k of copy l at 3 l + k (ld_u3 / st_u3 read p[0])
#pragma unroll
    for (int k = 0; k < 3; k++) {
        sp.uc[k] = uc + k;
        sp.up[k] = up + k;
        sp.un[k] = un + k;
        sp.ru[k] = static_cast<const T *>(kd.rq);  // (x, y, z, rate) per copy (Chunk::ld_rq)
    }
    // partial entries entry-major per parity (put_partial3 / get_partial3 read pp[0])
    for (int k = 0; k < 3; k++) sp.pp[k] = static_cast<T *>(kd.part) + (s & 1) * 3 * int64_t(kd.tp.n_part) + k;
    sp.flags = kd.flags;
    sp.acoef = static_cast<const T *>(kd.ab);  // (A, B') per copy (Chunk::ld_ab)
    sp.bprime = T(0);
    sp.sval = T(0);
    sp.want_res = false;
    sp.fout = nullptr;
    sp.bpc = nullptr;
    sp.rrate = nullptr;
    sp.n1 = T(n + 1);
    sp.pn = nullptr;
    return sp;
}

template <typename T, int V>
__global__ void __launch_bounds__((Kinds<T, V>::BLOCK), (Kinds<T, V>::WPE)) k_batch_step(BatchDev bd) {
    using K = Kinds<T, V>;
    constexpr int BLOCK = K::BLOCK;
    constexpr int KB = 4;  // chunks per shared-phase batch
    using CS = typename K::template C<0>;  // the shared-node phase does not depend on the kind
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int SS = 2;  // shared copies per thread per round (single-window FP32 path)
    __shared__ ChunkDesc s_ch[KMAXB];
    __shared__ int s_kind[KMAXB];
    __shared__ int s_pre[KMAXB + 1];  // shared copies of the workgroup's chunks before chunk k
    __shared__ int s_flag;
    const uint32_t G = gridDim.x;
    const int nmine = int(blockIdx.x) < bd.n_items ? (bd.n_items - int(blockIdx.x) + int(G) - 1) / int(G) : 0;
    // the workgroup's work items (kind, chunk descriptor) from w0 on: all in
    // LDS when they fit, otherwise in windows of KMAXB refilled as the loops
    // advance (batches too large for one list; not the prefetch variants)
    auto fill = [&](int w0, int wn) {
        for (int k = threadIdx.x; k < wn; k += BLOCK) {
            const int w = bd.work[blockIdx.x + (w0 + k) * G];
            const int kind = w >> 28, idx = w & 0x0fffffff;
            const ChunkDesc *cp = kind == 0 ? bd.k[0].tp.chunks
                                : kind == 1 ? bd.k[1].tp.chunks
                                : kind == 2 ? bd.k[2].tp.chunks
                                            : bd.k[3].tp.chunks;
            s_ch[k] = cp[idx];
            s_kind[k] = kind;
        }
    };
    auto window = [&](int w0) {
        const int wn = min(KMAXB, nmine - w0);
        if (nmine > KMAXB) {
            __syncthreads();  // no thread still reads the previous window
            fill(w0, wn);
            __syncthreads();
        }
        return wn;
    };
    fill(0, min(nmine, KMAXB));
    __syncthreads();
    if (threadIdx.x == 0) {
        s_flag = bd.status[0];
        int acc = 0;
        for (int k = 0; k < min(nmine, KMAXB); k++) {
            s_pre[k] = acc;
            acc += s_ch[k].copy_count - s_ch[k].n_interior;
        }
        s_pre[min(nmine, KMAXB)] = acc;
    }
    __syncthreads();
    if (s_flag != 0) return;  // an earlier launch of this run stopped on an error
    if (threadIdx.x == 0 && bd.first_launch) bd.tstamp[2 * blockIdx.x] = uint64_t(wall_clock64());
    // staged element data of chunk k + 1 is requested while chunk k is summed
    auto prefetch = [&](int k) {
        if constexpr (K::PF) {
            const int kind = __builtin_amdgcn_readfirstlane(s_kind[k]);
            on_kind(kind, [&](auto kc) {
                constexpr int KC = decltype(kc)::value;
                K::template C<KC>::prefetch(bd.k[KC].tp, s_ch[k], smem);
            });
        }
    };
    if (nmine > 0) prefetch(0);
    uint32_t epoch = 0;  // flags are cleared before every launch
    const int64_t step0 = bd.clock[0];
    int cur = int(bd.clock[1]);
    int code = DJ_OK;
    int s = 0;
    for (s = 0; s < bd.n_steps; s++) {
        const int nxt = (cur + 1) % 3, prv = (cur + 2) % 3;
        const int64_t n = step0 + s;
        INSTR_T(t0);
        PhaseOut po{0.0, 0.0, 0, -1};
        int bad_kind = -1;
        // FP32: runs of consecutive chunks of one kind, software-pipelined: the
        // element and copy data of chunk k + 1 are loaded while chunk k is
        // summed and updated, and chunk k's node results are stored during chunk
        // k + 1 (process_held; the LDS-staging variants load the copy data
        // ahead and the element data during the scatter).  FP64 and the
        // occupancy variant keep the plain order (their registers do not hold
        // the pipeline).
        for (int w0 = 0; w0 < nmine; w0 += KMAXB) {
        const int wn = window(w0);
        if constexpr (!K::PIPE) {
            for (int k = 0; k < wn; k++) {
                const int kind = __builtin_amdgcn_readfirstlane(s_kind[k]);
                const int kn = k + 1 < wn ? k + 1 : 0;
                on_kind(kind, [&](auto kc) {
                    constexpr int KC = decltype(kc)::value;
                    const StepPtrs<T> sp = kind_ptrs<T>(bd.k[KC], cur, prv, nxt, s, n);
                    K::template C<KC>::template element_phase<1>(bd.k[KC].tp, s_ch[k], sp, smem, po,
                                                                  [&]() { prefetch(kn); });
                });
                if (po.bad && bad_kind < 0) bad_kind = kind;
            }
        } else
        for (int k0 = 0; k0 < wn;) {
            const int kind = __builtin_amdgcn_readfirstlane(s_kind[k0]);
            int k1 = k0 + 1;
            while (k1 < wn && s_kind[k1] == kind) k1++;
            on_kind(kind, [&](auto kc) {
                constexpr int KC = decltype(kc)::value;
                using CK = typename K::template C<KC>;
                const StepPtrs<T> sp = kind_ptrs<T>(bd.k[KC], cur, prv, nxt, s, n);
                typename CK::CopyRegs cp;
                if constexpr (!K::PF) {
                    // one wait per chunk; the node results go out during the next chunk
                    typename CK::ElemRegs er;
                    typename CK::Held held;
                    CK::held_clear(held);
                    CK::load_elems(bd.k[KC].tp, s_ch[k0], er);
                    CK::template load_copies<1>(bd.k[KC].tp, s_ch[k0], sp, cp);
                    for (int k = k0; k < k1; k++) {
                        CK::process_held(
                            s_ch[k], sp, smem, po, er, cp, held,
                            [&](int j) {
                                if (k + 1 < k1) CK::load_elem(bd.k[KC].tp, s_ch[k + 1], er, j);
                            },
                            [&]() {
                                if (k + 1 < k1) CK::template load_copies<1>(bd.k[KC].tp, s_ch[k + 1], sp, cp);
                            });
                    }
                    CK::held_store(held, sp);
                    return;
                }
                CK::template load_copies<1>(bd.k[KC].tp, s_ch[k0], sp, cp);
                for (int k = k0; k < k1; k++) {
                    const int kn = k + 1 < wn ? k + 1 : 0;
                    typename CK::ElemRegs er;
                    CK::load_elems(bd.k[KC].tp, s_ch[k], er);
                    CK::template process<1, true>(bd.k[KC].tp, s_ch[k], sp, smem, po, er, cp, [&]() {
                        prefetch(kn);
                        if (k + 1 < k1) CK::template load_copies<1>(bd.k[KC].tp, s_ch[k + 1], sp, cp);
                    });
                }
            });
            if (po.bad && bad_kind < 0) bad_kind = kind;
            k0 = k1;
        }
        }
        INSTR_T(t1);
        // shared-node batches: up to KB consecutive chunks of one kind (window wn)
        auto batch_len = [&](int k0, int wn) {
            int nb = 1;
            while (nb < KB && k0 + nb < wn && s_kind[k0 + nb] == s_kind[k0]) nb++;
            return nb;
        };
        const int wn0 = nmine > 0 ? window(0) : 0;
        SharedRegs<T, KB> sr;
        const int nb0 = nmine > 0 ? batch_len(0, wn0) : 0;
        const int kind0 = nmine > 0 ? __builtin_amdgcn_readfirstlane(s_kind[0]) : 0;
        // FP32 register and staging variants with one window: one memory round per
        // round of shared copies (Chunk::shared_fetch_l); the first round's indices
        // go out before the barrier
        bool spipe = false;
        if constexpr (K::PIPE) spipe = nmine > 0 && nmine <= KMAXB;
        // the shared copies of a run of chunks of one kind, concatenated in chunk
        // order: copy g goes to thread g % BLOCK, slot (g / BLOCK) % SS of round g / (SS BLOCK)
        auto slots = [&](int r0, int r1, int g, int (&ls)[SS]) {
#pragma unroll
            for (int q = 0; q < SS; q++) {
                const int gq = g + q * BLOCK + int(threadIdx.x);
                ls[q] = -1;
                if (gq < s_pre[r1]) {
                    int lo = r0, hi = r1 - 1;  // the chunk k with s_pre[k] <= gq < s_pre[k + 1]
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= gq) lo = mid;
                        else hi = mid - 1;
                    }
                    ls[q] = s_ch[lo].copy_begin + s_ch[lo].n_interior + (gq - s_pre[lo]);
                }
            }
        };
        auto run_end = [&](int r0) {
            int r1 = r0 + 1;
            while (r1 < wn0 && s_kind[r1] == s_kind[r0]) r1++;
            return r1;
        };
        typename CS::template SharedIdx<SS> xa;
        int la[SS];
        if (nmine > 0)
            on_kind(kind0, [&](auto kc) {
                constexpr int KC = decltype(kc)::value;
                const StepPtrs<T> sp = kind_ptrs<T>(bd.k[KC], cur, prv, nxt, s, n);
                if constexpr (K::PIPE) {
                    if (spipe) {
                        slots(0, run_end(0), s_pre[0], la);
                        CS::template shared_idx_l<SS>(bd.k[KC].tp, sp, la, xa);
                        return;
                    }
                }
                CS::template shared_load<1, KB>(bd.k[KC].tp, s_ch, nb0, 0, sp, sr);
            });
        int32_t *errw = &bd.status[5 + (s & 1)];
        if (po.bad) {
            if (atomicCAS(errw, 0, po.bad) == 0) {
                // kind << 28 | element, or kind << 28 | 1 << 27 | copy for a node-level error
                bd.status[2] = po.bad_elem >= 0 ? ((bad_kind << 28) | po.bad_elem)
                             : po.bad_elem <= -2 ? ((bad_kind << 28) | (1 << 27) | (-2 - po.bad_elem)) : -1;
                bd.status[3] = int32_t(n);  // absolute step index
            }
        }
        INSTR_T(t2);
        if (!grid_barrier(bd.bar, G, epoch, bd.status)) {
            code = DJ_ERR_BARRIER;
            break;
        }
        INSTR_T(t3);
        if (threadIdx.x == 0) s_flag = ld_dev(errw);
        __syncthreads();
        if (s_flag != 0) {
            code = s_flag;
            break;
        }
        int late_kind = -1;
        bool shared_done = false;
        if constexpr (K::PIPE) {
            if (spipe) {
                // runs of chunks of one kind; per round of SS x BLOCK shared copies one
                // memory round: their state and partials, the next round's indices
                // and the previous round's stores.  The first round's indices went out
                // before the barrier; a later run fetches its first ones on entry.
                SharedRegs<T, SS> rs;
                for (int r0 = 0; r0 < wn0;) {
                    const int kind = __builtin_amdgcn_readfirstlane(s_kind[r0]);
                    const int r1 = run_end(r0);
                    on_kind(kind, [&](auto kc) {
                        constexpr int KC = decltype(kc)::value;
                        const StepPtrs<T> sp = kind_ptrs<T>(bd.k[KC], cur, prv, nxt, s, n);
                        const DevTopo &tp = bd.k[KC].tp;
                        const int g1 = s_pre[r1];
                        if (r0 > 0) {
                            slots(r0, r1, s_pre[r0], la);
                            CS::template shared_idx_l<SS>(tp, sp, la, xa);
                        }
                        typename CS::template SharedIdx<SS> xb;
                        typename CS::template SharedPart<SS> pt;
                        typename CS::template SharedHeld<SS> hs;
#pragma unroll
                        for (int q = 0; q < SS; q++) hs.l[q] = -1;
                        for (int g = s_pre[r0]; g < g1; g += SS * BLOCK) {
                            CS::template shared_fetch_l<SS>(sp, la, xa, rs, pt);
                            const bool live = g + SS * BLOCK < g1;
                            int lb[SS];
                            if (live) {
                                slots(r0, r1, g + SS * BLOCK, lb);
                                CS::template shared_idx_l<SS>(tp, sp, lb, xb);
                            }
#pragma unroll
                            for (int q = 0; q < SS; q++)
                                if (hs.l[q] >= 0)
                                    st_u3<true>(sp.un, hs.l[q], hs.v[q]);
                            __builtin_amdgcn_s_waitcnt(0);
                            __builtin_amdgcn_sched_barrier(0);
                            const bool was_bad = po.bad != 0;
                            CS::template shared_values<SS>(rs, pt, sp, po, hs);
                            if (!was_bad && po.bad) late_kind = kind;
                            if (!live) break;
                            xa = xb;
#pragma unroll
                            for (int q = 0; q < SS; q++) la[q] = lb[q];
                        }
#pragma unroll
                        for (int q = 0; q < SS; q++)
                            if (hs.l[q] >= 0)
                                st_u3<true>(sp.un, hs.l[q], hs.v[q]);
                    });
                    r0 = r1;
                }
                shared_done = true;
            }
        }
        if (!shared_done) {
        // the first batch (its round A is in registers), then the rest
        if (nmine > 0)
            on_kind(kind0, [&](auto kc) {
                constexpr int KC = decltype(kc)::value;
                const StepPtrs<T> sp = kind_ptrs<T>(bd.k[KC], cur, prv, nxt, s, n);
                CS::template shared_finish<1, KB>(bd.k[KC].tp, sr, sp, po);
                CS::template shared_batch<1, KB>(bd.k[KC].tp, s_ch, nb0, 1, sp, po);
            });
        late_kind = po.bad ? kind0 : -1;
        for (int w0 = 0; w0 < nmine; w0 += KMAXB) {
            const int wn = w0 == 0 ? wn0 : window(w0);
            for (int k0 = w0 == 0 ? nb0 : 0; k0 < wn;) {
                const int nb = batch_len(k0, wn);
                const int kind = __builtin_amdgcn_readfirstlane(s_kind[k0]);
                on_kind(kind, [&](auto kc) {
                    constexpr int KC = decltype(kc)::value;
                    const StepPtrs<T> sp = kind_ptrs<T>(bd.k[KC], cur, prv, nxt, s, n);
                    CS::template shared_batch<1, KB>(bd.k[KC].tp, s_ch + k0, nb, 0, sp, po);
                });
                if (po.bad && late_kind < 0) late_kind = kind;
                k0 += nb;
            }
        }
        }
        // a node-level error of the shared-node phase stops the run at the next barrier
        if (po.bad && po.bad_elem <= -2)
            publish_late_error(bd.status, s, po.bad, (late_kind << 28) | (1 << 27) | (-2 - po.bad_elem), int32_t(n));
        __syncthreads();  // shared copies written above are read by other threads next step
#ifdef DJ_INSTR
        INSTR_T(t4);
        instr_add(0, t1 - t0);
        instr_add(1, t2 - t1);
        instr_add(2, t3 - t2);
        instr_add(7, t4 - t3);
        instr_add(8, 1);
#endif
        cur = nxt;
    }
    __builtin_amdgcn_s_waitcnt(0);  // no staged load outlives the workgroup
    __syncthreads();
    if (code == DJ_ERR_BARRIER) {  // sticky for the launches that follow in this run
        if (threadIdx.x == 0) st_dev(&bd.status[0], int32_t(DJ_ERR_BARRIER));
        return;
    }
    if (threadIdx.x == 0) bd.tstamp[2 * blockIdx.x + 1] = uint64_t(wall_clock64());
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // on an error the failing step is not completed: cur still names u^n
        bd.status[0] = code;
        bd.status[1] = s;
        bd.clock[0] = step0 + s;
        bd.clock[1] = cur;
    }
}

__global__ void k_batch_reset(uint32_t *sync, int n_sync, int32_t *status, int clear_status) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_sync; i += gridDim.x * blockDim.x) sync[i] = 0u;
    // a run starts with a clear status; later launches of the run keep the
    // code, error and abort words and clear only the per-parity error words,
    // after making an error that the previous launch found in its last step's
    // shared-node phase (left in a parity word) the run's code
    if (clear_status && blockIdx.x == 0 && threadIdx.x < 8) status[threadIdx.x] = threadIdx.x == 2 ? -1 : 0;
    if (!clear_status && blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t late = status[5] != 0 ? status[5] : status[6];
        if (status[0] == 0 && late != 0) status[0] = late;
        status[5] = 0;
        status[6] = 0;
    }
}

template <typename T>
__global__ void k_pack_copy_pairs(int n_copies, const T *__restrict__ A, const T *__restrict__ bp,
                                  const T *__restrict__ ru, const T *__restrict__ rate, T *__restrict__ ab,
                                  T *__restrict__ rq) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_copies) return;
    ab[2 * int64_t(l)] = A[l];
    ab[2 * int64_t(l) + 1] = bp[l];
    if (rq) {
#pragma unroll
        for (int k = 0; k < 3; k++) rq[4 * int64_t(l) + k] = ru[int64_t(k) * n_copies + l];
        rq[4 * int64_t(l) + 3] = rate ? rate[l] : T(0);
    }
}

// canonical copies -> caller-order arrays of the kind's instances
template <typename T>
__global__ void k_gather_canon(const uint32_t *__restrict__ flags, const int32_t *__restrict__ cnode, int n_copies,
                               const T *__restrict__ uc, const T *__restrict__ up, T *__restrict__ oc,
                               T *__restrict__ op) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_copies || !(flags[l] & FLAG_CANON)) return;
    const int nd = cnode[l];
#pragma unroll
    for (int k = 0; k < 3; k++) {  // copy-major state
        oc[3 * int64_t(nd) + k] = uc[3 * int64_t(l) + k];
        op[3 * int64_t(nd) + k] = up[3 * int64_t(l) + k];
    }
}

template <typename T, int V>
hipError_t occ_t(int *bpc, size_t *lds, int *block) {
    *lds = Kinds<T, V>::LDS;
    *block = Kinds<T, V>::BLOCK;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_batch_step<T, V>, Kinds<T, V>::BLOCK,
                                                        Kinds<T, V>::LDS);
}

template <typename T, int V>
hipError_t launch_t(const BatchDev &bd, int grid, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&k_batch_step<T, V>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(Kinds<T, V>::LDS));
    if (e != hipSuccess) return e;
    BatchDev b = bd;
    void *args[] = {&b};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(Kinds<T, V>::BLOCK), args, Kinds<T, V>::LDS, s);
}

template <typename F>
hipError_t batch_dispatch(int prec, int v, F &&f) {
    if (prec == DJ_FP32) {
        switch (v) {
            case 0: return f(std::integral_constant<int, 0>(), float());
            case 1: return f(std::integral_constant<int, 1>(), float());
            case 2: return f(std::integral_constant<int, 2>(), float());
            case 3: return f(std::integral_constant<int, 3>(), float());
            case 4: return f(std::integral_constant<int, 4>(), float());
            case 5: return f(std::integral_constant<int, 5>(), float());
            case 6: return f(std::integral_constant<int, 6>(), float());
            case 7: return f(std::integral_constant<int, 7>(), float());
            case 8: return f(std::integral_constant<int, 8>(), float());
            default: return hipErrorInvalidValue;
        }
    }
    if (v == 0) return f(std::integral_constant<int, 0>(), double());
    return hipErrorInvalidValue;
}

}  // namespace

#ifdef DJ_INSTR
hipError_t instr_set(uint64_t *p) {
    unsigned long long *q = reinterpret_cast<unsigned long long *>(p);
    return hipMemcpyToSymbol(HIP_SYMBOL(dj_instr_buf), &q, sizeof(q));
}
#endif

bool batch_variant_ok(int prec, int v) { return prec == DJ_FP32 ? (v >= 0 && v < 9) : v == 0; }

int batch_geometry(int v) { return v < 8 ? (v & 3) : 2; }

hipError_t batch_occupancy(int prec, int v, int *bpc, size_t *lds, int *block) {
    return batch_dispatch(prec, v, [&](auto vc, auto t) {
        using T = decltype(t);
        return occ_t<T, decltype(vc)::value>(bpc, lds, block);
    });
}

hipError_t launch_batch_step(const BatchDev &bd, int prec, int v, int grid, hipStream_t s) {
    return batch_dispatch(prec, v, [&](auto vc, auto t) {
        using T = decltype(t);
        return launch_t<T, decltype(vc)::value>(bd, grid, s);
    });
}

hipError_t launch_batch_reset(uint32_t *bar, int n_sync, int32_t *status, bool clear_status, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3((n_sync + 255) / 256), dim3(256), 0, s, bar, n_sync, status,
                       clear_status ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pack_copy_pairs(int prec, int n_copies, const void *acoef, const void *bpc, const void *ru,
                                  const void *rate, void *ab, void *rq, hipStream_t s) {
    const int B = 256;
    const dim3 g((n_copies + B - 1) / B);
    if (prec == DJ_FP32)
        hipLaunchKernelGGL(k_pack_copy_pairs<float>, g, dim3(B), 0, s, n_copies, static_cast<const float *>(acoef),
                           static_cast<const float *>(bpc), static_cast<const float *>(ru),
                           static_cast<const float *>(rate), static_cast<float *>(ab), static_cast<float *>(rq));
    else
        hipLaunchKernelGGL(k_pack_copy_pairs<double>, g, dim3(B), 0, s, n_copies, static_cast<const double *>(acoef),
                           static_cast<const double *>(bpc), static_cast<const double *>(ru),
                           static_cast<const double *>(rate), static_cast<double *>(ab), static_cast<double *>(rq));
    return hipGetLastError();
}

hipError_t launch_gather_canon(const BatchKind &kd, int prec, int cur, void *oc, void *op, hipStream_t s) {
    const int L = kd.tp.n_copies, B = 256;
    const int prv = (cur + 2) % 3;
    if (prec == DJ_FP32)
        hipLaunchKernelGGL(k_gather_canon<float>, dim3((L + B - 1) / B), dim3(B), 0, s, kd.flags, kd.tp.cnode, L,
                           static_cast<const float *>(kd.ubuf[cur]), static_cast<const float *>(kd.ubuf[prv]),
                           static_cast<float *>(oc), static_cast<float *>(op));
    else
        hipLaunchKernelGGL(k_gather_canon<double>, dim3((L + B - 1) / B), dim3(B), 0, s, kd.flags, kd.tp.cnode, L,
                           static_cast<const double *>(kd.ubuf[cur]), static_cast<const double *>(kd.ubuf[prv]),
                           static_cast<double *>(oc), static_cast<double *>(op));
    return hipGetLastError();
}

hipError_t launch_scatter_state(const BatchKind &kd, int prec, int cur, const void *ic, const void *ip,
                                hipStream_t s) {
    const int L = kd.tp.n_copies, B = 256;
    const int prv = (cur + 2) % 3;
    if (prec == DJ_FP32)
        hipLaunchKernelGGL((k_scatter_in<float, true>), dim3((L + B - 1) / B), dim3(B), 0, s, kd.tp.cnode, L,
                           static_cast<const float *>(ic), static_cast<const float *>(ip),
                           static_cast<float *>(kd.ubuf[cur]), static_cast<float *>(kd.ubuf[prv]));
    else
        hipLaunchKernelGGL((k_scatter_in<double, true>), dim3((L + B - 1) / B), dim3(B), 0, s, kd.tp.cnode, L,
                           static_cast<const double *>(ic), static_cast<const double *>(ip),
                           static_cast<double *>(kd.ubuf[cur]), static_cast<double *>(kd.ubuf[prv]));
    return hipGetLastError();
}

}  // namespace dj
