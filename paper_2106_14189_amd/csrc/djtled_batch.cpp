// Batches of independent DJ-TLED instances (the djtled_batch_* entry points):
// grouping of the instances by element kind into multi-instance contexts,
// the batch work list, the autotuner, graph capture of a run, state copies.
// All arithmetic of the method runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "djtled_batch.h"
#include "djtled_internal.h"

using namespace dj;

namespace {

struct Batch {
    int device = 0, prec = DJ_FP32, n_inst = 0;
    int variant = 1, chunk_elems = 0, spl = 0, use_graph = 1;
    int grid = 0, block = 256, n_items = 0;
    Ctx *kc[4] = {nullptr, nullptr, nullptr, nullptr};
    LoadSet *kls[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<int> inst_kind, inst_pos;          // kind, position within the kind's instances
    std::vector<int> members[4];                   // instances of each kind, by position
    std::vector<std::vector<int>> inst_wgs;        // workgroups holding chunks of each instance
    std::vector<void *> allocs;
    void *d_ab[4] = {}, *d_rq[4] = {};  // per kind: (A, B') pairs and (load, rate) quads of the copies
    int32_t *d_work = nullptr;
    uint32_t *d_bar = nullptr;
    int32_t *d_status = nullptr;
    int64_t *d_clock = nullptr;
    uint64_t *d_ts = nullptr;
    int32_t *h_status = nullptr;
    int64_t *h_clock = nullptr;
    uint64_t *h_ts = nullptr;
    void *d_stage[4][2] = {};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t own = nullptr;   // runs of callers on the null stream (graphs need a real stream)
    // captured runs, one per (steps, stream), the most recent last
    struct Graph {
        int steps;
        hipStream_t stream;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    static constexpr size_t MAX_GRAPHS = 4;
    std::vector<Graph> graphs;
    int graph_used = 0;
    int64_t step = 0;
    int cur = 0;
    double bytes_per_step = 0, tune_ms = 0, wclk_khz = 0;
    int tune_candidates = 0, error_inst = -1;
    int64_t n_elems = 0, n_nodes = 0;
    std::vector<double> inst_ms;
};

void destroy_batch(Batch *b) {
    if (!b) return;
    hipSetDevice(b->device);
    hipDeviceSynchronize();
    for (auto &g : b->graphs) {
        hipGraphExecDestroy(g.exec);
        hipGraphDestroy(g.graph);
    }
    for (int k = 0; k < 4; k++) {
        if (b->kc[k]) free_all(b->kc[k]);  // frees the kind's load sets too
        for (int j = 0; j < 2; j++)
            if (b->d_stage[k][j]) hipFree(b->d_stage[k][j]);
    }
    for (void *p : b->allocs) hipFree(p);
    if (b->h_status) hipHostFree(b->h_status);
    if (b->h_clock) hipHostFree(b->h_clock);
    if (b->h_ts) hipHostFree(b->h_ts);
    if (b->ev0) hipEventDestroy(b->ev0);
    if (b->ev1) hipEventDestroy(b->ev1);
    if (b->own) hipStreamDestroy(b->own);
    delete b;
}

template <typename T>
hipError_t balloc(Batch &b, T **p, size_t n) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) {
        b.allocs.push_back(q);
        *p = static_cast<T *>(q);
    }
    return e;
}

int check_instance(int i, const djtled_mesh &m, const djtled_material &mat, const djtled_loads &ld) {
    const std::string w = "instance " + std::to_string(i) + ": ";
    if (m.n_nodes <= 0 || m.n_elems <= 0 || !m.X || !m.conn) return fail(DJ_ERR_ARG, w + "empty mesh or null arrays");
    if (m.elem_type != DJ_T4 && m.elem_type != DJ_H8) return fail(DJ_ERR_UNSUPPORTED, w + "elem_type must be 4 or 8");
    if (mat.model != DJ_NH && mat.model != DJ_TI) return fail(DJ_ERR_UNSUPPORTED, w + "model must be DJ_NH or DJ_TI");
    if (!(mat.rho > 0)) return fail(DJ_ERR_ARG, w + "rho must be > 0");
    if (mat.model == DJ_TI && !mat.fibre) return fail(DJ_ERR_ARG, w + "DJ_TI needs fibre directions");
    const int64_t nconn = int64_t(m.n_elems) * m.elem_type;
    for (int64_t j = 0; j < nconn; j++)
        if (m.conn[j] < 0 || m.conn[j] >= m.n_nodes)
            return fail(DJ_ERR_BAD_MESH, w + "node index out of range in element " + std::to_string(j / m.elem_type));
    for (int64_t j = 0; j < 3 * int64_t(m.n_nodes); j++)
        if (!std::isfinite(m.X[j])) return fail(DJ_ERR_BAD_MESH, w + "non-finite coordinate");
    if (ld.R) return fail(DJ_ERR_UNSUPPORTED, w + "external forces are not supported in batches");
    if (ld.n_bc < 0 || (ld.n_bc > 0 && (!ld.bc_node || !ld.bc_mask || !ld.bc_target)))
        return fail(DJ_ERR_ARG, w + "bad boundary-condition arrays");
    if (ld.ramp < DJ_RAMP_NONE || ld.ramp > DJ_RAMP_SMOOTH || !std::isfinite(ld.t_ramp))
        return fail(DJ_ERR_ARG, w + "bad ramp");
    for (int j = 0; j < ld.n_bc; j++) {
        if (ld.bc_node[j] < 0 || ld.bc_node[j] >= m.n_nodes)
            return fail(DJ_ERR_ARG, w + "boundary-condition node out of range");
        if (ld.bc_mask[j] & ~7) return fail(DJ_ERR_ARG, w + "boundary-condition mask must be within 0..7");
    }
    return DJ_OK;
}

// Builds the kind contexts, load sets and the work list of `sel` instances.
int build_batch(Batch &b, const std::vector<int> &sel, const djtled_mesh *meshes, const djtled_material *mats,
                const djtled_loads *loads, const double *alpha, const djtled_params *prm, int variant,
                int chunk_elems) {
    b.variant = variant;
    b.chunk_elems = chunk_elems;
    b.n_inst = int(sel.size());
    b.inst_kind.assign(b.n_inst, 0);
    b.inst_pos.assign(b.n_inst, 0);
    auto &members = b.members;
    for (int k = 0; k < 4; k++) members[k].clear();
    for (int i = 0; i < b.n_inst; i++) {
        const int s = sel[i];
        const int k = kind_of(meshes[s].elem_type, mats[s].model);
        b.inst_kind[i] = k;
        b.inst_pos[i] = int(members[k].size());
        members[k].push_back(i);
    }
    b.n_elems = 0;
    b.n_nodes = 0;
    b.bytes_per_step = 0;
    for (int k = 0; k < 4; k++) {
        if (members[k].empty()) continue;
        const int NE = (k >= 2) ? 8 : 4, model = (k & 1) ? DJ_TI : DJ_NH;
        const auto &mem = members[k];
        const int ni = int(mem.size());
        std::vector<int32_t> noff(ni + 1, 0), eoff(ni + 1, 0);
        for (int j = 0; j < ni; j++) {
            const int s = sel[mem[j]];
            noff[j + 1] = noff[j] + meshes[s].n_nodes;
            eoff[j + 1] = eoff[j] + meshes[s].n_elems;
            if (int64_t(noff[j + 1]) > (int64_t(1) << 30) || int64_t(eoff[j + 1]) >= (int64_t(1) << 27))
                return fail(DJ_ERR_UNSUPPORTED, "batch kind too large for 27-bit element indices");
        }
        const int N = noff[ni], E = eoff[ni];
        std::vector<double> X(size_t(3) * N), Ev(E), nuv(E), eta, fib, al(ni), rate(N, 0.0);
        std::vector<int32_t> conn(size_t(NE) * E);
        if (model == DJ_TI) {
            eta.resize(E);
            fib.resize(size_t(3) * E);
        }
        const djtled_material &m0 = mats[sel[mem[0]]];
        const double hgk0 = m0.hg_kappa < 0 ? 0.1 : m0.hg_kappa;
        std::vector<int32_t> bn, bm;
        std::vector<double> bt;
        for (int j = 0; j < ni; j++) {
            const int s = sel[mem[j]];
            const djtled_mesh &m = meshes[s];
            const djtled_material &mt = mats[s];
            if (mt.rho != m0.rho || (mt.hg_kappa < 0 ? 0.1 : mt.hg_kappa) != hgk0)
                return fail(DJ_ERR_UNSUPPORTED, "instances of one element kind must share rho and hg_kappa");
            std::memcpy(&X[size_t(3) * noff[j]], m.X, sizeof(double) * 3 * m.n_nodes);
            for (int64_t q = 0; q < int64_t(NE) * m.n_elems; q++) conn[size_t(NE) * eoff[j] + q] = m.conn[q] + noff[j];
            for (int e = 0; e < m.n_elems; e++) {
                Ev[eoff[j] + e] = mt.E ? mt.E[e] : mt.E_uniform;
                nuv[eoff[j] + e] = mt.nu ? mt.nu[e] : mt.nu_uniform;
                if (model == DJ_TI) {
                    eta[eoff[j] + e] = mt.eta_ratio ? mt.eta_ratio[e] : mt.eta_ratio_uniform;
                    for (int c = 0; c < 3; c++) fib[size_t(3) * (eoff[j] + e) + c] = mt.fibre[size_t(3) * e + c];
                }
            }
            al[j] = alpha ? alpha[s] : prm->alpha;
            if (!(al[j] >= 0)) return fail(DJ_ERR_ARG, "alpha must be >= 0");
            const djtled_loads &ld = loads[s];
            for (int q = 0; q < ld.n_bc; q++) {
                bn.push_back(ld.bc_node[q] + noff[j]);
                bm.push_back(ld.bc_mask[q]);
                for (int c = 0; c < 3; c++) bt.push_back(ld.bc_target[3 * q + c]);
            }
        }
        djtled_mesh um{N, E, NE, X.data(), conn.data()};
        djtled_material umat{};
        umat.model = model;
        umat.E = Ev.data();
        umat.nu = nuv.data();
        umat.rho = m0.rho;
        umat.hg_kappa = hgk0;
        if (model == DJ_TI) {
            umat.eta_ratio = eta.data();
            umat.fibre = fib.data();
        }
        djtled_params kp = *prm;
        kp.variant = batch_geometry(variant);  // the chunk geometry of the batch kernel's variant
        kp.chunk_elems = chunk_elems;
        kp.dt = 0.0;
        MultiInst mi;
        mi.n_inst = ni;
        mi.node_off = noff.data();
        mi.elem_off = eoff.data();
        mi.alpha = al.data();
        mi.batch = 1;
        Ctx *c = new Ctx();
        c->device = b.device;
        int rc = build(*c, &um, &umat, &kp, &mi);
        if (rc != DJ_OK) {
            std::string msg = g_err;
            free_all(c);
            return fail(rc, "element kind " + std::to_string(k) + ": " + msg);
        }
        b.kc[k] = c;
        // the instances' ramps as per-node signed rates (see ramp_rate in the kernels)
        for (int j = 0; j < ni; j++) {
            const djtled_loads &ld = loads[sel[mem[j]]];
            double q = 0.0;  // t_ramp < 0: |t_ramp| steps of the instance's own dt
            if (ld.ramp != DJ_RAMP_NONE && ld.t_ramp != 0) {
                q = ld.t_ramp > 0 ? c->inst_dt[j] / ld.t_ramp : 1.0 / -ld.t_ramp;
                if (ld.ramp == DJ_RAMP_LINEAR) q = -q;
            }
            for (int n = noff[j]; n < noff[j + 1]; n++) rate[n] = q;
        }
        djtled_loads uld{int32_t(bn.size()), bn.data(), bm.data(), bt.data(), DJ_RAMP_NONE, 0.0, nullptr};
        LoadSet *ls = nullptr;
        rc = make_loadset(*c, &uld, rate.data(), &ls);
        if (rc != DJ_OK) return rc;
        b.kls[k] = ls;
        {
            const size_t L = size_t(c->topo.n_copies), tsz = b.prec == DJ_FP32 ? 4 : 8;
            DJ_HIP(hipMalloc(&b.d_ab[k], std::max<size_t>(L, 1) * 2 * tsz));
            b.allocs.push_back(b.d_ab[k]);
            if (ls->d_ru) {
                DJ_HIP(hipMalloc(&b.d_rq[k], std::max<size_t>(L, 1) * 4 * tsz));
                b.allocs.push_back(b.d_rq[k]);
            }
            DJ_HIP(launch_pack_copy_pairs(b.prec, int(L), c->d_acoef, c->d_bpc, ls->d_ru, ls->d_rate, b.d_ab[k],
                                          b.d_rq[k], nullptr));
        }
        const size_t ts = b.prec == DJ_FP32 ? 4 : 8;
        for (int q = 0; q < 3; q++) DJ_HIP(hipMemset(c->d_ubuf[q], 0, size_t(3) * c->topo.n_copies * ts));
        b.n_elems += E;
        b.n_nodes += N;
        // traffic: the single-instance model plus the per-copy B' (and ramp rate of loaded copies)
        b.bytes_per_step += c->bytes_per_step + double(c->topo.n_copies) * ts;
    }
    // ---- work list: every chunk of every kind, sorted by kind, dealt round-robin
    std::vector<int32_t> work;
    for (int k = 0; k < 4; k++)
        if (b.kc[k])
            for (int ch = 0; ch < b.kc[k]->topo.n_chunks; ch++) work.push_back((k << 28) | ch);
    b.n_items = int(work.size());
    int bpc = 0, blk = 0;
    size_t lds = 0;
    DJ_HIP(batch_occupancy(b.prec, variant, &bpc, &lds, &blk));
    hipDeviceProp_t prop;
    DJ_HIP(hipGetDeviceProperties(&prop, b.device));
    if (bpc < 1) return fail(DJ_ERR_UNSUPPORTED, "batch kernel variant does not fit on a compute unit");
    b.block = blk;
    b.grid = std::min(bpc * prop.multiProcessorCount, b.n_items);
    // the prefetch variants keep every work item of a workgroup in its LDS list
    if (variant >= 4 && variant < 8 && (b.n_items + b.grid - 1) / b.grid > KMAXB)
        return fail(DJ_ERR_UNSUPPORTED, "batch needs more than " + std::to_string(KMAXB) +
                                            " chunks per workgroup for the prefetch variants 4..7");
    // workgroups holding each instance's chunks (for per-instance completion times)
    b.inst_wgs.assign(b.n_inst, {});
    for (int j = 0; j < b.n_items; j++) {
        const int k = work[j] >> 28, ch = work[j] & 0x0fffffff;
        const Ctx &c = *b.kc[k];
        const int wg = j % b.grid;
        // chunk element range -> instances (elements of an instance are contiguous internally)
        const int32_t eb = c.h_chunk_elem[2 * ch], ee = eb + c.h_chunk_elem[2 * ch + 1];
        int last = -1;
        for (int e = eb; e < ee; e++) {
            const int ce = c.elem_perm[e];
            const int jj = int(std::upper_bound(c.inst_elem_off.begin(), c.inst_elem_off.end(), ce) -
                               c.inst_elem_off.begin()) - 1;
            if (jj == last) continue;
            last = jj;
            auto &v = b.inst_wgs[members[k][jj]];
            if (std::find(v.begin(), v.end(), wg) == v.end()) v.push_back(wg);
        }
    }
    DJ_HIP(balloc(b, &b.d_work, work.size()));
    DJ_HIP(hipMemcpy(b.d_work, work.data(), work.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    DJ_HIP(balloc(b, &b.d_bar, size_t(b.grid + 16) * 32));
    DJ_HIP(hipMemset(b.d_bar, 0, size_t(b.grid + 16) * 32 * sizeof(uint32_t)));
    DJ_HIP(balloc(b, &b.d_status, 8));
    DJ_HIP(hipMemset(b.d_status, 0, 8 * sizeof(int32_t)));
    DJ_HIP(balloc(b, &b.d_clock, 2));
    DJ_HIP(hipMemset(b.d_clock, 0, 2 * sizeof(int64_t)));
#ifdef DJ_INSTR
    DJ_HIP(balloc(b, &b.d_ts, size_t(18) * b.grid));  // + 16 sub-phase counters per workgroup
    DJ_HIP(hipMemset(b.d_ts, 0, size_t(18) * b.grid * sizeof(uint64_t)));
#else
    DJ_HIP(balloc(b, &b.d_ts, size_t(2) * b.grid));
#endif
    DJ_HIP(hipHostMalloc(reinterpret_cast<void **>(&b.h_status), 8 * sizeof(int32_t), hipHostMallocDefault));
    DJ_HIP(hipHostMalloc(reinterpret_cast<void **>(&b.h_clock), 2 * sizeof(int64_t), hipHostMallocDefault));
    DJ_HIP(hipHostMalloc(reinterpret_cast<void **>(&b.h_ts), size_t(2) * b.grid * sizeof(uint64_t),
                         hipHostMallocDefault));
    DJ_HIP(hipEventCreate(&b.ev0));
    DJ_HIP(hipEventCreate(&b.ev1));
    DJ_HIP(hipStreamCreateWithFlags(&b.own, hipStreamNonBlocking));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b.device) == hipSuccess) b.wclk_khz = khz;
    b.inst_ms.assign(b.n_inst, 0.0);
    DJ_HIP(hipDeviceSynchronize());
    return DJ_OK;
}

BatchDev make_dev(const Batch &b) {
    BatchDev bd;
    for (int k = 0; k < 4; k++) {
        BatchKind &kd = bd.k[k];
        if (!b.kc[k]) continue;
        const Ctx &c = *b.kc[k];
        kd.tp = c.topo;
        kd.flags = b.kls[k]->d_flags;
        kd.ru = b.kls[k]->d_ru;
        kd.rate = b.kls[k]->d_rate;
        for (int q = 0; q < 3; q++) kd.ubuf[q] = c.d_ubuf[q];
        kd.part = c.d_part;
        kd.ab = b.d_ab[k];
        kd.rq = b.d_rq[k];
    }
    bd.work = b.d_work;
    bd.n_items = b.n_items;
    bd.clock = b.d_clock;
    bd.bar = b.d_bar;
    bd.status = b.d_status;
    bd.tstamp = b.d_ts;
    return bd;
}

// enqueue one run of n_steps (reset, then launches of at most spl steps)
hipError_t enqueue_run(Batch &b, int n_steps, hipStream_t s) {
    const int n_sync = (b.grid + 16) * 32;
    const int spl = b.spl > 0 ? b.spl : std::max(n_steps, 1);
    BatchDev bd = make_dev(b);
    hipError_t e = launch_batch_reset(b.d_bar, n_sync, b.d_status, true, s);
    for (int done = 0, j = 0; e == hipSuccess && done < n_steps; j++) {
        const int len = std::min(spl, n_steps - done);
        if (j > 0) e = launch_batch_reset(b.d_bar, n_sync, b.d_status, false, s);
        if (e != hipSuccess) break;
        bd.n_steps = len;
        bd.first_launch = j == 0 ? 1 : 0;
        e = launch_batch_step(bd, b.prec, b.variant, b.grid, s);
        done += len;
    }
    return e;
}

int run_batch(Batch &b, int n_steps, djtled_status *out, hipStream_t s) {
    djtled_status r{DJ_OK, 0, -1, -1, std::numeric_limits<double>::quiet_NaN(), 0.0};
    if (s == nullptr) {  // order after the caller's null-stream work, then use the batch's stream
        DJ_HIP(hipStreamSynchronize(nullptr));
        s = b.own;
    }
    b.error_inst = -1;
    if (n_steps > 0) {
        hipGraphExec_t exec = nullptr;
        if (b.use_graph) {
            for (const auto &g : b.graphs)
                if (g.steps == n_steps && g.stream == s) exec = g.exec;
            if (!exec) {
                if (b.graphs.size() >= Batch::MAX_GRAPHS) {  // drop the oldest capture
                    DJ_HIP(hipStreamSynchronize(b.graphs.front().stream));
                    hipGraphExecDestroy(b.graphs.front().exec);
                    hipGraphDestroy(b.graphs.front().graph);
                    b.graphs.erase(b.graphs.begin());
                }
                // capture; a runtime that cannot record cooperative launches
                // leaves the batch on direct launches
                if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                    const hipError_t ec = enqueue_run(b, n_steps, s);
                    hipGraph_t g = nullptr;
                    const hipError_t ee = hipStreamEndCapture(s, &g);
                    hipGraphExec_t x = nullptr;
                    if (ec == hipSuccess && ee == hipSuccess && g &&
                        hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) {
                        b.graphs.push_back(Batch::Graph{n_steps, s, g, x});
                        exec = x;
                    } else {
                        if (g) hipGraphDestroy(g);
                        (void)hipGetLastError();
                        b.use_graph = 0;
                    }
                } else {
                    (void)hipGetLastError();
                    b.use_graph = 0;
                }
            }
        }
        const bool replay = exec != nullptr;
        DJ_HIP(hipEventRecord(b.ev0, s));
        if (replay) {
            DJ_HIP(hipGraphLaunch(exec, s));
        } else {
            DJ_HIP(enqueue_run(b, n_steps, s));
        }
        DJ_HIP(hipEventRecord(b.ev1, s));
        b.graph_used = replay ? 1 : 0;
    }
    DJ_HIP(hipMemcpyAsync(b.h_status, b.d_status, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DJ_HIP(hipMemcpyAsync(b.h_clock, b.d_clock, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DJ_HIP(hipMemcpyAsync(b.h_ts, b.d_ts, size_t(2) * b.grid * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    DJ_HIP(hipStreamSynchronize(s));
    if (n_steps > 0) {
        float ms = 0.0f;
        r.kernel_ms = hipEventElapsedTime(&ms, b.ev0, b.ev1) == hipSuccess ? double(ms) : -1.0;
        r.code = b.h_status[4] ? DJ_ERR_BARRIER : b.h_status[0];
        // an error of the last step's shared-node phase is left in a parity word
        if (r.code == DJ_OK) r.code = b.h_status[5] != 0 ? b.h_status[5] : b.h_status[6];
        r.steps_done = int32_t(b.h_clock[0] - b.step);
        // per-instance completion: latest end stamp of its workgroups after the earliest start
        uint64_t t0 = std::numeric_limits<uint64_t>::max();
        for (int g = 0; g < b.grid; g++) t0 = std::min(t0, b.h_ts[2 * g]);
        for (int i = 0; i < b.n_inst; i++) {
            uint64_t t1 = t0;
            for (int g : b.inst_wgs[i]) t1 = std::max(t1, b.h_ts[2 * g + 1]);
            b.inst_ms[i] = b.wclk_khz > 0 ? double(t1 - t0) / b.wclk_khz : -1.0;
        }
    }
    if (r.code == DJ_ERR_BARRIER) {
        g_err = "batch kernel grid barrier timed out";
    } else if (r.code == DJ_ERR_INVERTED || r.code == DJ_ERR_NONFINITE) {
        r.error_step = b.h_status[3];  // absolute step index of the failing step
        const int w = b.h_status[2];
        if (w >= 0) {
            const int k = w >> 28;
            const Ctx *c = b.kc[k];
            if (c && (w & (1 << 27))) {  // node-level: the copy's instance
                const int l = w & 0x07ffffff;
                if (l < c->topo.n_copies) {
                    const int cn = c->node_perm[c->h_copy_node[l]];
                    const int jj = int(std::upper_bound(c->inst_node_off.begin(), c->inst_node_off.end(), cn) -
                                       c->inst_node_off.begin()) - 1;
                    b.error_inst = b.members[k][jj];
                }
            } else if (c && (w & 0x07ffffff) < c->n_elems) {
                const int ce = c->elem_perm[w & 0x07ffffff];
                const int jj = int(std::upper_bound(c->inst_elem_off.begin(), c->inst_elem_off.end(), ce) -
                                   c->inst_elem_off.begin()) - 1;
                b.error_inst = b.members[k][jj];
                r.error_elem = ce - c->inst_elem_off[jj];
            }
        }
        g_err = std::string(r.code == DJ_ERR_INVERTED ? "element inverted (J <= 0)" : "non-finite value") +
                " in instance " + std::to_string(b.error_inst) + " at step " + std::to_string(r.error_step);
    }
    if (n_steps > 0) {
        b.step = b.h_clock[0];
        b.cur = int(b.h_clock[1]);
    }
    if (out) *out = r;
    return r.code;
}

int reset_batch(Batch &b, hipStream_t s) {
    const size_t ts = b.prec == DJ_FP32 ? 4 : 8;
    for (int k = 0; k < 4; k++)
        if (b.kc[k])
            for (int q = 0; q < 3; q++)
                DJ_HIP(hipMemsetAsync(b.kc[k]->d_ubuf[q], 0, size_t(3) * b.kc[k]->topo.n_copies * ts, s));
    DJ_HIP(hipMemsetAsync(b.d_clock, 0, 2 * sizeof(int64_t), s));
    DJ_HIP(hipStreamSynchronize(s));
    b.step = 0;
    b.cur = 0;
    return DJ_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int djtled_batch_create(int32_t n, const djtled_mesh *meshes, const djtled_material *materials,
                        const djtled_loads *loads, const double *alpha, const djtled_params *params,
                        const djtled_tune *tune, djtled_batch **out) {
    g_err.clear();
    if (!out) return fail(DJ_ERR_ARG, "null argument");
    *out = nullptr;
    if (n <= 0 || !meshes || !materials || !loads || !params) return fail(DJ_ERR_ARG, "empty batch or null arrays");
    if (params->precision != DJ_FP32 && params->precision != DJ_FP64) return fail(DJ_ERR_UNSUPPORTED, "precision");
    if (params->formulation != DJ_FORM_JACOBIAN)
        return fail(DJ_ERR_UNSUPPORTED, "batches use the Jacobian form (DJ_FORM_JACOBIAN) only");
    if (params->dt != 0.0) return fail(DJ_ERR_ARG, "batches take each instance's own step: dt must be 0");
    if (!(params->alpha >= 0)) return fail(DJ_ERR_ARG, "alpha must be >= 0");
    for (int i = 0; i < n; i++) {
        const int rc = check_instance(i, meshes[i], materials[i], loads[i]);
        if (rc != DJ_OK) return rc;
    }
    djtled_tune tn{0, -1, 0, 0, 1, 0};
    if (tune) tn = *tune;
    const int prec = params->precision;
    int variant = tn.variant < 0 ? (prec == DJ_FP32 ? 1 : 0) : tn.variant;
    if (!batch_variant_ok(prec, variant)) return fail(DJ_ERR_ARG, "unknown batch kernel variant");
    if (tn.chunk_elems < 0 || tn.steps_per_launch < 0 || tn.tune_steps < 0) return fail(DJ_ERR_ARG, "bad tune values");
    int dev = params->device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipSetDevice(dev) != hipSuccess) return fail(DJ_ERR_HIP, "hipSetDevice failed");
    std::vector<int> all(n);
    for (int i = 0; i < n; i++) all[i] = i;
    int chunk = tn.chunk_elems;
    int n_cand = 0;
    std::vector<std::pair<int, int>> cands;  // (variant, chunk) in order of preference
    double t_tune = 0;
    const int tsteps = tn.tune_steps > 0 ? tn.tune_steps : 20;
    if (tn.autotune) {
        // candidates timed on every m-th instance (m <= 8, at least 16 instances when there are that many)
        const double t0 = now_ms();
        const int m = std::max(1, std::min(8, n / 16));
        std::vector<int> sub;
        for (int i = 0; i < n; i += m) sub.push_back(i);
        std::vector<int> vs = prec == DJ_FP32 ? std::vector<int>{1, 2, 5, 6, 0, 3, 4, 7, 8} : std::vector<int>{0};
        std::vector<std::pair<double, std::pair<int, int>>> ranked;  // time per element-step, (variant, chunk)
        for (int v : vs)
            for (int cf : {0, 2}) {
                Batch *t = new Batch();
                t->device = dev;
                t->prec = prec;
                t->use_graph = 0;
                int rc = build_batch(*t, sub, meshes, materials, loads, alpha, params, v, 0);
                if (rc == DJ_OK && cf == 2) {  // half-capacity chunks
                    const int cap = t->kc[0] ? t->kc[0]->cmax : (t->kc[2] ? t->kc[2]->cmax : 0);
                    destroy_batch(t);
                    t = new Batch();
                    t->device = dev;
                    t->prec = prec;
                    t->use_graph = 0;
                    rc = build_batch(*t, sub, meshes, materials, loads, alpha, params, v, std::max(64, cap / 2));
                }
                if (rc == DJ_OK) {
                    djtled_status st;
                    rc = run_batch(*t, 2, &st, nullptr);  // warm-up
                    if (rc == DJ_OK) rc = run_batch(*t, tsteps, &st, nullptr);
                    if (rc == DJ_OK && st.kernel_ms > 0) {
                        n_cand++;
                        ranked.push_back({st.kernel_ms / (double(t->n_elems) * tsteps), {v, t->chunk_elems}});
                    }
                }
                destroy_batch(t);
                g_err.clear();
            }
        t_tune = now_ms() - t0;
        if (n_cand == 0) return fail(DJ_ERR_UNSUPPORTED, "autotuner: no batch kernel candidate ran");
        std::sort(ranked.begin(), ranked.end());
        for (auto &r : ranked) cands.push_back(r.second);
    } else {
        cands.push_back({variant, chunk});
    }
    // the best candidate that can hold the whole batch
    Batch *b = nullptr;
    int rc = DJ_OK;
    for (auto &c : cands) {
        b = new Batch();
        b->device = dev;
        b->prec = prec;
        b->spl = tn.steps_per_launch;
        b->use_graph = tn.use_graph ? 1 : 0;
        rc = build_batch(*b, all, meshes, materials, loads, alpha, params, c.first, c.second);
        if (rc == DJ_OK) break;
        std::string msg = g_err;
        destroy_batch(b);
        b = nullptr;
        g_err = msg;
    }
    if (!b) return rc;
    if (tn.autotune && tn.steps_per_launch == 0) {
        // steps per launch: one launch per run against launches of 32 steps
        const double t0 = now_ms();
        double best = std::numeric_limits<double>::infinity();
        int best_spl = 0;
        const int use_graph = b->use_graph;
        b->use_graph = 0;
        for (int spl : {0, 32}) {
            b->spl = spl;
            djtled_status st;
            rc = run_batch(*b, 64, &st, nullptr);
            if (rc == DJ_OK && st.kernel_ms > 0 && st.kernel_ms < best) {
                best = st.kernel_ms;
                best_spl = spl;
            }
            n_cand++;
        }
        b->spl = best_spl;
        b->use_graph = use_graph;
        rc = reset_batch(*b, nullptr);
        t_tune += now_ms() - t0;
        if (rc != DJ_OK) {
            destroy_batch(b);
            return rc;
        }
    }
    b->tune_candidates = n_cand;
    b->tune_ms = t_tune;
    *out = reinterpret_cast<djtled_batch *>(b);
    return DJ_OK;
}

int djtled_batch_destroy(djtled_batch *p) {
    if (!p) return fail(DJ_ERR_ARG, "null batch");
    destroy_batch(reinterpret_cast<Batch *>(p));
    return DJ_OK;
}

int djtled_batch_info(const djtled_batch *p, djtled_batch_info_t *o) {
    if (!p || !o) return fail(DJ_ERR_ARG, "null argument");
    const Batch &b = *reinterpret_cast<const Batch *>(p);
    int nk = 0;
    for (int k = 0; k < 4; k++) nk += b.kc[k] ? 1 : 0;
    o->n_inst = b.n_inst;
    o->n_kinds = nk;
    o->n_items = b.n_items;
    o->grid_blocks = b.grid;
    o->block_threads = b.block;
    o->variant = b.variant;
    o->chunk_elems = b.chunk_elems;
    o->steps_per_launch = b.spl;
    o->graph = b.graph_used;
    o->tune_candidates = b.tune_candidates;
    o->n_elems = b.n_elems;
    o->n_nodes = b.n_nodes;
    o->bytes_per_step = b.bytes_per_step;
    o->tune_ms = b.tune_ms;
    o->error_inst = b.error_inst;
    return DJ_OK;
}

int djtled_batch_instance(const djtled_batch *p, int32_t inst, djtled_info_t *o) {
    if (!p || !o) return fail(DJ_ERR_ARG, "null argument");
    const Batch &b = *reinterpret_cast<const Batch *>(p);
    if (inst < 0 || inst >= b.n_inst) return fail(DJ_ERR_ARG, "instance out of range");
    const int k = b.inst_kind[inst], j = b.inst_pos[inst];
    const Ctx &c = *b.kc[k];
    std::memset(o, 0, sizeof(*o));
    o->n_nodes = c.inst_node_off[j + 1] - c.inst_node_off[j];
    o->n_elems = c.inst_elem_off[j + 1] - c.inst_elem_off[j];
    o->elem_type = c.ne;
    o->model = c.model;
    o->precision = c.prec;
    o->dt = c.inst_dt[j];
    o->dt_crit = c.inst_dt_crit[j];
    o->alpha = c.inst_alpha[j];
    o->n_chunks = c.topo.n_chunks;
    o->chunk_elems = c.chunk_elems;
    o->n_copies = c.topo.n_copies;
    o->n_shared_copies = c.n_shared_copies;
    o->grid_blocks = b.grid;
    o->block_threads = b.block;
    o->variant = b.variant;
    o->bytes_per_step = c.bytes_per_step;
    o->elem_bytes = c.elem_bytes;
    return DJ_OK;
}

int djtled_batch_run(djtled_batch *p, int32_t n_steps, djtled_status *out, void *stream) {
    if (!p) return fail(DJ_ERR_ARG, "null batch");
    if (n_steps < 0) return fail(DJ_ERR_ARG, "n_steps must be >= 0");
    Batch &b = *reinterpret_cast<Batch *>(p);
    DJ_HIP(hipSetDevice(b.device));
    return run_batch(b, n_steps, out, static_cast<hipStream_t>(stream));
}

#ifdef DJ_INSTR
// instrumented build only: per-workgroup sub-phase counters (16 each)
int djtled_batch_instr(djtled_batch *p, uint64_t *out, int clear) {
    Batch &b = *reinterpret_cast<Batch *>(p);
    DJ_HIP(hipDeviceSynchronize());
    DJ_HIP(instr_set(b.d_ts + 2 * size_t(b.grid)));
    DJ_HIP(hipMemcpy(out, b.d_ts + 2 * size_t(b.grid), size_t(16) * b.grid * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (clear) DJ_HIP(hipMemset(b.d_ts + 2 * size_t(b.grid), 0, size_t(16) * b.grid * sizeof(uint64_t)));
    return b.grid;
}
#endif

int djtled_batch_stats(const djtled_batch *p, double *inst_ms) {
    if (!p || !inst_ms) return fail(DJ_ERR_ARG, "null argument");
    const Batch &b = *reinterpret_cast<const Batch *>(p);
    std::copy(b.inst_ms.begin(), b.inst_ms.end(), inst_ms);
    return DJ_OK;
}

static int stage(Batch &b, int k) {
    const size_t ts = b.prec == DJ_FP32 ? 4 : 8;
    for (int j = 0; j < 2; j++)
        if (!b.d_stage[k][j]) DJ_HIP(hipMalloc(&b.d_stage[k][j], size_t(3) * b.kc[k]->n_nodes * ts));
    return DJ_OK;
}

int djtled_batch_read(djtled_batch *p, int32_t inst, void *u_cur, void *u_prev, void *stream) {
    if (!p || !u_cur) return fail(DJ_ERR_ARG, "null argument");
    Batch &b = *reinterpret_cast<Batch *>(p);
    if (inst < 0 || inst >= b.n_inst) return fail(DJ_ERR_ARG, "instance out of range");
    DJ_HIP(hipSetDevice(b.device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int k = b.inst_kind[inst], j = b.inst_pos[inst];
    const Ctx &c = *b.kc[k];
    const int rc = stage(b, k);
    if (rc != DJ_OK) return rc;
    BatchDev bd = make_dev(b);
    DJ_HIP(launch_gather_canon(bd.k[k], b.prec, b.cur, b.d_stage[k][0], b.d_stage[k][1], s));
    const size_t ts = b.prec == DJ_FP32 ? 4 : 8;
    const size_t off = size_t(3) * c.inst_node_off[j] * ts, len = size_t(3) * (c.inst_node_off[j + 1] - c.inst_node_off[j]) * ts;
    DJ_HIP(hipMemcpyAsync(u_cur, static_cast<char *>(b.d_stage[k][0]) + off, len, hipMemcpyDeviceToDevice, s));
    if (u_prev)
        DJ_HIP(hipMemcpyAsync(u_prev, static_cast<char *>(b.d_stage[k][1]) + off, len, hipMemcpyDeviceToDevice, s));
    return DJ_OK;
}

int djtled_batch_write(djtled_batch *p, int32_t inst, const void *u_cur, const void *u_prev, void *stream) {
    if (!p || !u_cur) return fail(DJ_ERR_ARG, "null argument");
    Batch &b = *reinterpret_cast<Batch *>(p);
    if (inst < 0 || inst >= b.n_inst) return fail(DJ_ERR_ARG, "instance out of range");
    DJ_HIP(hipSetDevice(b.device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int k = b.inst_kind[inst], j = b.inst_pos[inst];
    const Ctx &c = *b.kc[k];
    const int rc = stage(b, k);
    if (rc != DJ_OK) return rc;
    BatchDev bd = make_dev(b);
    // the kind's whole state goes through the staging arrays
    DJ_HIP(launch_gather_canon(bd.k[k], b.prec, b.cur, b.d_stage[k][0], b.d_stage[k][1], s));
    const size_t ts = b.prec == DJ_FP32 ? 4 : 8;
    const size_t off = size_t(3) * c.inst_node_off[j] * ts, len = size_t(3) * (c.inst_node_off[j + 1] - c.inst_node_off[j]) * ts;
    DJ_HIP(hipMemcpyAsync(static_cast<char *>(b.d_stage[k][0]) + off, u_cur, len, hipMemcpyDeviceToDevice, s));
    DJ_HIP(hipMemcpyAsync(static_cast<char *>(b.d_stage[k][1]) + off, u_prev ? u_prev : u_cur, len,
                          hipMemcpyDeviceToDevice, s));
    DJ_HIP(launch_scatter_state(bd.k[k], b.prec, b.cur, b.d_stage[k][0], b.d_stage[k][1], s));
    return DJ_OK;
}

int djtled_batch_reset(djtled_batch *p, void *stream) {
    if (!p) return fail(DJ_ERR_ARG, "null batch");
    Batch &b = *reinterpret_cast<Batch *>(p);
    DJ_HIP(hipSetDevice(b.device));
    return reset_batch(b, static_cast<hipStream_t>(stream));
}

}  // extern "C"
