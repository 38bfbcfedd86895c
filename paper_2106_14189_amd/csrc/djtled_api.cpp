// C ABI of libdjtled: validation, mesh reordering and partitioning, device
// buffers, and the entry points declared in include/djtled.h.  All numerical
// work of the method runs in the HIP kernels (djtled_kernels.hip); this file
// only builds index structures and moves buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "djtled_internal.h"

using namespace dj;

namespace dj {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

}  // namespace dj

namespace {

template <typename T>
hipError_t dalloc(Ctx &c, T **p, size_t n) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) {
        c.allocs.push_back(q);
        *p = static_cast<T *>(q);
    }
    return e;
}

template <typename T>
hipError_t upload(Ctx &c, T **p, const std::vector<T> &v) {
    hipError_t e = dalloc(c, p, v.size());
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

}  // namespace

namespace dj {

void free_all(Ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (void *p : c->loadsets) {
        LoadSet *ls = static_cast<LoadSet *>(p);
        hipFree(ls->d_flags);
        hipFree(ls->d_ru);
        hipFree(ls->d_rate);
        delete ls;
    }
    for (void *p : c->allocs) hipFree(p);
    for (int b = 0; b < 3; b++) hipFree(c->d_mubuf[b]);
    hipFree(c->d_mpart);
    hipFree(c->d_mred);
    hipFree(c->d_mflags);
    hipFree(c->d_mru);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    if (c->h_status) hipHostFree(c->h_status);
    if (c->h_res) hipHostFree(c->h_res);
    delete c;
}

}  // namespace dj

namespace {

// 21-bit spread for 3-D Morton codes
uint64_t spread3(uint64_t x) {
    x &= 0x1fffffULL;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

struct TempBufs {
    std::vector<void *> v;
    ~TempBufs() {
        for (void *p : v) hipFree(p);
    }
    template <typename T>
    hipError_t up(T **p, const std::vector<T> &h) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(h.size(), 1) * sizeof(T));
        if (e != hipSuccess) return e;
        v.push_back(q);
        *p = static_cast<T *>(q);
        if (!h.empty()) e = hipMemcpy(q, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        return e;
    }
};

}  // namespace

namespace dj {

int build(Ctx &c, const djtled_mesh *mesh, const djtled_material *mat, const djtled_params *prm,
          const MultiInst *mi) {
    const int N = mesh->n_nodes, E = mesh->n_elems, NE = mesh->elem_type;
    const int NI = mi ? mi->n_inst : 1;
    c.n_inst = NI;
    std::vector<int32_t> einst_c(E, 0), ninst_c(N, 0);  // instance of each caller element / node
    if (mi) {
        for (int i = 0; i < NI; i++) {
            for (int e = mi->elem_off[i]; e < mi->elem_off[i + 1]; e++) einst_c[e] = i;
            for (int n = mi->node_off[i]; n < mi->node_off[i + 1]; n++) ninst_c[n] = i;
        }
        c.inst_node_off.assign(mi->node_off, mi->node_off + NI + 1);
        c.inst_elem_off.assign(mi->elem_off, mi->elem_off + NI + 1);
    } else {
        c.inst_node_off = {0, N};
        c.inst_elem_off = {0, E};
    }
    c.n_nodes = N;
    c.n_elems = E;
    c.ne = NE;
    c.model = mat->model;
    c.prec = prm->precision;
    c.form = prm->formulation;
    c.rho = mat->rho;
    c.alpha = prm->alpha;
    c.hg_kappa = mat->hg_kappa < 0 ? 0.1 : mat->hg_kappa;
    // automatic: the fastest variant measured on the 64^3 cubes (FP32 H8: 512
    // threads with one workgroup per compute unit; otherwise variant 0)
    c.variant = prm->variant >= 0 ? prm->variant : (NE == 8 && c.prec == DJ_FP32 ? 2 : 0);
    const Variant var = variants(NE, c.prec)[c.variant];
    c.block = var.block;
    c.ept = var.ept;
    c.mcopy = var.mcopy;
    c.cmax = var.block * var.ept;

    // ---- reorder: elements by the Morton code of their centroid, nodes by first touch
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int n = 0; n < N; n++)
        for (int k = 0; k < 3; k++) {
            lo[k] = std::min(lo[k], mesh->X[3 * n + k]);
            hi[k] = std::max(hi[k], mesh->X[3 * n + k]);
        }
    double span = 0;
    for (int k = 0; k < 3; k++) span = std::max(span, hi[k] - lo[k]);
    if (!(span > 0)) span = 1.0;
    std::vector<uint64_t> code(E);
    for (int e = 0; e < E; e++) {
        double cc[3] = {0, 0, 0};
        for (int a = 0; a < NE; a++)
            for (int k = 0; k < 3; k++) cc[k] += mesh->X[3 * mesh->conn[int64_t(NE) * e + a] + k];
        uint64_t q[3];
        for (int k = 0; k < 3; k++) {
            double t = (cc[k] / NE - lo[k]) / span;
            q[k] = uint64_t(std::min(std::max(t, 0.0), 1.0) * 2097151.0);
        }
        code[e] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    }
    c.elem_perm.resize(E);
    std::iota(c.elem_perm.begin(), c.elem_perm.end(), 0);
    // instances stay contiguous (a chunk then rarely spans two of them)
    std::stable_sort(c.elem_perm.begin(), c.elem_perm.end(), [&](int a, int b) {
        return einst_c[a] != einst_c[b] ? einst_c[a] < einst_c[b] : code[a] < code[b];
    });
    std::vector<int32_t> node_new(N, -1);
    c.node_perm.clear();
    c.node_perm.reserve(N);
    std::vector<int32_t> conn(int64_t(E) * NE);
    for (int e = 0; e < E; e++) {
        const int o = c.elem_perm[e];
        for (int a = 0; a < NE; a++) {
            const int n = mesh->conn[int64_t(NE) * o + a];
            if (node_new[n] < 0) {
                node_new[n] = int32_t(c.node_perm.size());
                c.node_perm.push_back(n);
            }
            conn[int64_t(NE) * e + a] = node_new[n];
        }
    }
    for (int n = 0; n < N; n++)
        if (node_new[n] < 0) {
            node_new[n] = int32_t(c.node_perm.size());
            c.node_perm.push_back(n);
        }

    // ---- node -> element incidence (internal ids, ascending element)
    std::vector<int32_t> deg(N, 0);
    for (int64_t i = 0; i < int64_t(E) * NE; i++) deg[conn[i]]++;
    std::vector<int32_t> ne_off(N + 1, 0);
    for (int n = 0; n < N; n++) ne_off[n + 1] = ne_off[n] + deg[n];
    std::vector<int32_t> ne_list(ne_off[N]);
    {
        std::vector<int32_t> fill(ne_off.begin(), ne_off.end() - 1);
        for (int e = 0; e < E; e++)
            for (int a = 0; a < NE; a++) ne_list[fill[conn[int64_t(NE) * e + a]]++] = e;
    }
    for (int e = 0; e < E; e++)
        for (int a = 0; a < NE; a++)
            for (int b = a + 1; b < NE; b++)
                if (conn[int64_t(NE) * e + a] == conn[int64_t(NE) * e + b])
                    return fail(DJ_ERR_BAD_MESH, "element " + std::to_string(c.elem_perm[e]) + " repeats a node");

    // ---- grid size from occupancy, then balanced chunks
    int bpc = 0;
    size_t lds = 0;
    DJ_HIP(occupancy(NE, c.model, c.form, c.prec, c.variant, &bpc, &lds));
    hipDeviceProp_t prop;
    DJ_HIP(hipGetDeviceProperties(&prop, c.device));
    if (bpc < 1) return fail(DJ_ERR_UNSUPPORTED, "kernel variant does not fit on a compute unit");
    const int gmax = bpc * prop.multiProcessorCount;
    int C = c.cmax;
    if (prm->chunk_elems > 0) C = std::min(prm->chunk_elems, c.cmax);
    else C = std::min(c.cmax, std::max(64, (E + gmax - 1) / gmax));

    // ---- chunks, node copies, local CSR, shared-node partial groups.  A chunk
    // may hold at most mcopy * block node copies; larger meshes per chunk are
    // re-partitioned with smaller chunks.
    int64_t nch = 0;
    std::vector<ChunkDesc> chunks;
    std::vector<uint32_t> crange;
    std::vector<uint16_t> wpos;  // NE planes over elements, stride estride
    const int64_t estride = (int64_t(E) + 63) / 64 * 64;
    std::vector<uint32_t> flags;
    std::vector<int32_t> copy_node;  // internal node id of each copy
    std::vector<int32_t> local_of(N, -1), in_chunk(N, 0);
    std::vector<std::vector<int32_t>> node_copies(N);
    int max_copies = 0;
    for (int attempt = 0;; attempt++) {
    const bool in_batch = mi && mi->batch;
    nch = (E + C - 1) / C;
    if (nch > gmax && !in_batch) nch = (nch + gmax - 1) / gmax * gmax;  // whole rounds of the resident grid
    if (nch > E) nch = E;
    c.chunk_elems = int((E + nch - 1) / nch);
    c.grid = int(std::min<int64_t>(nch, gmax));
    // (a workgroup with more than KMAX chunks reads its chunk list in windows)
    chunks.assign(nch, ChunkDesc{});
    crange.clear();
    wpos.assign(size_t(NE) * estride, 0);
    flags.clear();
    copy_node.clear();
    for (auto &v : node_copies) v.clear();
    max_copies = 0;
    for (int64_t ch = 0; ch < nch; ch++) {
        const int eb = int(ch * E / nch), ee = int((ch + 1) * E / nch);
        if (ee - eb > c.cmax) return fail(DJ_ERR_ARG, "internal: chunk exceeds capacity");
        std::vector<int32_t> touched;
        for (int e = eb; e < ee; e++)
            for (int a = 0; a < NE; a++) {
                const int n = conn[int64_t(NE) * e + a];
                if (in_chunk[n]++ == 0) touched.push_back(n);
            }
        std::vector<int32_t> interior, shared;
        for (int n : touched) (in_chunk[n] == deg[n] ? interior : shared).push_back(n);
        ChunkDesc d{};
        d.elem_begin = eb;
        d.elem_count = ee - eb;
        d.copy_begin = int32_t(copy_node.size());
        d.copy_count = int32_t(touched.size());
        d.n_interior = int32_t(interior.size());
        chunks[ch] = d;
        max_copies = std::max(max_copies, d.copy_count);
        std::vector<int32_t> order(interior);
        order.insert(order.end(), shared.begin(), shared.end());
        for (size_t i = 0; i < order.size(); i++) local_of[order[i]] = int32_t(i);
        // incidences numbered in copy order, (element, node) order within a copy
        std::vector<int32_t> cnt(order.size(), 0);
        for (int e = eb; e < ee; e++)
            for (int a = 0; a < NE; a++) cnt[local_of[conn[int64_t(NE) * e + a]]]++;
        std::vector<int32_t> pos(order.size());
        int32_t acc = 0;
        // ranges start an odd distance apart (a padding slot after an even
        // count): a wave's copies then walk their ranges on distinct LDS banks;
        // at most one padding slot per copy, which the kernels' slot planes hold
        for (size_t i = 0; i < order.size(); i++) {
            pos[i] = acc;
            crange.push_back(uint32_t(acc) | (uint32_t(cnt[i]) << 16));
            acc += cnt[i] + ((cnt[i] & 1) ? 0 : 1);
        }
        for (int e = eb; e < ee; e++)
            for (int a = 0; a < NE; a++) {
                const int li = local_of[conn[int64_t(NE) * e + a]];
                wpos[size_t(a) * estride + e] = uint16_t(pos[li]++);
            }
        for (size_t i = 0; i < order.size(); i++) {
            const int n = order[i];
            const int l = int32_t(copy_node.size());
            copy_node.push_back(n);
            flags.push_back(i >= interior.size() ? FLAG_SHARED : 0u);
            node_copies[n].push_back(l);
        }
        for (int n : touched) {
            in_chunk[n] = 0;
            local_of[n] = -1;
        }
    }
    if (max_copies <= c.mcopy * c.block) break;
    if (attempt >= 12 || C <= 8)
        return fail(DJ_ERR_UNSUPPORTED, "a chunk touches " + std::to_string(max_copies) +
                                            " nodes, above the kernel's per-chunk capacity");
    C = std::max(8, int(double(C) * 0.9 * c.mcopy * c.block / max_copies));
    }
    const int64_t L = copy_node.size();
    if (L >= (int64_t(1) << 31))
        return fail(DJ_ERR_UNSUPPORTED, "mesh too large for 32-bit copy indices");
    // shared nodes: copies of one node form a contiguous partial group, in ascending chunk order
    std::vector<int32_t> pidx(L, 0), cnode(L);
    int32_t n_part = 0;
    for (int n = 0; n < N; n++) {
        const auto &cp = node_copies[n];
        if (cp.empty()) continue;
        flags[cp[0]] |= FLAG_CANON;
        if (cp.size() > 1) {
            if (cp.size() > 255) return fail(DJ_ERR_UNSUPPORTED, "node shared by more than 255 chunks");
            for (size_t j = 0; j < cp.size(); j++) {
                pidx[cp[j]] = n_part;
                flags[cp[j]] |= (uint32_t(cp.size()) << FLAG_NCOPY_SHIFT) | (uint32_t(j) << FLAG_RANK_SHIFT);
            }
            n_part += int32_t(cp.size());
        }
    }
    for (int64_t l = 0; l < L; l++) cnode[l] = c.node_perm[copy_node[l]];
    c.n_shared_copies = n_part;
    c.h_flags = flags;
    c.h_copy_node = copy_node;
    c.h_chunk_elem.resize(2 * size_t(nch));
    for (int64_t ch = 0; ch < nch; ch++) {
        c.h_chunk_elem[2 * ch] = chunks[ch].elem_begin;
        c.h_chunk_elem[2 * ch + 1] = chunks[ch].elem_count;
    }

    // ---- device buffers
    const size_t ts = c.prec == DJ_FP32 ? 4 : 8;
    const int NP = n_planes(NE, c.model);
    c.topo.estride = estride;
    c.topo.n_chunks = int32_t(nch);
    c.topo.n_copies = int32_t(L);
    c.topo.n_part = n_part;
    c.topo.cmax = c.cmax;
    ChunkDesc *d_chunks;
    int32_t *d_pidx, *d_cnode;
    uint32_t *d_crange;
    uint16_t *d_wpos;
    uint32_t *d_flags;
    DJ_HIP(upload(c, &d_chunks, chunks));
    DJ_HIP(upload(c, &d_crange, crange));
    DJ_HIP(upload(c, &d_wpos, wpos));
    DJ_HIP(upload(c, &d_flags, flags));
    DJ_HIP(upload(c, &d_pidx, pidx));
    DJ_HIP(upload(c, &d_cnode, cnode));
    DJ_HIP(upload(c, &c.d_inode, copy_node));
    DJ_HIP(upload(c, &c.d_elem_perm, c.elem_perm));
    DJ_HIP(upload(c, &c.d_node_perm, c.node_perm));
    c.topo.chunks = d_chunks;
    c.topo.crange = d_crange;
    c.topo.wpos = d_wpos;
    c.topo.flags = d_flags;
    c.topo.pidx = d_pidx;
    c.topo.cnode = d_cnode;
    unsigned char *p;
    DJ_HIP(dalloc(c, &p, size_t(NP) * c.topo.estride * ts));
    c.d_elem = p;
    DJ_HIP(hipMemset(c.d_elem, 0, size_t(NP) * c.topo.estride * ts));
    c.topo.elem = c.d_elem;
    DJ_HIP(dalloc(c, &p, L * ts));
    c.d_acoef = p;
    c.topo.acoef = c.d_acoef;
    for (int b = 0; b < 3; b++) {
        DJ_HIP(dalloc(c, &p, 3 * L * ts));
        c.d_ubuf[b] = p;
    }
    DJ_HIP(dalloc(c, &p, 6 * size_t(std::max(n_part, 1)) * ts));  // 2 parities x 3 planes
    c.d_part = p;
    DJ_HIP(dalloc(c, &c.d_bar, size_t(c.grid + 16) * 32));  // barrier flags, one 128-B line each
    DJ_HIP(dalloc(c, &c.d_status, 8));
    DJ_HIP(dalloc(c, &c.d_red, size_t(4) * c.grid + 2));
    DJ_HIP(hipMemset(c.d_bar, 0, size_t(c.grid + 16) * 32 * sizeof(uint32_t)));
    DJ_HIP(dalloc(c, &c.d_V64, E));
    DJ_HIP(dalloc(c, &c.d_jinv64, size_t(9) * E));
    DJ_HIP(dalloc(c, &c.d_mass64, N));
    DJ_HIP(hipHostMalloc(reinterpret_cast<void **>(&c.h_status), 8 * sizeof(int32_t), hipHostMallocDefault));
    DJ_HIP(hipHostMalloc(reinterpret_cast<void **>(&c.h_res), sizeof(double), hipHostMallocDefault));
    DJ_HIP(hipEventCreate(&c.ev0));
    DJ_HIP(hipEventCreate(&c.ev1));

    // ---- per-element inputs in internal order; pre-computation on the GPU (FP64)
    std::vector<double> Xi(size_t(3) * N), Ei(E), nui(E), etai, fibi, etabi, fibbi, c01i;
    for (int n = 0; n < N; n++)
        for (int k = 0; k < 3; k++) Xi[3 * size_t(n) + k] = mesh->X[3 * size_t(c.node_perm[n]) + k];
    for (int e = 0; e < E; e++) {
        const int o = c.elem_perm[e];
        Ei[e] = mat->E ? mat->E[o] : mat->E_uniform;
        nui[e] = mat->nu ? mat->nu[o] : mat->nu_uniform;
        if (!(Ei[e] > 0) || !(nui[e] > -1.0 && nui[e] < 0.5))
            return fail(DJ_ERR_ARG, "element " + std::to_string(o) + ": need E > 0 and -1 < nu < 0.5");
    }
    // per-element copies in internal order, with the uniform fallbacks
    auto gather = [&](const double *arr, double uni, std::vector<double> &out) {
        out.resize(E);
        for (int e = 0; e < E; e++) out[e] = arr ? arr[c.elem_perm[e]] : uni;
    };
    auto gather3 = [&](const double *arr, std::vector<double> &out) {
        out.resize(size_t(3) * E);
        for (int e = 0; e < E; e++)
            for (int k = 0; k < 3; k++) out[3 * size_t(e) + k] = arr[3 * size_t(c.elem_perm[e]) + k];
    };
    const bool fib_a = c.model == DJ_TI || c.model == DJ_OT, fib_b = c.model == DJ_OT;
    if (fib_a) {
        gather(mat->eta_ratio, mat->eta_ratio_uniform, etai);
        gather3(mat->fibre, fibi);
    }
    if (fib_b) {
        gather(mat->eta_b_ratio, mat->eta_b_ratio_uniform, etabi);
        gather3(mat->fibre_b, fibbi);
    }
    if (c.model == DJ_MR) gather(mat->c01, mat->c01_uniform, c01i);
    for (int e = 0; e < E; e++) {
        const bool okm = (!fib_a || etai[e] >= 0) && (!fib_b || etabi[e] >= 0) && (c.model != DJ_MR || c01i[e] >= 0);
        if (!okm) return fail(DJ_ERR_ARG, "element " + std::to_string(c.elem_perm[e]) + ": negative fibre or C01 modulus");
    }
    {
        std::vector<double> kap(E);
        for (int e = 0; e < E; e++) kap[e] = Ei[e] / (3.0 * (1.0 - 2.0 * nui[e]));
        DJ_HIP(upload(c, &c.d_kappa64, kap));
    }
    TempBufs tb;
    double *dX, *dE, *dnu, *ddt;
    int32_t *dconn, *dbad, *dneoff, *dnelist;
    MatDev md{};
    DJ_HIP(tb.up(&dX, Xi));
    DJ_HIP(upload(c, &dconn, conn));  // kept (element nodes, internal ids)
    c.d_enode = dconn;
    DJ_HIP(tb.up(&dE, Ei));
    DJ_HIP(tb.up(&dnu, nui));
    md.E = dE;
    md.nu = dnu;
    double *tmp = nullptr;
    if (fib_a) {
        DJ_HIP(tb.up(&tmp, etai));
        md.eta = tmp;
        DJ_HIP(tb.up(&tmp, fibi));
        md.fib = tmp;
    }
    if (fib_b) {
        DJ_HIP(tb.up(&tmp, etabi));
        md.etab = tmp;
        DJ_HIP(tb.up(&tmp, fibbi));
        md.fibb = tmp;
    }
    if (c.model == DJ_MR) {
        DJ_HIP(tb.up(&tmp, c01i));
        md.c01 = tmp;
    }
    const double inf = std::numeric_limits<double>::infinity();
    int32_t *dei = nullptr;
    if (NI > 1) {
        std::vector<int32_t> ei(E);
        for (int e = 0; e < E; e++) ei[e] = einst_c[c.elem_perm[e]];
        DJ_HIP(tb.up(&dei, ei));
    }
    DJ_HIP(tb.up(&ddt, std::vector<double>(NI, inf)));
    DJ_HIP(tb.up(&dbad, std::vector<int32_t>{0}));
    DJ_HIP(upload(c, &dneoff, ne_off));  // kept: the average-nodal-pressure forces use them
    DJ_HIP(upload(c, &dnelist, ne_list));
    c.d_ne_off = dneoff;
    c.d_ne_list = dnelist;
    DJ_HIP(launch_precompute(c, dX, dconn, md, dei, ddt, dbad, nullptr));
    int32_t bad = 0;
    std::vector<double> dtc(NI);
    DJ_HIP(hipMemcpy(&bad, dbad, sizeof(int32_t), hipMemcpyDeviceToHost));
    DJ_HIP(hipMemcpy(dtc.data(), ddt, NI * sizeof(double), hipMemcpyDeviceToHost));
    if (bad) return fail(DJ_ERR_BAD_MESH, std::to_string(bad) + " element(s) with det(0J) <= 0 or zero fibre");
    if (c.prec == DJ_FP32) {
        // the register path of the FP32 kernels reads the interleaved copy (16-byte loads)
        DJ_HIP(dalloc(c, &p, size_t(NP + NE / 2) * c.topo.estride * 4));
        DJ_HIP(launch_pack_elem4(c, p, nullptr));
        DJ_HIP(hipDeviceSynchronize());
        c.topo.elem4 = p;
    }
    const double fac = prm->dt_factor > 0 ? prm->dt_factor : 0.9;
    c.inst_dt.resize(NI);
    c.inst_dt_crit = dtc;
    c.inst_alpha.assign(NI, prm->alpha);
    for (int i = 0; i < NI; i++) {
        if (!(dtc[i] < inf)) return fail(DJ_ERR_BAD_MESH, "instance " + std::to_string(i) + " has no elements");
        if (mi && mi->alpha) c.inst_alpha[i] = mi->alpha[i];
        c.inst_dt[i] = prm->dt > 0 ? prm->dt : fac * dtc[i];
        if (c.inst_dt[i] > dtc[i] && !prm->allow_unstable_dt)
            return fail(DJ_ERR_UNSTABLE_DT, "dt " + std::to_string(c.inst_dt[i]) + " exceeds the critical step " +
                                                std::to_string(dtc[i]) + (NI > 1 ? " of instance " + std::to_string(i) : ""));
    }
    c.dt_crit = *std::min_element(dtc.begin(), dtc.end());
    c.dt = c.inst_dt[0];
    double *dc2 = nullptr, *dbpn = nullptr;
    if (NI > 1 || (mi && mi->batch)) {  // the batch kernel always reads B' per copy
        // per-node coefficients of the node's instance; B' per copy
        std::vector<double> c2n(N), bpn(N);
        for (int n = 0; n < N; n++) {
            const int i = ninst_c[c.node_perm[n]];
            const double dt = c.inst_dt[i], al = c.inst_alpha[i];
            c2n[n] = 2.0 * dt * dt / (2.0 + al * dt);
            bpn[n] = (2.0 - al * dt) / (2.0 + al * dt);
        }
        DJ_HIP(tb.up(&dc2, c2n));
        DJ_HIP(tb.up(&dbpn, bpn));
        unsigned char *pb;
        DJ_HIP(dalloc(c, &pb, size_t(L) * ts));
        c.d_bpc = pb;
        c.topo.bpc = pb;
    }
    DJ_HIP(launch_mass_acoef(c, dneoff, dnelist, dc2, dbpn, nullptr));
    if (c.form == DJ_FORM_NODAL_PRESSURE) {
        unsigned char *q;
        DJ_HIP(dalloc(c, &q, size_t(L) * ts));
        c.d_anps_c = q;
        DJ_HIP(dalloc(c, &q, size_t(L) * ts));
        c.d_anps_p = q;
        DJ_HIP(hipMemset(c.d_anps_p, 0, size_t(L) * ts));
        DJ_HIP(dalloc(c, &q, size_t(std::max(c.topo.n_part, 1)) * ts));
        c.d_anps_j = q;
        DJ_HIP(launch_anps_setup(c, nullptr));
    }
    std::vector<double> m(N);
    DJ_HIP(hipMemcpy(m.data(), c.d_mass64, N * sizeof(double), hipMemcpyDeviceToHost));
    c.mass_total = std::accumulate(m.begin(), m.end(), 0.0);
    DJ_HIP(hipDeviceSynchronize());

    // ---- traffic model of one fused step: bytes that must cross HBM once per step
    //   elements : NP planes + NE incidence positions (uint16)
    //   interior copies : slot range, flags, u^n, u^{n-1}, A (read), u^{n+1} (write)
    //   shared copies   : slot range, flags, partial index, u^n (element phase);
    //                     partial write (3 values); then flags, partial
    //                     index, A, u^n, u^{n-1}, the node's cnt slots (read) and
    //                     u^{n+1} (write)
    double eb = double(NP) * ts + 2.0 * NE;
    double interior = 0, shared = 0;
    for (int64_t l = 0; l < L; l++) {
        if (flags[l] & FLAG_SHARED) {
            const int k = (flags[l] >> FLAG_NCOPY_SHIFT) & 255;
            shared += (4 + 4 + 4 + 3 * ts) + 3 * ts + (4 + 4 + ts + 6 * ts + k * 3.0 * ts + 3 * ts);
        } else {
            interior += 4 + 4 + 6 * ts + ts + 3 * ts;
        }
    }
    c.bytes_per_step = eb * E + interior + shared + double(nch) * sizeof(ChunkDesc);
    if (c.form == DJ_FORM_NODAL_PRESSURE) {
        // the J pass: element data again; per copy slot range, flags, u^n, and
        // c_n + p_n (interior) or the J partial (shared); the shared copies'
        // flags, partial index, group of J partials, c_n and p_n; the force
        // pass reads p_n of every copy
        double jp = eb * E;
        for (int64_t l = 0; l < L; l++) {
            if (flags[l] & FLAG_SHARED) {
                const int k = (flags[l] >> FLAG_NCOPY_SHIFT) & 255;
                jp += (4 + 4 + 4 + 3 * ts) + ts + (4 + 4 + k * ts + 2 * ts) + ts;
            } else {
                jp += 4 + 4 + 3 * ts + 2 * ts + ts;
            }
        }
        c.bytes_per_step += jp + double(nch) * sizeof(ChunkDesc);
    }
    c.elem_bytes = eb;
    return DJ_OK;
}

// node_rate (batches): per caller node, the signed ramp rate of its instance
// (see ramp_rate in the kernels); null for a single instance.
int make_loadset(Ctx &c, const djtled_loads *ld, const double *node_rate, LoadSet **out) {
    *out = nullptr;
    if (ld->n_bc < 0 || (ld->n_bc > 0 && (!ld->bc_node || !ld->bc_mask || !ld->bc_target)))
        return fail(DJ_ERR_ARG, "bad boundary-condition arrays");
    if (ld->ramp < DJ_RAMP_NONE || ld->ramp > DJ_RAMP_SMOOTH || !(ld->t_ramp >= 0))
        return fail(DJ_ERR_ARG, "bad ramp");
    std::vector<int32_t> bc_of(c.n_nodes, -1);
    for (int j = 0; j < ld->n_bc; j++) {
        const int n = ld->bc_node[j];
        if (n < 0 || n >= c.n_nodes) return fail(DJ_ERR_ARG, "boundary-condition node out of range");
        if (ld->bc_mask[j] & ~7) return fail(DJ_ERR_ARG, "boundary-condition mask must be within 0..7");
        bc_of[n] = j;
    }
    const int64_t L = c.topo.n_copies;
    std::vector<uint32_t> fl(c.h_flags);
    std::vector<double> ru(3 * L, 0.0), rate(node_rate ? L : 0, 0.0);
    for (int64_t l = 0; l < L; l++) {
        const int n = c.node_perm[c.h_copy_node[l]];
        const int j = bc_of[n];
        const uint32_t mask = j >= 0 ? uint32_t(ld->bc_mask[j]) : 0u;
        if (mask == 0 && !ld->R) continue;
        fl[l] |= mask | FLAG_RU;
        if (node_rate) rate[l] = node_rate[n];
        for (int k = 0; k < 3; k++)
            ru[k * L + l] = ((mask >> k) & 1u) ? ld->bc_target[3 * j + k] : (ld->R ? ld->R[3 * size_t(n) + k] : 0.0);
    }
    LoadSet *ls = new LoadSet();
    ls->ctx = &c;
    ls->ramp = ld->ramp;
    ls->t_ramp = ld->t_ramp;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&ls->d_flags), L * sizeof(uint32_t));
    const size_t ts = c.prec == DJ_FP32 ? 4 : 8;
    if (e == hipSuccess) e = hipMalloc(&ls->d_ru, 3 * L * ts);
    if (e == hipSuccess) e = hipMemcpy(ls->d_flags, fl.data(), L * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && node_rate) e = hipMalloc(&ls->d_rate, L * ts);
    auto put = [&](void *dst, const std::vector<double> &v) {
        if (c.prec == DJ_FP32) {
            std::vector<float> rf(v.begin(), v.end());
            return hipMemcpy(dst, rf.data(), rf.size() * 4, hipMemcpyHostToDevice);
        }
        return hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    };
    if (e == hipSuccess) e = put(ls->d_ru, ru);
    if (e == hipSuccess && node_rate) e = put(ls->d_rate, rate);
    if (e != hipSuccess) {
        hipFree(ls->d_flags);
        hipFree(ls->d_ru);
        hipFree(ls->d_rate);
        delete ls;
        return fail(DJ_ERR_HIP, std::string("loadset upload: ") + hipGetErrorString(e));
    }
    c.loadsets.push_back(ls);
    *out = ls;
    return DJ_OK;
}

}  // namespace dj

namespace dj {

// n_steps explicit steps of nrhs load cases (one persistent launch); see
// djtled_step and djtled_step_multi.  st->u_cur / u_prev: nrhs x n_nodes x 3.
int step_cases(djtled_ctx *ctx, int nrhs, djtled_state *st, const djtled_loadset *const *lsp, int32_t n_steps,
               const djtled_step_opts *opts, djtled_status *out, double *residuals, int32_t *error_case,
               void *stream) {
    if (!ctx || !st || !st->u_cur || !st->u_prev) return fail(DJ_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > MAX_RHS) return fail(DJ_ERR_ARG, "nrhs must be 1.." + std::to_string(MAX_RHS));
    if (n_steps < 0) return fail(DJ_ERR_ARG, "n_steps must be >= 0");
    if (st->u_cur == st->u_prev) return fail(DJ_ERR_ARG, "u_cur and u_prev must be distinct arrays");
    Ctx &c = *reinterpret_cast<Ctx *>(ctx);
    if (c.n_inst > 1) return fail(DJ_ERR_ARG, "batch contexts step through djtled_batch_run");
    if (nrhs > 1 && (c.prec != DJ_FP32 || c.form != DJ_FORM_JACOBIAN || c.variant >= 4))
        return fail(DJ_ERR_UNSUPPORTED, "several load cases per launch: FP32, Jacobian form, variants 0..3");
    if (nrhs > 1 && (c.topo.n_chunks + c.grid - 1) / c.grid > KMAX)
        return fail(DJ_ERR_UNSUPPORTED, "several load cases per launch: at most " + std::to_string(KMAX) +
                                            " chunks per workgroup");
    // load sets: all absent, or one per case with a common ramp
    const bool has_loads = lsp && lsp[0];
    for (int r = 0; r < nrhs; r++) {
        const LoadSet *ls = lsp ? reinterpret_cast<const LoadSet *>(lsp[r]) : nullptr;
        if (bool(ls) != has_loads) return fail(DJ_ERR_ARG, "give a load set for every case or for none");
        if (!ls) continue;
        if (ls->ctx != &c) return fail(DJ_ERR_ARG, "load set belongs to another context");
        const LoadSet *l0 = reinterpret_cast<const LoadSet *>(lsp[0]);
        if (ls->ramp != l0->ramp || ls->t_ramp != l0->t_ramp)
            return fail(DJ_ERR_ARG, "the load cases of one call must share the ramp kind and duration");
    }
    djtled_step_opts def{DJ_MODE_FIXED, 0.0, 1};
    const djtled_step_opts &o = opts ? *opts : def;
    if (o.mode != DJ_MODE_FIXED && o.mode != DJ_MODE_RELAX) return fail(DJ_ERR_ARG, "bad mode");
    if (o.mode == DJ_MODE_RELAX && o.check_every < 1) return fail(DJ_ERR_ARG, "check_every must be >= 1");
    DJ_HIP(hipSetDevice(c.device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t ts = c.prec == DJ_FP32 ? sizeof(float) : sizeof(double);
    const size_t L = size_t(c.topo.n_copies);
    if (nrhs > 1) {  // the several-cases kernel's grid must be co-resident like the single-case one's
        int bpc = 0, ncu = 0;
        DJ_HIP(occupancy_multi(c, &bpc));
        DJ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device));
        if (int64_t(bpc) * ncu < c.grid)
            return fail(DJ_ERR_UNSUPPORTED, "the several-cases kernel does not fit this context's grid");
    }
    StepArgs a;
    a.nrhs = nrhs;
    const LoadSet *l0 = has_loads ? reinterpret_cast<const LoadSet *>(lsp[0]) : nullptr;
    a.ramp = l0 ? l0->ramp : DJ_RAMP_NONE;
    a.t_ramp = l0 ? l0->t_ramp : 0.0;
    a.anp_c = c.d_anps_c;
    a.anp_p = c.d_anps_p;
    a.anp_jpart = c.d_anps_j;
    if (nrhs == 1) {
        for (int b = 0; b < 3; b++) a.ubuf[b] = c.d_ubuf[b];
        a.part = c.d_part;
        a.red = c.d_red;
        a.res_out = c.d_red + size_t(4) * c.grid;
        a.flags = l0 ? l0->d_flags : c.topo.flags;
        a.ru = l0 ? l0->d_ru : nullptr;
    } else {
        if (c.rhs_cap < nrhs) {  // grow the case buffers (no launch of this context is in flight)
            DJ_HIP(hipStreamSynchronize(s));
            for (int b = 0; b < 3; b++) {
                hipFree(c.d_mubuf[b]);
                c.d_mubuf[b] = nullptr;
            }
            hipFree(c.d_mpart);
            hipFree(c.d_mred);
            hipFree(c.d_mflags);
            hipFree(c.d_mru);
            c.d_mpart = c.d_mru = nullptr;
            c.d_mred = nullptr;
            c.d_mflags = nullptr;
            c.rhs_cap = 0;
            const size_t NP = size_t(std::max<int64_t>(c.topo.n_part, 1));
            for (int b = 0; b < 3; b++) DJ_HIP(hipMalloc(&c.d_mubuf[b], size_t(nrhs) * 3 * L * ts));
            DJ_HIP(hipMalloc(&c.d_mpart, size_t(nrhs) * 6 * NP * ts));
            DJ_HIP(hipMalloc(reinterpret_cast<void **>(&c.d_mred), (size_t(4) * c.grid + 1) * nrhs * sizeof(double)));
            DJ_HIP(hipMalloc(reinterpret_cast<void **>(&c.d_mflags), size_t(nrhs) * L * sizeof(uint32_t)));
            DJ_HIP(hipMalloc(&c.d_mru, size_t(nrhs) * 3 * L * ts));
            c.rhs_cap = nrhs;
        }
        for (int b = 0; b < 3; b++) a.ubuf[b] = c.d_mubuf[b];
        a.part = c.d_mpart;
        a.red = c.d_mred;
        a.res_out = c.d_mred + size_t(4) * c.grid * nrhs;
        // gather the cases' flags and load values into consecutive planes
        for (int r = 0; r < nrhs; r++) {
            const LoadSet *ls = has_loads ? reinterpret_cast<const LoadSet *>(lsp[r]) : nullptr;
            DJ_HIP(hipMemcpyAsync(c.d_mflags + r * L, ls ? ls->d_flags : c.topo.flags, L * sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, s));
            // (a load set without load values flags no copy for them: its planes are never read)
            if (has_loads && ls->d_ru)
                DJ_HIP(hipMemcpyAsync(static_cast<char *>(c.d_mru) + r * 3 * L * ts, ls->d_ru, 3 * L * ts,
                                      hipMemcpyDeviceToDevice, s));
        }
        a.flags = c.d_mflags;
        a.ru = has_loads ? c.d_mru : nullptr;
    }
    a.u_out_cur = st->u_cur;
    a.u_out_prev = st->u_prev;
    a.out_stride = int64_t(3) * c.n_nodes;
    a.dt = c.dt;
    a.bprime = (2.0 - c.alpha * c.dt) / (2.0 + c.alpha * c.dt);
    a.step0 = st->step;
    a.n_steps = n_steps;
    a.relax = o.mode == DJ_MODE_RELAX;
    a.tol = o.tol;
    a.check_every = std::max(1, o.check_every);
    a.cur0 = 0;
    a.bar = c.d_bar;
    a.status = c.d_status;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::vector<double> hres(nrhs, nan);
    DJ_HIP(hipMemcpyAsync(a.res_out, hres.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    DJ_HIP(launch_step(c, a, st->u_cur, st->u_prev, s, c.ev0, c.ev1));
    DJ_HIP(hipMemcpyAsync(c.h_status, c.d_status, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DJ_HIP(hipMemcpyAsync(hres.data(), a.res_out, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    DJ_HIP(hipStreamSynchronize(s));
    djtled_status r;
    r.code = c.h_status[4] ? DJ_ERR_BARRIER : c.h_status[0];
    // an error of the last step's shared-node phase is left in a parity word
    // (that step counts as done; the returned state holds the bad value)
    if (r.code == DJ_OK) r.code = c.h_status[5] != 0 ? c.h_status[5] : c.h_status[6];
    r.steps_done = c.h_status[1];
    r.error_step = -1;
    r.error_elem = -1;
    r.residual = hres[0];
    for (int q = 1; q < nrhs; q++)  // the largest (NaN if any is)
        if (!(r.residual >= hres[q])) r.residual = hres[q];
    float ms = 0.0f;
    r.kernel_ms = hipEventElapsedTime(&ms, c.ev0, c.ev1) == hipSuccess ? double(ms) : -1.0;
    if (error_case) *error_case = -1;
    if (r.code == DJ_ERR_BARRIER) {
        r.steps_done = 0;
        g_err = "persistent kernel grid barrier timed out";
    } else if (r.code == DJ_ERR_INVERTED || r.code == DJ_ERR_NONFINITE) {
        r.error_step = st->step + c.h_status[3];
        const int ie = c.h_status[2];
        r.error_elem = (ie >= 0 && ie < c.n_elems) ? c.elem_perm[ie] : -1;
        if (error_case) *error_case = c.h_status[7];
        g_err = (r.code == DJ_ERR_INVERTED ? "element inverted (J <= 0) at step " : "non-finite value at step ") +
                std::to_string(r.error_step) + (nrhs > 1 ? " in load case " + std::to_string(c.h_status[7]) : "");
    }
    st->step += r.steps_done;
    if (residuals)
        for (int q = 0; q < nrhs; q++) residuals[q] = hres[q];
    if (out) *out = r;
    return r.code;
}

}  // namespace dj

extern "C" {

const char *djtled_last_error(void) { return g_err.c_str(); }

int djtled_precompute(const djtled_mesh *mesh, const djtled_material *mat, const djtled_params *prm,
                      djtled_ctx **out) {
    g_err.clear();
    if (!mesh || !mat || !prm || !out) return fail(DJ_ERR_ARG, "null argument");
    *out = nullptr;
    if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || !mesh->X || !mesh->conn)
        return fail(DJ_ERR_ARG, "empty mesh or null arrays");
    if (mesh->elem_type != DJ_T4 && mesh->elem_type != DJ_H8) return fail(DJ_ERR_UNSUPPORTED, "elem_type must be 4 or 8");
    if (mat->model < DJ_NH || mat->model > DJ_MR) return fail(DJ_ERR_UNSUPPORTED, "model must be DJ_NH, DJ_TI, DJ_OT or DJ_MR");
    if (prm->precision != DJ_FP32 && prm->precision != DJ_FP64) return fail(DJ_ERR_UNSUPPORTED, "precision");
    if (!(mat->rho > 0)) return fail(DJ_ERR_ARG, "rho must be > 0");
    if ((mat->model == DJ_TI || mat->model == DJ_OT) && !mat->fibre)
        return fail(DJ_ERR_ARG, "DJ_TI and DJ_OT need fibre directions");
    if (mat->model == DJ_OT && !mat->fibre_b) return fail(DJ_ERR_ARG, "DJ_OT needs second fibre directions");
    if ((mat->model == DJ_OT || mat->model == DJ_MR) && prm->variant >= 4)
        return fail(DJ_ERR_UNSUPPORTED, "variants 4 and 5 are built for DJ_NH and DJ_TI only");
    if (prm->formulation != DJ_FORM_JACOBIAN && prm->formulation != DJ_FORM_CLASSICAL &&
        prm->formulation != DJ_FORM_NODAL_PRESSURE)
        return fail(DJ_ERR_ARG, "formulation must be DJ_FORM_JACOBIAN, DJ_FORM_CLASSICAL or DJ_FORM_NODAL_PRESSURE");
    if (prm->formulation == DJ_FORM_NODAL_PRESSURE && ((mat->model != DJ_NH && mat->model != DJ_TI) || prm->variant >= 4))
        return fail(DJ_ERR_UNSUPPORTED, "the average-nodal-pressure form: DJ_NH / DJ_TI, variants 0..3");
    if (prm->formulation == DJ_FORM_CLASSICAL && (prm->precision != DJ_FP32 || prm->variant >= 4))
        return fail(DJ_ERR_UNSUPPORTED, "the classical TLED form is built for FP32 and variants 0..3");
    if (!(prm->alpha >= 0) || !(prm->dt >= 0)) return fail(DJ_ERR_ARG, "alpha and dt must be >= 0");
    if (prm->variant < -1 || prm->variant >= int(variants(mesh->elem_type, prm->precision).size()))
        return fail(DJ_ERR_ARG, "unknown kernel variant");
    if (prm->chunk_elems < 0) return fail(DJ_ERR_ARG, "chunk_elems must be >= 0");
    const int64_t nconn = int64_t(mesh->n_elems) * mesh->elem_type;
    for (int64_t i = 0; i < nconn; i++)
        if (mesh->conn[i] < 0 || mesh->conn[i] >= mesh->n_nodes)
            return fail(DJ_ERR_BAD_MESH, "node index out of range in element " + std::to_string(i / mesh->elem_type));
    for (int64_t i = 0; i < 3 * int64_t(mesh->n_nodes); i++)
        if (!std::isfinite(mesh->X[i])) return fail(DJ_ERR_BAD_MESH, "non-finite coordinate");
    Ctx *c = new Ctx();
    int dev = prm->device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    }
    c->device = dev;
    if (hipSetDevice(dev) != hipSuccess) {
        delete c;
        return fail(DJ_ERR_HIP, "hipSetDevice failed");
    }
    int rc = build(*c, mesh, mat, prm);
    // set-up of the allocation-free entry point on this GPU (once per device):
    // the device address of its fixed scratch array
    void *scr = nullptr;
    if (rc == DJ_OK && noalloc_scratch(dev, &scr) != hipSuccess)
        rc = fail(DJ_ERR_HIP, "hipGetSymbolAddress of the fixed scratch array failed");
    if (rc != DJ_OK) {
        std::string msg = g_err;
        free_all(c);
        g_err = msg;
        return rc;
    }
    *out = reinterpret_cast<djtled_ctx *>(c);
    return DJ_OK;
}

int djtled_destroy(djtled_ctx *ctx) {
    if (!ctx) return fail(DJ_ERR_ARG, "null context");
    free_all(reinterpret_cast<Ctx *>(ctx));
    return DJ_OK;
}

int djtled_info(const djtled_ctx *ctx, djtled_info_t *o) {
    if (!ctx || !o) return fail(DJ_ERR_ARG, "null argument");
    const Ctx &c = *reinterpret_cast<const Ctx *>(ctx);
    o->n_nodes = c.n_nodes;
    o->n_elems = c.n_elems;
    o->elem_type = c.ne;
    o->model = c.model;
    o->precision = c.prec;
    o->dt = c.dt;
    o->dt_crit = c.dt_crit;
    o->alpha = c.alpha;
    o->n_chunks = c.topo.n_chunks;
    o->chunk_elems = c.chunk_elems;
    o->n_copies = c.topo.n_copies;
    o->n_shared_copies = c.n_shared_copies;
    o->grid_blocks = c.grid;
    o->block_threads = c.block;
    o->variant = c.variant;
    o->formulation = c.form;
    o->bytes_per_step = c.bytes_per_step;
    o->elem_bytes = c.elem_bytes;
    o->mass_total = c.mass_total;
    return DJ_OK;
}

int djtled_forces(djtled_ctx *ctx, const void *u_dev, void *f_dev, void *stream) {
    if (!ctx || !u_dev || !f_dev) return fail(DJ_ERR_ARG, "null argument");
    Ctx &c = *reinterpret_cast<Ctx *>(ctx);
    if (c.form == DJ_FORM_NODAL_PRESSURE) return djtled_forces_anp(ctx, u_dev, f_dev, stream);
    DJ_HIP(hipSetDevice(c.device));
    DJ_HIP(launch_forces(c, u_dev, f_dev, static_cast<hipStream_t>(stream)));
    return DJ_OK;
}

int djtled_forces_noalloc(djtled_ctx *ctx, const void *u_dev, void *f_dev, void *stream) {
    if (!ctx || !u_dev || !f_dev) return fail(DJ_ERR_ARG, "null argument");
    Ctx &c = *reinterpret_cast<Ctx *>(ctx);
    if (c.n_inst > 1) return fail(DJ_ERR_ARG, "batch contexts have no forces entry point");
    if (c.form == DJ_FORM_NODAL_PRESSURE)
        return fail(DJ_ERR_UNSUPPORTED, "djtled_forces_noalloc: not for average-nodal-pressure contexts");
    const size_t ts = c.prec == DJ_FP32 ? sizeof(float) : sizeof(double);
    const size_t ubytes = (size_t(3) * c.topo.n_copies * ts + 255) & ~size_t(255);
    const size_t need = ubytes + size_t(3) * std::max(c.topo.n_part, 1) * ts;
    if (need > noalloc_scratch_bytes())
        return fail(DJ_ERR_UNSUPPORTED, "djtled_forces_noalloc: this context needs " + std::to_string(need) +
                                            " bytes of scratch; the fixed scratch holds " +
                                            std::to_string(noalloc_scratch_bytes()));
    DJ_HIP(hipSetDevice(c.device));
    void *base = nullptr;
    DJ_HIP(noalloc_scratch(c.device, &base));  // looked up at precompute; a table read here
    DJ_HIP(launch_forces_in(c, u_dev, f_dev, base, static_cast<char *>(base) + ubytes,
                            static_cast<hipStream_t>(stream)));
    return DJ_OK;
}

int djtled_forces_anp(djtled_ctx *ctx, const void *u_dev, void *f_dev, void *stream) {
    if (!ctx || !u_dev || !f_dev) return fail(DJ_ERR_ARG, "null argument");
    Ctx &c = *reinterpret_cast<Ctx *>(ctx);
    if (c.n_inst > 1) return fail(DJ_ERR_ARG, "batch contexts have no forces entry point");
    if ((c.model != DJ_NH && c.model != DJ_TI) || c.form == DJ_FORM_CLASSICAL || c.variant >= 4)
        return fail(DJ_ERR_UNSUPPORTED, "average nodal pressure: DJ_NH / DJ_TI, Jacobian form, variants 0..3");
    DJ_HIP(hipSetDevice(c.device));
    if (!c.d_anp_planes) {
        const size_t ts = c.prec == DJ_FP32 ? sizeof(float) : sizeof(double);
        DJ_HIP(dalloc(c, reinterpret_cast<char **>(&c.d_anp_planes),
                      size_t(n_planes(c.ne, c.model)) * c.topo.estride * ts));
        DJ_HIP(dalloc(c, &c.d_anp_je, size_t(c.n_elems)));
        DJ_HIP(dalloc(c, &c.d_anp_pn, size_t(c.n_nodes)));
    }
    DJ_HIP(launch_forces_anp(c, u_dev, f_dev, static_cast<hipStream_t>(stream)));
    return DJ_OK;
}

int djtled_loadset_create(djtled_ctx *ctx, const djtled_loads *ld, djtled_loadset **out) {
    if (!ctx || !ld || !out) return fail(DJ_ERR_ARG, "null argument");
    *out = nullptr;
    Ctx &c = *reinterpret_cast<Ctx *>(ctx);
    DJ_HIP(hipSetDevice(c.device));
    LoadSet *ls = nullptr;
    const int rc = make_loadset(c, ld, nullptr, &ls);
    if (rc == DJ_OK) *out = reinterpret_cast<djtled_loadset *>(ls);
    return rc;
}

int djtled_loadset_destroy(djtled_loadset *p) {
    if (!p) return fail(DJ_ERR_ARG, "null load set");
    LoadSet *ls = reinterpret_cast<LoadSet *>(p);
    Ctx &c = *ls->ctx;
    auto it = std::find(c.loadsets.begin(), c.loadsets.end(), static_cast<void *>(ls));
    if (it == c.loadsets.end()) return fail(DJ_ERR_ARG, "unknown load set");
    c.loadsets.erase(it);
    hipDeviceSynchronize();
    hipFree(ls->d_flags);
    hipFree(ls->d_ru);
    hipFree(ls->d_rate);
    delete ls;
    return DJ_OK;
}

int djtled_step(djtled_ctx *ctx, djtled_state *st, const djtled_loadset *lsp, int32_t n_steps,
                const djtled_step_opts *opts, djtled_status *out, void *stream) {
    return step_cases(ctx, 1, st, &lsp, n_steps, opts, out, nullptr, nullptr, stream);
}

int djtled_step_multi(djtled_ctx *ctx, int32_t nrhs, djtled_state *state, const djtled_loadset *const *loads,
                      int32_t n_steps, const djtled_step_opts *opts, djtled_status *out, double *residuals,
                      int32_t *error_case, void *stream) {
    return step_cases(ctx, nrhs, state, loads, n_steps, opts, out, residuals, error_case, stream);
}

int djtled_export_constants(djtled_ctx *ctx, double *V, double *dhdX, double *mass) {
    if (!ctx) return fail(DJ_ERR_ARG, "null context");
    Ctx &c = *reinterpret_cast<Ctx *>(ctx);
    DJ_HIP(hipSetDevice(c.device));
    double *dV = nullptr, *dB = nullptr, *dM = nullptr;
    TempBufs tb;
    if (V) DJ_HIP(tb.up(&dV, std::vector<double>(c.n_elems)));
    if (dhdX) DJ_HIP(tb.up(&dB, std::vector<double>(size_t(c.n_elems) * 3 * c.ne)));
    if (mass) DJ_HIP(tb.up(&dM, std::vector<double>(c.n_nodes)));
    DJ_HIP(launch_export(c, dV, dB, dM, nullptr));
    DJ_HIP(hipDeviceSynchronize());
    if (V) DJ_HIP(hipMemcpy(V, dV, sizeof(double) * c.n_elems, hipMemcpyDeviceToHost));
    if (dhdX) DJ_HIP(hipMemcpy(dhdX, dB, sizeof(double) * c.n_elems * 3 * c.ne, hipMemcpyDeviceToHost));
    if (mass) DJ_HIP(hipMemcpy(mass, dM, sizeof(double) * c.n_nodes, hipMemcpyDeviceToHost));
    return DJ_OK;
}

}  // extern "C"
