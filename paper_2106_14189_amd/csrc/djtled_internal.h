// Internal declarations shared by the host side (djtled_api.cpp) and the HIP
// kernels (djtled_kernels.hip) of libdjtled.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/djtled.h"

namespace dj {

// Per-copy flag bits.  A "copy" is one chunk's private instance of a node:
// every chunk keeps the state of all nodes its elements touch.
enum : uint32_t {
    FLAG_BC_MASK = 7u,       // bit k: component k prescribed
    FLAG_SHARED = 8u,        // node has copies in more than one chunk
    FLAG_CANON = 16u,        // the copy that writes the node to caller arrays
    FLAG_RU = 32u,           // the loads hold a value for this node (R or BC target)
    FLAG_NCOPY_SHIFT = 8u,   // bits 8..15: number of copies of a shared node
    FLAG_RANK_SHIFT = 16u    // bits 16..23: this copy's rank among them (ascending chunk)
};

// One chunk = a contiguous range of (reordered) elements processed by one
// workgroup, plus its private node copies [copy_begin, copy_begin + copy_count);
// the first n_interior copies are nodes touched by this chunk only.  The
// chunk's (element, node) incidences are numbered in node-copy order; copy l
// owns the contiguous positions crange[l], and wpos[a][e] is the position of
// node a of element e.
// chunks per workgroup of the single-context step kernel (its LDS list:
// 4 KB, which still lets three 1024-element FP32 chunks share a CU)
constexpr int KMAX = 128;

struct ChunkDesc {
    int32_t elem_begin, elem_count, copy_begin, copy_count;
    int32_t n_interior, tag, pad1, pad2;  // tag: element kind (batches)
};

// Element kinds of a batch: slot t holds the group of (T4|H8) x (NH|TI)
// instances, t = 2 * (element is H8) + (model is TI).
inline int kind_of(int ne, int model) { return (ne == 8 ? 2 : 0) + (model == DJ_TI ? 1 : 0); }

// Element-constant plane indices.  Each plane holds one scalar per element
// (structure of arrays, element stride `estride`).
// Kernel template MODEL = material model | DJ_FORM_TLED for the classical
// TLED force (Eq. 4) instead of the Table 3 force; both read the same planes.
constexpr int DJ_FORM_TLED = 16;
// MODEL | DJ_FORM_ANP: the kappa 0V plane holds the element's average nodal
// pressure times 0V, which replaces kappa (J - 1) 0V in the force
constexpr int DJ_FORM_ANP = 32;
constexpr int base_model(int model) { return model & 15; }

constexpr int model_planes(int model) {  // planes of the material part, after 0J^-1, mu 0V, kappa 0V
    return base_model(model) == DJ_TI ? 4 : base_model(model) == DJ_OT ? 8 : base_model(model) == DJ_MR ? 1 : 0;
}

template <int NE, int MODEL>
struct Planes {
    static constexpr int JINV = 0;                        // 0J^-1, row-major 3 x 3
    static constexpr int MUV = 9;                         // mu * 0V (MR: 2 C10 0V)
    static constexpr int KAV = 10;                        // kappa * 0V
    static constexpr int FIB = 11;                        // TI, OT: unit fibre a (3)
    static constexpr int ETAV = 14;                       // TI, OT: eta_a * 0V
    static constexpr int FIBB = 15;                       // OT: unit fibre b (3)
    static constexpr int ETABV = 18;                      // OT: eta_b * 0V
    static constexpr int C01V = 11;                       // MR: C01 * 0V
    static constexpr int HG = 11 + model_planes(MODEL);   // H8: g_alpha (4 x 3)
    static constexpr int KHG = HG + 12;                   // H8: hourglass stiffness
    static constexpr int N = (NE == 8) ? KHG + 1 : HG;    // number of planes
};

inline int n_planes(int ne, int model) {
    const int n = 11 + model_planes(model);
    return ne == 8 ? n + 13 : n;
}

// Kernel variants (threads per workgroup, elements per thread); the chunk
// capacity is block * ept elements.
struct Variant {
    int block, ept, mcopy;  // mcopy: node copies per thread a chunk may hold
    int wpe;                // minimum waves per SIMD the step kernel is compiled for (register budget)
};
constexpr int N_VARIANTS = 6;
const std::vector<Variant> &variants(int ne, int prec);

// Everything the kernels need, as device pointers.
struct DevTopo {
    const ChunkDesc *chunks = nullptr;
    int32_t n_chunks = 0;
    int32_t n_copies = 0;
    int32_t cmax = 0;           // chunk capacity (slot stride in LDS)
    const uint32_t *crange = nullptr;    // per copy: first incidence position in the chunk
                                         // | number of incidences << 16
    const uint16_t *wpos = nullptr;      // NE planes over elements (stride estride)
    const uint32_t *flags = nullptr;
    const int32_t *pidx = nullptr;       // shared copies: start of the node's partial group
    const int32_t *cnode = nullptr;      // caller node index of each copy
    int32_t n_part = 0;                  // partial-force entries (one per shared copy)
    const void *elem = nullptr;          // element planes (context precision)
    // FP32 contexts: the same planes and slot positions interleaved per element,
    // D = NP + NE / 2 words (two positions per word): words 4g .. 4g + 3 of
    // element e at 16-byte entry g * estride + e (g < D / 4), the last D % 4
    // words as single planes after them (word 4 (D / 4) + r at r * estride + e)
    const void *elem4 = nullptr;
    int64_t estride = 0;
    const void *acoef = nullptr;         // per copy A_i = 2 dt^2 / ((2 + alpha dt) m_i)
    const void *bpc = nullptr;           // batches: per copy B' = (2 - alpha dt) / (2 + alpha dt)
};

// load cases stepped together by one launch (multi-RHS)
constexpr int MAX_RHS = 8;

struct StepArgs {
    int32_t nrhs = 1;           // load cases; case r's planes follow those of case r - 1 in every array below
    const uint32_t *flags = nullptr;  // nrhs x copies: topology flags | load bits
    const void *ru = nullptr;   // nrhs x 3 planes over copies (BC target or R), or null (no loads)
    int32_t ramp = DJ_RAMP_NONE;  // common to the cases
    double t_ramp = 0.0;
    double dt = 0.0;
    double bprime = 0.0;        // (2 - alpha dt) / (2 + alpha dt)
    int64_t step0 = 0;
    int32_t n_steps = 0;
    int32_t relax = 0;
    double tol = 0.0;
    int32_t check_every = 1;
    int32_t cur0 = 0;           // buffer index of u^n at entry (prev = cur0 + 2 mod 3)
    void *ubuf[3] = {nullptr, nullptr, nullptr};  // each: nrhs x 3 planes over copies
    void *part = nullptr;       // partial forces: nrhs x 2 parities x 3 planes over n_part entries
    void *u_out_cur = nullptr;  // caller arrays written at the end: nrhs x n_nodes x 3 each
    void *u_out_prev = nullptr;
    int64_t out_stride = 0;     // 3 n_nodes
    uint32_t *bar = nullptr;    // barrier flags: (grid + 16) x 32 uint32
    int32_t *status = nullptr;  // [0] code [1] steps done [2] error element (internal) [3] error step offset
                                // [4] barrier abort [5..6] per-parity error words [7] case of the error
    double *red = nullptr;      // residual partials: 2 parities x grid x nrhs x 2
    double *res_out = nullptr;  // last residual per case
    // average-nodal-pressure step: per copy c_n = kappa_n / V_n and nodal
    // pressure p_n, and the J partial sums of shared copies (one plane)
    const void *anp_c = nullptr;
    void *anp_p = nullptr;
    void *anp_jpart = nullptr;
};

struct Ctx {
    int device = 0;
    int n_nodes = 0, n_elems = 0, ne = 4, model = DJ_NH, prec = DJ_FP32, form = DJ_FORM_JACOBIAN;
    int variant = 0, block = 256, ept = 4, mcopy = 2, cmax = 1024, grid = 1, chunk_elems = 0;
    double dt = 0, dt_crit = 0, alpha = 0, rho = 0, hg_kappa = 0.1, mass_total = 0;
    int n_shared_copies = 0;
    double bytes_per_step = 0, elem_bytes = 0;
    std::vector<int32_t> elem_perm;  // internal element -> caller element
    std::vector<int32_t> node_perm;  // internal node -> caller node
    DevTopo topo;
    // device allocations owned by the context
    std::vector<void *> allocs;
    void *d_elem = nullptr, *d_acoef = nullptr;
    void *d_ubuf[3] = {nullptr, nullptr, nullptr};
    void *d_part = nullptr;
    uint32_t *d_bar = nullptr;
    int32_t *d_status = nullptr;
    double *d_red = nullptr;
    // average nodal pressure (forces entry point): element nodes, node -> element
    // lists (internal ids), kappa per element (FP64), scratch planes and pressures
    int32_t *d_enode = nullptr, *d_ne_off = nullptr, *d_ne_list = nullptr;
    double *d_kappa64 = nullptr;
    void *d_anp_planes = nullptr;
    double *d_anp_je = nullptr, *d_anp_pn = nullptr;
    // average-nodal-pressure step (formulation DJ_FORM_NODAL_PRESSURE): per copy
    // c_n and p_n, J partials (context precision)
    void *d_anps_c = nullptr, *d_anps_p = nullptr, *d_anps_j = nullptr;
    // several load cases per launch: buffers grown on demand (case capacity rhs_cap)
    int rhs_cap = 0;
    void *d_mubuf[3] = {nullptr, nullptr, nullptr};
    void *d_mpart = nullptr;
    double *d_mred = nullptr;
    uint32_t *d_mflags = nullptr;   // rhs_cap x copies
    void *d_mru = nullptr;          // rhs_cap x 3 planes over copies
    double *d_V64 = nullptr, *d_jinv64 = nullptr, *d_mass64 = nullptr;
    int32_t *d_elem_perm = nullptr, *d_node_perm = nullptr, *d_inode = nullptr;
    int32_t *h_status = nullptr;     // pinned
    double *h_res = nullptr;         // pinned
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // brackets the persistent kernel
    std::vector<uint32_t> h_flags;   // topology flags per copy
    std::vector<int32_t> h_copy_node;  // internal node of each copy
    std::vector<int32_t> h_chunk_elem; // per chunk: first element, element count
    std::vector<void *> loadsets;
    // several instances in one context (batches): per-instance step, damping
    int n_inst = 1;
    std::vector<double> inst_dt, inst_dt_crit, inst_alpha;
    std::vector<int32_t> inst_node_off, inst_elem_off;  // caller numbering, n_inst + 1 entries
    void *d_bpc = nullptr;
};

// Extra inputs of a multi-instance context: caller nodes and elements are
// numbered instance by instance (offsets below); every instance has its own
// damping and time step.
struct MultiInst {
    int n_inst = 1;
    const int32_t *node_off = nullptr;  // n_inst + 1
    const int32_t *elem_off = nullptr;  // n_inst + 1
    const double *alpha = nullptr;      // per instance
    int batch = 0;                      // chunks feed a batch work list (no per-context grid rounds)
};

struct LoadSet {
    Ctx *ctx = nullptr;
    uint32_t *d_flags = nullptr;     // topology flags | BC mask | FLAG_RU
    void *d_ru = nullptr;
    int ramp = DJ_RAMP_NONE;
    double t_ramp = 0.0;
    void *d_rate = nullptr;          // batches: per copy ramp rate (see ramp_rate)
};

// ---- host side (djtled_api.cpp) ----
extern thread_local std::string g_err;  // djtled_last_error()
int fail(int code, const std::string &msg);
void free_all(Ctx *c);
int build(Ctx &c, const djtled_mesh *mesh, const djtled_material *mat, const djtled_params *prm,
          const MultiInst *mi = nullptr);
int make_loadset(Ctx &c, const djtled_loads *ld, const double *node_rate, LoadSet **out);

#define DJ_HIP(call)                                                                                         \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return ::dj::fail(DJ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---- kernel launchers (djtled_kernels.hip) ----
hipError_t occupancy(int ne, int model, int form, int prec, int variant, int *blocks_per_cu, size_t *lds_bytes);
hipError_t occupancy_multi(const Ctx &c, int *blocks_per_cu);  // several-cases kernel; 0 if not built
// per-element material arrays (device, FP64, original element order); the
// fibre and C01 arrays are read only by the models that use them
struct MatDev {
    const double *E, *nu;
    const double *eta, *fib;    // TI, OT: fibre a
    const double *etab, *fibb;  // OT: fibre b
    const double *c01;          // MR
};
hipError_t launch_precompute(Ctx &c, const double *dX, const int32_t *dconn, const MatDev &m, const int32_t *d_einst,
                             double *d_dtmin, int32_t *d_bad, hipStream_t s);
// c2: per internal node 2 dt^2 / (2 + alpha dt) of its instance; bp: per node
// B' (written per copy to c.d_bpc when that is allocated)
// FP32 batches: interleave the element planes and slot positions into elem4
hipError_t launch_pack_elem4(Ctx &c, void *dst, hipStream_t s);
hipError_t launch_mass_acoef(Ctx &c, const int32_t *d_ne_off, const int32_t *d_ne_list, const double *d_c2,
                             const double *d_bp, hipStream_t s);
hipError_t launch_forces(Ctx &c, const void *u, void *f, hipStream_t s);
// the same in caller-given device buffers: 3 x n_copies u planes, 3 x max(n_part, 1) partials
hipError_t launch_forces_in(Ctx &c, const void *u, void *f, void *ubuf0, void *part, hipStream_t s);
// device address of the fixed scratch array of the allocation-free entry points
// on the current device (looked up once per device); its size in bytes
hipError_t noalloc_scratch(int device, void **ptr);
size_t noalloc_scratch_bytes();
hipError_t launch_step(Ctx &c, const StepArgs &a, const void *u_cur_in, const void *u_prev_in, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_export(Ctx &c, double *d_V, double *d_dhdX, double *d_mass, hipStream_t s);
// internal forces with the average nodal pressure (u, f: caller order)
hipError_t launch_forces_anp(Ctx &c, const void *u, void *f, hipStream_t s);
// average-nodal-pressure step contexts: kappa plane <- 0V, per-copy c_n
hipError_t launch_anps_setup(Ctx &c, hipStream_t s);

// One launcher operation for one (precision, element type, form), dispatched
// over (model, variant) by the instantiating unit inst_<p><ne> (f: FP32,
// d: FP64, c: FP32 classical TLED form).
enum class Op { OCC, OCC_MULTI, FORCES, STEP, FORCES_ANP };
struct OpArgs {
    Op op = Op::OCC;
    Ctx *c = nullptr;
    int model = DJ_NH, variant = 0;
    int *bpc = nullptr;          // OCC, OCC_MULTI: workgroups per CU
    size_t *lds = nullptr;       // OCC: dynamic LDS bytes
    const void *u = nullptr;     // FORCES, FORCES_ANP: caller-order u and f
    void *f = nullptr;
    hipStream_t s = nullptr;
    const StepArgs *a = nullptr;  // STEP
    const void *u_cur_in = nullptr, *u_prev_in = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    void *ubuf0 = nullptr;        // FORCES: node-copy u planes and partial sums to use instead of
    void *part = nullptr;         //   the context's (both or neither)
    int anp = 0;                  // OCC, STEP: the average-nodal-pressure step kernel
};
hipError_t inst_f4(const OpArgs &o);
hipError_t inst_f8(const OpArgs &o);
hipError_t inst_d4(const OpArgs &o);
hipError_t inst_d8(const OpArgs &o);
hipError_t inst_c4(const OpArgs &o);
hipError_t inst_c8(const OpArgs &o);

}  // namespace dj
