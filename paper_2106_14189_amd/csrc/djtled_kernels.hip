// HIP kernels of the single-mesh DJ-TLED context for gfx950 (MI355X):
// pre-computation and the launchers.  The step and force kernels are
// templates in djtled_step.h, instantiated per (precision, element type,
// form) in the djtled_inst_*.hip translation units.
#include <mutex>

#include "djtled_device.h"

namespace dj {

// ---------------------------------------------------------------------------
// Pre-computation (Algorithm 1) in FP64, one thread per element
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tri_area(const double *p, const double *q, const double *r) {
    const double u0 = q[0] - p[0], u1 = q[1] - p[1], u2 = q[2] - p[2];
    const double v0 = r[0] - p[0], v1 = r[1] - p[1], v2 = r[2] - p[2];
    const double w0 = u1 * v2 - u2 * v1, w1 = u2 * v0 - u0 * v2, w2 = u0 * v1 - u1 * v0;
    return 0.5 * sqrt(w0 * w0 + w1 * w1 + w2 * w2);
}

template <typename T, int NE, int MODEL>
__global__ void k_precompute(const double *__restrict__ X, const int32_t *__restrict__ conn, int E,
                             const double *__restrict__ Ein, const double *__restrict__ nuin,
                             const double *__restrict__ etar, const double *__restrict__ fib,
                             const double *__restrict__ etabr, const double *__restrict__ fibb,
                             const double *__restrict__ c01in, double hg_kappa, double rho, T *__restrict__ planes, int64_t es, double *__restrict__ V64,
                             double *__restrict__ jinv64, const int32_t *__restrict__ einst,
                             unsigned long long *__restrict__ dtmin, int32_t *__restrict__ bad) {
    using P = Planes<NE, MODEL>;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double x[NE][3];
    for (int a = 0; a < NE; a++)
        for (int k = 0; k < 3; k++) x[a][k] = X[3 * int64_t(conn[int64_t(NE) * e + a]) + k];
    // 0J = H_xi X_e (Eq. 3); coordinates relative to node 0 (rows of H_xi sum to zero)
    double J0[3][3];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) {
            double s = 0.0;
            if (NE == 4) {
                s = x[i + 1][k] - x[0][k];
            } else {
                for (int a = 1; a < 8; a++) s += h8s(a, i) * (x[a][k] - x[0][k]);
                s *= 0.125;
            }
            J0[i][k] = s;
        }
    const double det = det3d(J0);
    if (!(det > 0.0)) {
        atomicAdd(bad, 1);
        return;
    }
    const double V = (NE == 4) ? det / 6.0 : 8.0 * det;
    double Ji[3][3];
    Ji[0][0] = (J0[1][1] * J0[2][2] - J0[1][2] * J0[2][1]) / det;
    Ji[0][1] = (J0[0][2] * J0[2][1] - J0[0][1] * J0[2][2]) / det;
    Ji[0][2] = (J0[0][1] * J0[1][2] - J0[0][2] * J0[1][1]) / det;
    Ji[1][0] = (J0[1][2] * J0[2][0] - J0[1][0] * J0[2][2]) / det;
    Ji[1][1] = (J0[0][0] * J0[2][2] - J0[0][2] * J0[2][0]) / det;
    Ji[1][2] = (J0[0][2] * J0[1][0] - J0[0][0] * J0[1][2]) / det;
    Ji[2][0] = (J0[1][0] * J0[2][1] - J0[1][1] * J0[2][0]) / det;
    Ji[2][1] = (J0[0][1] * J0[2][0] - J0[0][0] * J0[2][1]) / det;
    Ji[2][2] = (J0[0][0] * J0[1][1] - J0[0][1] * J0[1][0]) / det;
    const double Ev = Ein[e], nu = nuin[e];
    const double mu = Ev / (2.0 * (1.0 + nu));
    const double ka = Ev / (3.0 * (1.0 - 2.0 * nu));
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            planes[(P::JINV + 3 * i + j) * es + e] = T(Ji[i][j]);
            jinv64[9 * int64_t(e) + 3 * i + j] = Ji[i][j];
        }
    planes[P::MUV * es + e] = T(mu * V);
    planes[P::KAV * es + e] = T(ka * V);
    V64[e] = V;
    // fibre stiffness (TI: a; OT: a and b) and the Mooney-Rivlin C01; they
    // raise the dilatational wave speed of Eq. 14 and the hourglass stiffness
    double eta = 0.0, c01 = 0.0;
    if constexpr (MODEL == DJ_TI || MODEL == DJ_OT) {
        for (int f = 0; f < (MODEL == DJ_OT ? 2 : 1); f++) {
            const double *v = (f == 0 ? fib : fibb) + 3 * int64_t(e);
            const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(nrm > 0.0)) {
                atomicAdd(bad, 1);
                return;
            }
            const double et = (f == 0 ? etar : etabr)[e] * mu;
            const int fp = f == 0 ? P::FIB : P::FIBB, ep = f == 0 ? P::ETAV : P::ETABV;
            for (int k = 0; k < 3; k++) planes[(fp + k) * es + e] = T(v[k] / nrm);
            planes[ep * es + e] = T(et * V);
            eta += et;
        }
    }
    if constexpr (MODEL == DJ_MR) {
        c01 = c01in[e];
        planes[P::C01V * es + e] = T(c01 * V);
    }
    const double mu_eff = mu + 2.0 * c01;  // initial shear modulus 2 (C10 + C01)
    // characteristic length of Eq. 14
    double L;
    if (NE == 4) {
        double amax = tri_area(x[1], x[2], x[3]);
        amax = fmax(amax, tri_area(x[0], x[2], x[3]));
        amax = fmax(amax, tri_area(x[0], x[1], x[3]));
        amax = fmax(amax, tri_area(x[0], x[1], x[2]));
        L = 3.0 * V / amax;
    } else {
        // dh/dX = 0J^-1 H_xi; hourglass vectors and stiffness (Flanagan-Belytschko)
        double sb = 0.0;
        for (int a = 0; a < 8; a++)
            for (int i = 0; i < 3; i++) {
                const double b = 0.125 * (Ji[i][0] * h8s(a, 0) + Ji[i][1] * h8s(a, 1) + Ji[i][2] * h8s(a, 2));
                sb += b * b;
            }
        for (int al = 0; al < 4; al++)
            for (int i = 0; i < 3; i++) {
                double g = 0.0;
                for (int b = 1; b < 8; b++) g += hgG(al, b) * (x[b][i] - x[0][i]);
                planes[(P::HG + 3 * al + i) * es + e] = T(g);
            }
        planes[P::KHG * es + e] = T(hg_kappa * (ka + 4.0 * mu_eff / 3.0) * V * sb / 8.0);
        L = 1.0 / sqrt(2.0 * sb);
    }
    const double cw = sqrt((ka + 4.0 * mu_eff / 3.0 + 4.0 * eta) / rho);
    const double dte = L / cw;
    // positive doubles order like their bit patterns
    atomicMin(dtmin + (einst ? einst[e] : 0), __double_as_longlong(dte));
}

__global__ void k_node_mass(const int32_t *__restrict__ off, const int32_t *__restrict__ lst, int n_nodes, int ne,
                            double rho, const double *__restrict__ V64, double *__restrict__ mass) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    double m = 0.0;
    for (int j = off[n]; j < off[n + 1]; j++) m += rho * V64[lst[j]] / ne;
    mass[n] = m;
}

// A per copy (and B' per copy for batches) from the node's instance coefficients
template <typename T>
__global__ void k_acoef(const int32_t *__restrict__ inode, int n_copies, const double *__restrict__ mass, double c2,
                        const double *__restrict__ c2n, const double *__restrict__ bpn, T *__restrict__ acoef,
                        T *__restrict__ bpc) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_copies) return;
    const int n = inode[l];
    acoef[l] = T((c2n ? c2n[n] : c2) / mass[n]);
    if (bpc) bpc[l] = T(bpn[n]);
}

template <int NE>
__global__ void k_export(const double *__restrict__ V64, const double *__restrict__ jinv64,
                         const int32_t *__restrict__ eperm, int E, double *__restrict__ V, double *__restrict__ dhdX) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int o = eperm[e];
    if (V) V[o] = V64[e];
    if (dhdX) {
        const double *Ji = jinv64 + 9 * int64_t(e);
        for (int i = 0; i < 3; i++)
            for (int a = 0; a < NE; a++) {
                double s;
                if (NE == 4) {
                    s = (a == 0) ? -(Ji[3 * i] + Ji[3 * i + 1] + Ji[3 * i + 2]) : Ji[3 * i + a - 1];
                } else {
                    s = 0.125 * (Ji[3 * i] * h8s(a, 0) + Ji[3 * i + 1] * h8s(a, 1) + Ji[3 * i + 2] * h8s(a, 2));
                }
                dhdX[(int64_t(o) * 3 + i) * NE + a] = s;
            }
    }
}

__global__ void k_export_mass(const double *__restrict__ mass, const int32_t *__restrict__ nperm, int N,
                              double *__restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    out[nperm[n]] = mass[n];
}

// ---------------------------------------------------------------------------
// Dispatch over (precision, element type, form) to the instantiating units;
// each dispatches over (model, variant).  The classical TLED form is built in
// FP32 only (a comparison path).
// ---------------------------------------------------------------------------
static hipError_t dispatch_op(int prec, int ne, int form, OpArgs o) {
    if (form == DJ_FORM_CLASSICAL) {
        if (prec != DJ_FP32) return hipErrorInvalidValue;
        return ne == 4 ? inst_c4(o) : inst_c8(o);
    }
    if (form == DJ_FORM_NODAL_PRESSURE) o.anp = 1;  // the Jacobian units hold the ANP step kernels
    if (prec == DJ_FP32) return ne == 4 ? inst_f4(o) : inst_f8(o);
    return ne == 4 ? inst_d4(o) : inst_d8(o);
}

const std::vector<Variant> &variants(int ne, int prec) {
    static const std::vector<Variant> t4f(VAR_T4F, VAR_T4F + N_VARIANTS), h8f(VAR_H8F, VAR_H8F + N_VARIANTS);
    static const std::vector<Variant> t4d(VAR_T4D, VAR_T4D + N_VARIANTS), h8d(VAR_H8D, VAR_H8D + N_VARIANTS);
    if (prec == DJ_FP32) return ne == 4 ? t4f : h8f;
    return ne == 4 ? t4d : h8d;
}

hipError_t occupancy(int ne, int model, int form, int prec, int variant, int *blocks_per_cu, size_t *lds_bytes) {
    OpArgs o;
    o.op = Op::OCC;
    o.model = model;
    o.variant = variant;
    o.bpc = blocks_per_cu;
    o.lds = lds_bytes;
    return dispatch_op(prec, ne, form, o);
}

hipError_t occupancy_multi(const Ctx &c, int *blocks_per_cu) {
    OpArgs o;
    o.op = Op::OCC_MULTI;
    o.model = c.model;
    o.variant = c.variant;
    o.bpc = blocks_per_cu;
    return dispatch_op(c.prec, c.ne, c.form, o);
}

hipError_t launch_forces_anp(Ctx &c, const void *u, void *f, hipStream_t s) {
    OpArgs o;
    o.op = Op::FORCES_ANP;
    o.c = &c;
    o.model = c.model;
    o.variant = c.variant;
    o.u = u;
    o.f = f;
    o.s = s;
    return dispatch_op(c.prec, c.ne, DJ_FORM_JACOBIAN, o);
}

hipError_t launch_forces(Ctx &c, const void *u, void *f, hipStream_t s) {
    OpArgs o;
    o.op = Op::FORCES;
    o.c = &c;
    o.model = c.model;
    o.variant = c.variant;
    o.u = u;
    o.f = f;
    o.s = s;
    return dispatch_op(c.prec, c.ne, c.form, o);
}

hipError_t launch_forces_in(Ctx &c, const void *u, void *f, void *ubuf0, void *part, hipStream_t s) {
    OpArgs o;
    o.op = Op::FORCES;
    o.c = &c;
    o.model = c.model;
    o.variant = c.variant;
    o.u = u;
    o.f = f;
    o.s = s;
    o.ubuf0 = ubuf0;
    o.part = part;
    return dispatch_op(c.prec, c.ne, c.form, o);
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free entry point (djtled_forces_noalloc):
// the node-copy u planes and shared-node partial sums of one force
// evaluation live in this file-scope device array, one per GPU, held until
// the process ends.  In host code the array's name is only a stand-in: its
// device address on each GPU is looked up once, with that GPU current, and
// only that address is ever passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DJTLED_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

size_t noalloc_scratch_bytes() { return DJTLED_NOALLOC_SCRATCH_BYTES; }

hipError_t noalloc_scratch(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_step(Ctx &c, const StepArgs &a, const void *u_cur_in, const void *u_prev_in, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
    OpArgs o;
    o.op = Op::STEP;
    o.c = &c;
    o.model = c.model;
    o.variant = c.variant;
    o.a = &a;
    o.u_cur_in = u_cur_in;
    o.u_prev_in = u_prev_in;
    o.s = s;
    o.ev0 = ev0;
    o.ev1 = ev1;
    return dispatch_op(c.prec, c.ne, c.form, o);
}

template <typename T, int NE, int MODEL>
static void precompute_m(Ctx &c, const double *dX, const int32_t *dconn, const MatDev &m, const int32_t *dei,
                         unsigned long long *dtm, int32_t *d_bad, hipStream_t s) {
    const int B = 256, G = (c.n_elems + B - 1) / B;
    hipLaunchKernelGGL((k_precompute<T, NE, MODEL>), dim3(G), dim3(B), 0, s, dX, dconn, c.n_elems, m.E, m.nu, m.eta,
                       m.fib, m.etab, m.fibb, m.c01, c.hg_kappa, c.rho, static_cast<T *>(c.d_elem), c.topo.estride,
                       c.d_V64, c.d_jinv64, dei, dtm, d_bad);
}

template <typename T, int NE>
static void precompute_ne(Ctx &c, const double *dX, const int32_t *dconn, const MatDev &m, const int32_t *dei,
                          unsigned long long *dtm, int32_t *d_bad, hipStream_t s) {
    switch (c.model) {
        case DJ_NH: return precompute_m<T, NE, DJ_NH>(c, dX, dconn, m, dei, dtm, d_bad, s);
        case DJ_TI: return precompute_m<T, NE, DJ_TI>(c, dX, dconn, m, dei, dtm, d_bad, s);
        case DJ_OT: return precompute_m<T, NE, DJ_OT>(c, dX, dconn, m, dei, dtm, d_bad, s);
        default: return precompute_m<T, NE, DJ_MR>(c, dX, dconn, m, dei, dtm, d_bad, s);
    }
}

hipError_t launch_precompute(Ctx &c, const double *dX, const int32_t *dconn, const MatDev &m, const int32_t *d_einst,
                             double *d_dtmin, int32_t *d_bad, hipStream_t s) {
    auto *dtm = reinterpret_cast<unsigned long long *>(d_dtmin);
    if (c.prec == DJ_FP32) {
        if (c.ne == 4) precompute_ne<float, 4>(c, dX, dconn, m, d_einst, dtm, d_bad, s);
        else precompute_ne<float, 8>(c, dX, dconn, m, d_einst, dtm, d_bad, s);
    } else {
        if (c.ne == 4) precompute_ne<double, 4>(c, dX, dconn, m, d_einst, dtm, d_bad, s);
        else precompute_ne<double, 8>(c, dX, dconn, m, d_einst, dtm, d_bad, s);
    }
    return hipGetLastError();
}

// one thread per element position (padding included): word d of the element
// goes to its 16-byte group or, past the last full group, to its own plane
__global__ void k_pack_elem4(const uint32_t *__restrict__ planes, const uint16_t *__restrict__ wpos, int np, int ne,
                             int64_t es, uint32_t *__restrict__ dst) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= es) return;
    const int D = np + ne / 2, G = D / 4;
    for (int d = 0; d < D; d++) {
        uint32_t w;
        if (d < np) {
            w = planes[d * es + e];
        } else {
            const int a = 2 * (d - np);
            w = uint32_t(wpos[a * es + e]) | (uint32_t(wpos[(a + 1) * es + e]) << 16);
        }
        if (d < 4 * G) dst[((d / 4) * es + e) * 4 + (d % 4)] = w;
        else dst[4 * G * es + (d - 4 * G) * es + e] = w;
    }
}

hipError_t launch_pack_elem4(Ctx &c, void *dst, hipStream_t s) {
    if (c.prec != DJ_FP32) return hipErrorInvalidValue;
    const int B = 256;
    const int64_t es = c.topo.estride;
    hipLaunchKernelGGL(k_pack_elem4, dim3(unsigned((es + B - 1) / B)), dim3(B), 0, s,
                       static_cast<const uint32_t *>(c.d_elem), c.topo.wpos, n_planes(c.ne, c.model), c.ne, es,
                       static_cast<uint32_t *>(dst));
    return hipGetLastError();
}

hipError_t launch_mass_acoef(Ctx &c, const int32_t *d_ne_off, const int32_t *d_ne_list, const double *d_c2,
                             const double *d_bp, hipStream_t s) {
    const int B = 256;
    hipLaunchKernelGGL(k_node_mass, dim3((c.n_nodes + B - 1) / B), dim3(B), 0, s, d_ne_off, d_ne_list, c.n_nodes, c.ne,
                       c.rho, c.d_V64, c.d_mass64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double c2 = 2.0 * c.dt * c.dt / (2.0 + c.alpha * c.dt);
    const int G = (c.topo.n_copies + B - 1) / B;
    if (c.prec == DJ_FP32)
        hipLaunchKernelGGL(k_acoef<float>, dim3(G), dim3(B), 0, s, c.d_inode, c.topo.n_copies, c.d_mass64, c2, d_c2,
                           d_bp, static_cast<float *>(c.d_acoef), static_cast<float *>(c.d_bpc));
    else
        hipLaunchKernelGGL(k_acoef<double>, dim3(G), dim3(B), 0, s, c.d_inode, c.topo.n_copies, c.d_mass64, c2, d_c2,
                           d_bp, static_cast<double *>(c.d_acoef), static_cast<double *>(c.d_bpc));
    return hipGetLastError();
}

// ---- average-nodal-pressure step set-up: the kappa plane holds 0V, and every
// copy gets c_n = kappa_n / V_n of its node (V_n = sum_e 0V_e / n_e, kappa_n
// the 0V_e / n_e-weighted mean of kappa_e), summed in ascending element order
template <typename T>
__global__ void k_anps_vplane(int E, const double *__restrict__ V64, T *__restrict__ plane) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) plane[e] = T(V64[e]);
}

template <typename T>
__global__ void k_anps_c(const int32_t *__restrict__ inode, int L, const int32_t *__restrict__ off,
                         const int32_t *__restrict__ lst, int ne, const double *__restrict__ V64,
                         const double *__restrict__ kappa, T *__restrict__ cn) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    const int n = inode[l];
    double v = 0.0, vk = 0.0;
    for (int j = off[n]; j < off[n + 1]; j++) {
        const int e = lst[j];
        const double w = V64[e] / ne;
        v += w;
        vk += w * kappa[e];
    }
    cn[l] = T(v > 0.0 ? vk / (v * v) : 0.0);
}

hipError_t launch_anps_setup(Ctx &c, hipStream_t s) {
    const int B = 256, E = c.n_elems, L = c.topo.n_copies;
    const int64_t kav = int64_t(Planes<4, DJ_NH>::KAV) * c.topo.estride;
    if (c.prec == DJ_FP32) {
        hipLaunchKernelGGL(k_anps_vplane<float>, dim3((E + B - 1) / B), dim3(B), 0, s, E, c.d_V64,
                           static_cast<float *>(c.d_elem) + kav);
        hipLaunchKernelGGL(k_anps_c<float>, dim3((L + B - 1) / B), dim3(B), 0, s, c.d_inode, L, c.d_ne_off,
                           c.d_ne_list, c.ne, c.d_V64, c.d_kappa64, static_cast<float *>(c.d_anps_c));
    } else {
        hipLaunchKernelGGL(k_anps_vplane<double>, dim3((E + B - 1) / B), dim3(B), 0, s, E, c.d_V64,
                           static_cast<double *>(c.d_elem) + kav);
        hipLaunchKernelGGL(k_anps_c<double>, dim3((L + B - 1) / B), dim3(B), 0, s, c.d_inode, L, c.d_ne_off,
                           c.d_ne_list, c.ne, c.d_V64, c.d_kappa64, static_cast<double *>(c.d_anps_c));
    }
    return hipGetLastError();
}

hipError_t launch_export(Ctx &c, double *d_V, double *d_dhdX, double *d_mass, hipStream_t s) {
    const int B = 256;
    if (d_V || d_dhdX) {
        if (c.ne == 4)
            hipLaunchKernelGGL(k_export<4>, dim3((c.n_elems + B - 1) / B), dim3(B), 0, s, c.d_V64, c.d_jinv64,
                               c.d_elem_perm, c.n_elems, d_V, d_dhdX);
        else
            hipLaunchKernelGGL(k_export<8>, dim3((c.n_elems + B - 1) / B), dim3(B), 0, s, c.d_V64, c.d_jinv64,
                               c.d_elem_perm, c.n_elems, d_V, d_dhdX);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (d_mass) {
        hipLaunchKernelGGL(k_export_mass, dim3((c.n_nodes + B - 1) / B), dim3(B), 0, s, c.d_mass64, c.d_node_perm,
                           c.n_nodes, d_mass);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace dj
