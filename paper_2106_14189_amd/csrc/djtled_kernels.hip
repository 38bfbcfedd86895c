// HIP kernels of the DJ-TLED time step for gfx950 (MI355X).
//
// Data layout (all structure-of-arrays, coalesced):
//   element planes  : one scalar per element per plane, chunk-contiguous
//   node copies     : every chunk (workgroup tile of <= cmax elements) owns a
//                     private copy of each node its elements touch; the copy
//                     state (u^n, u^{n-1}, u^{n+1} in three rotating buffers)
//                     is stored as 3 planes over copies
//   LDS             : 3 planes x (nodes per element) x cmax slots; slot
//                     a * cmax + e holds node a of local element e, first its
//                     displacement (scattered in from the copies through the
//                     local node -> slot CSR), then its element force
//   partials        : shared nodes (copies in several chunks) exchange their
//                     per-chunk force sums through a double-buffered array,
//                     read back in ascending chunk order after the step's
//                     single grid barrier, so every copy forms the same sum.
//
// Element force: Table 3 (neo-Hookean and transversely isotropic rows) in an
// increment form that is equal in exact arithmetic but has no O(1)
// cancellation in single precision:
//   tJ = 0J + dJ, dJ = H_xi Ue (Eq. 11),  D = 0J^-1 dJ,  tJ^-1 = (I + D)^-1 0J^-1
//   J - 1 = tr D + (tr^2 D - tr D^2) / 2 + det D      (Eq. 12)
//   I1 - 3 = g_hat^T m1 - 3 = 2 tr D + |D|^2           (Eq. 27; m1 from I1m = 2 0V 0J^-T 0J^-1)
//   I4 - 1 = g_hat^T m4 - 1 = 2 a.D a + |D^T a|^2      (Eq. 31; m4 from I4m, Eq. 45)
//   F = 0V [ c0 I + mu J^-2/3 D^T + 2 J^-2/3 psi4 (a + D^T a) a^T
//            - (p / J) D adj(I + D) ] 0J^-1 H_xi
// with p the volumetric coefficient of Table 3, c0 = mu J^-2/3 + p, and
// psi4 = eta_a (I4bar - 1).  The first three terms are J^-2/3 tJ^T (mu/2 I1m +
// psi4 I4m) with their O(1) part moved into c0; the last is p 0V tJ^-1 less
// that same O(1) part.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "djtled_internal.h"

namespace dj {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Cube root and reciprocal.  FP32 uses the hardware base-2 log / exp and
// reciprocal (about 1 ulp each): they only ever multiply O(strain) terms in the
// increment form below, so their error stays relative to the force.  FP64
// uses the correctly rounded library cbrt and division.
template <typename T>
__device__ __forceinline__ T dj_cbrt(T x);
template <>
__device__ __forceinline__ float dj_cbrt<float>(float x) {
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f));
}
template <>
__device__ __forceinline__ double dj_cbrt<double>(double x) { return cbrt(x); }
template <typename T>
__device__ __forceinline__ T dj_rcp(T x);
template <>
__device__ __forceinline__ float dj_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double dj_rcp<double>(double x) { return 1.0 / x; }

// H8 natural coordinate (+1 / -1) of node a along direction i, node order
// (---, +--, ++-, -+-, --+, +-+, +++, -++)
__host__ __device__ constexpr int h8s(int a, int i) {
    return (i == 0) ? ((((a + 1) >> 1) & 1) ? 1 : -1) : (i == 1) ? (((a >> 1) & 1) ? 1 : -1) : (((a >> 2) & 1) ? 1 : -1);
}
// Flanagan-Belytschko hourglass base vectors Gamma_alpha[a]
__host__ __device__ constexpr int hgG(int al, int a) {
    return al == 0 ? h8s(a, 0) * h8s(a, 1)
         : al == 1 ? h8s(a, 1) * h8s(a, 2)
         : al == 2 ? h8s(a, 2) * h8s(a, 0)
                   : h8s(a, 0) * h8s(a, 1) * h8s(a, 2);
}
static_assert(h8s(0, 0) == -1 && h8s(1, 0) == 1 && h8s(2, 0) == 1 && h8s(3, 0) == -1, "H8 order");
static_assert(h8s(2, 1) == 1 && h8s(3, 1) == 1 && h8s(4, 1) == -1 && h8s(7, 2) == 1, "H8 order");

__device__ __forceinline__ double ramp_value(int ramp, double t, double t_ramp) {
    if (ramp == DJ_RAMP_NONE || t_ramp <= 0.0) return 1.0;
    double tau = t / t_ramp;
    if (tau >= 1.0) return 1.0;
    if (tau <= 0.0) return 0.0;
    if (ramp == DJ_RAMP_LINEAR) return tau;
    return tau * tau * tau * (10.0 - 15.0 * tau + 6.0 * tau * tau);
}

// Device-scope relaxed store / load: write through to, and read from, the
// coherence point shared by all XCDs (used for every value one workgroup
// publishes to another).
template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// element force (register-resident).  cst: the element's planes.  u: nodal
// displacements.  F: nodal forces.  Returns J.
// ---------------------------------------------------------------------------
template <typename T, int NE, int MODEL>
__device__ __forceinline__ T element_force(const T *__restrict__ cst, const T (&u)[NE][3], T (&F)[NE][3]) {
    using P = Planes<NE, MODEL>;
    // relative displacements: differences of nearby values; the base node drops
    // out because every row of H_xi sums to zero
    T du[NE][3];
#pragma unroll
    for (int a = 1; a < NE; a++)
#pragma unroll
        for (int k = 0; k < 3; k++) du[a][k] = u[a][k] - u[0][k];
    // dJ = H_xi Ue (the increment of Eq. 11), rows = natural directions
    T dJ[3][3];
    if constexpr (NE == 4) {
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) dJ[i][k] = du[i + 1][k];
    } else {
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                T s = 0;
#pragma unroll
                for (int a = 1; a < 8; a++) s += (h8s(a, i) > 0) ? du[a][k] : -du[a][k];
                dJ[i][k] = s * T(0.125);
            }
    }
    const T *Ji = cst + P::JINV;
    // D = 0J^-1 dJ  (the transposed displacement gradient)
    T D[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) D[i][k] = Ji[3 * i] * dJ[0][k] + Ji[3 * i + 1] * dJ[1][k] + Ji[3 * i + 2] * dJ[2][k];
    const T trD = D[0][0] + D[1][1] + D[2][2];
    T trD2 = 0, nD2 = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            trD2 += D[i][j] * D[j][i];
            nD2 += D[i][j] * D[i][j];
        }
    const T detD = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) - D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                   D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    const T Jm1 = trD + T(0.5) * (trD * trD - trD2) + detD;  // J - 1  (Eq. 12)
    const T J = T(1) + Jm1;
    const T I1m3 = T(2) * trD + nD2;                          // I1 - 3 (Eq. 27)
    const T c = dj_cbrt(J);
    const T Jm23 = dj_rcp(c * c);                             // J^-2/3
    const T muV = cst[P::MUV], kaV = cst[P::KAV];
    T c0 = -(muV * T(1.0 / 3.0)) * Jm23 * I1m3 + kaV * J * Jm1;  // (mu J^-2/3 + p) 0V
    T Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) Q[i][k] = muV * Jm23 * D[k][i];
    if constexpr (MODEL == DJ_TI) {
        const T av[3] = {cst[P::FIB], cst[P::FIB + 1], cst[P::FIB + 2]};
        const T etaV = cst[P::ETAV];
        T Dta[3];
#pragma unroll
        for (int k = 0; k < 3; k++) Dta[k] = D[0][k] * av[0] + D[1][k] * av[1] + D[2][k] * av[2];
        const T aDa = av[0] * Dta[0] + av[1] * Dta[1] + av[2] * Dta[2];
        const T I4m1 = T(2) * aDa + Dta[0] * Dta[0] + Dta[1] * Dta[1] + Dta[2] * Dta[2];  // I4 - 1 (Eq. 31)
        const T Jm23m1 = -Jm1 * (c + T(1)) * dj_rcp(c * c * (c * c + c + T(1)));      // J^-2/3 - 1
        const T I4bm1 = Jm23 * I4m1 + Jm23m1;                                            // I4bar - 1
        const T psi4V = etaV * I4bm1;                                                    // eta (I4bar - 1) 0V
        c0 -= T(2.0 / 3.0) * psi4V * (T(1) + I4bm1);
        const T w = T(2) * Jm23 * psi4V;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) Q[i][k] += w * (av[i] + Dta[i]) * av[k];
    }
    const T pJ = (c0 - muV * Jm23) * dj_rcp(J);  // p 0V / J
    // adj(I + D)
    const T A00 = T(1) + D[0][0], A11 = T(1) + D[1][1], A22 = T(1) + D[2][2];
    T adj[3][3];
    adj[0][0] = A11 * A22 - D[1][2] * D[2][1];
    adj[0][1] = D[0][2] * D[2][1] - D[0][1] * A22;
    adj[0][2] = D[0][1] * D[1][2] - D[0][2] * A11;
    adj[1][0] = D[1][2] * D[2][0] - D[1][0] * A22;
    adj[1][1] = A00 * A22 - D[0][2] * D[2][0];
    adj[1][2] = D[0][2] * D[1][0] - A00 * D[1][2];
    adj[2][0] = D[1][0] * D[2][1] - A11 * D[2][0];
    adj[2][1] = D[0][1] * D[2][0] - A00 * D[2][1];
    adj[2][2] = A00 * A11 - D[0][1] * D[1][0];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        Q[i][i] += c0;
#pragma unroll
        for (int k = 0; k < 3; k++) Q[i][k] -= pJ * (D[i][0] * adj[0][k] + D[i][1] * adj[1][k] + D[i][2] * adj[2][k]);
    }
    // M = Q 0J^-1  (rows: force component, columns: natural direction)
    T M[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) M[i][j] = Q[i][0] * Ji[j] + Q[i][1] * Ji[3 + j] + Q[i][2] * Ji[6 + j];
    if constexpr (NE == 4) {
        // F = M H_xi with H_xi = [-1 1 0 0; -1 0 1 0; -1 0 0 1]: node 1 takes minus the sum
#pragma unroll
        for (int k = 0; k < 3; k++) {
            F[1][k] = M[k][0];
            F[2][k] = M[k][1];
            F[3][k] = M[k][2];
            F[0][k] = -(M[k][0] + M[k][1] + M[k][2]);
        }
    } else {
        // hourglass control: q_alpha = gamma_alpha^T Ue, gamma_alpha = Gamma_alpha - (dh/dX)^T g_alpha
        const T kh = cst[P::KHG];
        T q[4][3];
#pragma unroll
        for (int al = 0; al < 4; al++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                T s = 0;
#pragma unroll
                for (int a = 1; a < 8; a++) s += (hgG(al, a) > 0) ? du[a][k] : -du[a][k];
                const T *g = cst + P::HG + 3 * al;
                q[al][k] = s - (g[0] * D[0][k] + g[1] * D[1][k] + g[2] * D[2][k]);
            }
        // f_a = kh sum_alpha gamma_alpha[a] q_alpha: the dh/dX part joins M as - kh Qh^T 0J^-1
        T Qh[3][3];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                T s = 0;
#pragma unroll
                for (int al = 0; al < 4; al++) s += cst[P::HG + 3 * al + i] * q[al][k];
                Qh[i][k] = kh * s;
            }
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int j = 0; j < 3; j++) M[k][j] -= Qh[0][k] * Ji[j] + Qh[1][k] * Ji[3 + j] + Qh[2][k] * Ji[6 + j];
#pragma unroll
        for (int a = 0; a < 8; a++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const T s = M[k][0] * T(h8s(a, 0)) + M[k][1] * T(h8s(a, 1)) + M[k][2] * T(h8s(a, 2));
                const T h = T(hgG(0, a)) * q[0][k] + T(hgG(1, a)) * q[1][k] + T(hgG(2, a)) * q[2][k] +
                            T(hgG(3, a)) * q[3][k];
                F[a][k] = s * T(0.125) + kh * h;
            }
    }
    return J;
}

// ---------------------------------------------------------------------------
// Per-step pointers and node update
// ---------------------------------------------------------------------------
template <typename T>
struct StepPtrs {
    const T *uc[3];   // u^n planes (over copies)
    const T *up[3];   // u^{n-1}
    T *un[3];         // u^{n+1}
    T *pp[3];         // partial-force planes of this step's parity (over partial entries)
    const uint32_t *flags;
    const T *ru[3];   // load planes (null if no loads)
    const T *acoef;
    T bprime;
    T sval;           // ramp value s(t_{n+1})
    bool want_res;
    T *fout;          // forces entry point: caller-order output
};

struct PhaseOut {
    double num, den;  // residual partial sums over canonical copies
    int bad;          // 0, DJ_ERR_INVERTED or DJ_ERR_NONFINITE
    int bad_elem;     // internal element index
};

// u^{n+1} = u^n + B'(u^n - u^{n-1}) + A (R - F); prescribed components = s(t) target
template <typename T>
__device__ __forceinline__ void node_update(int l, uint32_t fl, const T (&f)[3], const T (&uc)[3], const T (&up)[3],
                                            T A, const T (&rv)[3], const StepPtrs<T> &sp, PhaseOut &po) {
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const bool pres = (fl >> k) & 1u;
        T un;
        if (pres) {
            un = sp.sval * rv[k];
            if (sp.want_res && (fl & FLAG_CANON)) po.den += double(f[k]) * double(f[k]);
        } else {
            un = uc[k] + sp.bprime * (uc[k] - up[k]) + A * (rv[k] - f[k]);
            if (sp.want_res && (fl & FLAG_CANON)) {
                const double d = double(f[k]) - double(rv[k]);
                po.num += d * d;
            }
        }
        fin = fin && isfinite(un);
        sp.un[k][l] = un;
    }
    if (!fin && po.bad == 0) {
        po.bad = DJ_ERR_NONFINITE;
        po.bad_elem = -1;
    }
}

// ---------------------------------------------------------------------------
// Chunk element phase.  Everything the chunk needs is requested in one round
// (element planes, each element's incidence positions, per-copy data).  In
// LDS the chunk's (element, node) incidences are numbered in node-copy order,
// so every copy owns a contiguous range: the scatter writes u^n of a copy over
// its range, each element reads its nodes' u from (and writes its forces to)
// its own positions, and each copy sums its contiguous range in fixed order.
// Interior copies are finished at once (force output or update); shared
// copies publish their partial sum into their node's group.
// ---------------------------------------------------------------------------
template <typename T, int KB>
struct SharedRegs {  // round-A data of one shared copy per chunk of a batch
    uint32_t fl[KB];
    int pb[KB], li[KB];
    bool ok[KB];
    T uc[KB][3], up[KB][3], rv[KB][3], A[KB];
};

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC>
struct Chunk {
    static constexpr int CMAX = BLOCK * EPT;
    static constexpr int NP = Planes<NE, MODEL>::N;
    static constexpr size_t LDS = size_t(3) * NE * CMAX * sizeof(T);

    // MODE 0: forces to the caller array; MODE 1: time-step update
    template <int MODE>
    __device__ static void element_phase(const DevTopo &tp, const ChunkDesc &ch, const StepPtrs<T> &sp,
                                         unsigned char *smem, PhaseOut &po) {
        const int tid = threadIdx.x;
        T *lx = reinterpret_cast<T *>(smem);
        T *ly = lx + NE * CMAX;
        T *lz = lx + 2 * NE * CMAX;
        const T *__restrict__ ep = static_cast<const T *>(tp.elem);
        const int64_t es = tp.estride;
        // ---- one round of requests
        T cst[EPT][NP];
        int wp[EPT][NE];
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            const int e = tid + j * BLOCK;
            if (e < ch.elem_count) {
                const T *src = ep + ch.elem_begin + e;
#pragma unroll
                for (int q = 0; q < NP; q++) cst[j][q] = __builtin_nontemporal_load(src + q * es);
                const uint16_t *w = tp.wpos + ch.elem_begin + e;
#pragma unroll
                for (int a = 0; a < NE; a++) wp[j][a] = __builtin_nontemporal_load(w + a * es);
            }
        }
        uint32_t cr[MC], fl[MC];
        int pb[MC];
        T ux[MC][3], upv[MC][3], A[MC];
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            if (i < ch.copy_count) {
                const int l = ch.copy_begin + i;
                cr[m] = tp.crange[l];
                fl[m] = sp.flags[l];
#pragma unroll
                for (int k = 0; k < 3; k++) ux[m][k] = sp.uc[k][l];
                if (i >= ch.n_interior) {
                    pb[m] = tp.pidx[l];
                } else if (MODE == 1) {
#pragma unroll
                    for (int k = 0; k < 3; k++) upv[m][k] = sp.up[k][l];
                    A[m] = sp.acoef[l];
                }
            }
        }
        // loads (BC targets / forces) of interior copies, needed only at the update
        T rv[MC][3];
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
#pragma unroll
            for (int k = 0; k < 3; k++) rv[m][k] = T(0);
            if (MODE == 1 && i < ch.n_interior && (fl[m] & FLAG_RU)) {
                const int l = ch.copy_begin + i;
#pragma unroll
                for (int k = 0; k < 3; k++) rv[m][k] = sp.ru[k][l];
            }
        }
        // ---- scatter u^n over each copy's contiguous incidence range
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            if (i < ch.copy_count) {
                const int b = cr[m] & 0xffffu, n = cr[m] >> 16;
                for (int q = b; q < b + n; q++) {
                    lx[q] = ux[m][0];
                    ly[q] = ux[m][1];
                    lz[q] = ux[m][2];
                }
            }
        }
        __syncthreads();
        // ---- element forces, written back over the element's own positions
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            const int e = tid + j * BLOCK;
            if (e < ch.elem_count) {
                T u[NE][3], F[NE][3];
#pragma unroll
                for (int a = 0; a < NE; a++) {
                    u[a][0] = lx[wp[j][a]];
                    u[a][1] = ly[wp[j][a]];
                    u[a][2] = lz[wp[j][a]];
                }
                const T J = element_force<T, NE, MODEL>(cst[j], u, F);
#pragma unroll
                for (int a = 0; a < NE; a++) {
                    lx[wp[j][a]] = F[a][0];
                    ly[wp[j][a]] = F[a][1];
                    lz[wp[j][a]] = F[a][2];
                }
                // a non-finite force also reaches the node sums, which are checked
                if (!isfinite(J)) {
                    po.bad = DJ_ERR_NONFINITE;
                    po.bad_elem = ch.elem_begin + e;
                } else if (!(J > T(0)) && po.bad == 0) {
                    po.bad = DJ_ERR_INVERTED;
                    po.bad_elem = ch.elem_begin + e;
                }
            }
        }
        __syncthreads();
        // ---- node sums over each copy's range, in fixed order
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            if (i < ch.copy_count) {
                const int b = cr[m] & 0xffffu, n = cr[m] >> 16;
                T f[3] = {T(0), T(0), T(0)};
                for (int q = b; q < b + n; q++) {
                    f[0] += lx[q];
                    f[1] += ly[q];
                    f[2] += lz[q];
                }
                const int l = ch.copy_begin + i;
                if (i >= ch.n_interior) {
                    const int q = pb[m] + int((fl[m] >> FLAG_RANK_SHIFT) & 255u);
                    st_dev(&sp.pp[0][q], f[0]);
                    st_dev(&sp.pp[1][q], f[1]);
                    st_dev(&sp.pp[2][q], f[2]);
                    if (!(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2])) && po.bad == 0) {
                        po.bad = DJ_ERR_NONFINITE;
                        po.bad_elem = -1;
                    }
                } else if constexpr (MODE == 0) {
                    const int nd = tp.cnode[l];
                    sp.fout[3 * nd] = f[0];
                    sp.fout[3 * nd + 1] = f[1];
                    sp.fout[3 * nd + 2] = f[2];
                } else {
                    node_update<T>(l, fl[m], f, ux[m], upv[m], A[m], rv[m], sp, po);
                }
            }
        }
        __syncthreads();  // LDS is reused by the next chunk
    }

    // Round A for the shared copies of up to KB chunks (one per thread per
    // chunk, pass `pass`): everything but the partial sums.  Issued before the
    // grid barrier for the first batch, so its latency hides in the wait.
    template <int MODE, int KB>
    __device__ static void shared_load(const DevTopo &tp, const ChunkDesc *chs, int nb, int pass,
                                       const StepPtrs<T> &sp, SharedRegs<T, KB> &r) {
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            r.ok[kb] = false;
            if (kb < nb) {
                const ChunkDesc &ch = chs[kb];
                const int i = ch.n_interior + threadIdx.x + pass * BLOCK;
                if (i < ch.copy_count) {
                    const int l = ch.copy_begin + i;
                    r.li[kb] = l;
                    r.ok[kb] = true;
                    r.fl[kb] = sp.flags[l];
                    r.pb[kb] = tp.pidx[l];
                    if (MODE == 1) {
                        r.A[kb] = sp.acoef[l];
#pragma unroll
                        for (int k = 0; k < 3; k++) {
                            r.uc[kb][k] = sp.uc[k][l];
                            r.up[kb][k] = sp.up[k][l];
                            r.rv[kb][k] = sp.ru[0] ? sp.ru[k][l] : T(0);
                        }
                    }
                }
            }
        }
    }

    // Round B (the node's partial group) and finish: sum in rank order, then
    // force output (MODE 0, canonical copy) or update (MODE 1).
    template <int MODE, int KB>
    __device__ static void shared_finish(const DevTopo &tp, SharedRegs<T, KB> &r, const StepPtrs<T> &sp,
                                         PhaseOut &po) {
        constexpr int UNR = 4;
        T px[KB][UNR][3];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            if (r.ok[kb]) {
                const int cnt = (r.fl[kb] >> FLAG_NCOPY_SHIFT) & 255u;
#pragma unroll
                for (int q = 0; q < UNR; q++)
                    if (q < cnt)
#pragma unroll
                        for (int k = 0; k < 3; k++) px[kb][q][k] = ld_dev(&sp.pp[k][r.pb[kb] + q]);
            }
        }
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            if (!r.ok[kb]) continue;
            const int cnt = (r.fl[kb] >> FLAG_NCOPY_SHIFT) & 255u;
            T f[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < UNR; q++)
                if (q < cnt)
#pragma unroll
                    for (int k = 0; k < 3; k++) f[k] += px[kb][q][k];
            for (int q = UNR; q < cnt; q++)
#pragma unroll
                for (int k = 0; k < 3; k++) f[k] += ld_dev(&sp.pp[k][r.pb[kb] + q]);
            const int l = r.li[kb];
            if constexpr (MODE == 0) {
                if (r.fl[kb] & FLAG_CANON) {
                    const int nd = tp.cnode[l];
                    sp.fout[3 * nd] = f[0];
                    sp.fout[3 * nd + 1] = f[1];
                    sp.fout[3 * nd + 2] = f[2];
                }
            } else {
                if (!(r.fl[kb] & FLAG_RU))
#pragma unroll
                    for (int k = 0; k < 3; k++) r.rv[kb][k] = T(0);
                node_update<T>(l, r.fl[kb], f, r.uc[kb], r.up[kb], r.A[kb], r.rv[kb], sp, po);
            }
        }
    }

    // all passes of one batch of chunks
    template <int MODE, int KB>
    __device__ static void shared_batch(const DevTopo &tp, const ChunkDesc *chs, int nb, int first_pass,
                                        const StepPtrs<T> &sp, PhaseOut &po) {
        for (int pass = first_pass;; pass++) {
            bool more = false;
            for (int kb = 0; kb < nb; kb++) more |= chs[kb].n_interior + pass * BLOCK < chs[kb].copy_count;
            if (!more) break;
            SharedRegs<T, KB> r;
            shared_load<MODE, KB>(tp, chs, nb, pass, sp, r);
            shared_finish<MODE, KB>(tp, r, sp, po);
        }
    }
};

// ---------------------------------------------------------------------------
// block-wide sum of two doubles in a fixed order (result valid in thread 0)
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ __forceinline__ void block_sum2(double &x, double &y, double *sred) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        x += __shfl_xor(x, o, 64);
        y += __shfl_xor(y, o, 64);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
        sred[2 * w] = x;
        sred[2 * w + 1] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int i = 0; i < BLOCK / 64; i++) {
            a += sred[2 * i];
            b += sred[2 * i + 1];
        }
        x = a;
        y = b;
    }
}

// ---------------------------------------------------------------------------
// Cross-workgroup communication.  On gfx950 the L2 of each XCD is not coherent
// with the others, and agent-scope fences write back / invalidate whole L2s
// (tens of microseconds with hundreds of workgroups).  So every value one
// workgroup publishes to another (partial node forces, residual partials,
// flags) is stored and loaded with device-scope relaxed atomics, which write
// through to and read from the coherence point; a thread waits for its own
// stores to be acknowledged before its workgroup signals arrival.
// ---------------------------------------------------------------------------

constexpr unsigned SPIN_LIMIT = 1u << 24;
constexpr int N_RELEASE = 16;   // release-flag copies, one cache line apart
constexpr int FLAG_STRIDE = 32; // uint32 per flag slot (128 B)

// Grid barrier for the persistent kernel (all workgroups co-resident through
// a cooperative launch).  Arrival: one flag per workgroup; workgroup 0 polls
// them all and then raises N_RELEASE release flags.  Bounded spins: a broken
// co-residency ends in DJ_ERR_BARRIER instead of a hang.
//   sync[0 .. G*FLAG_STRIDE)        arrival flags
//   sync[G*FLAG_STRIDE ...)         release flags
//   status[4]                       abort flag
__device__ __forceinline__ bool grid_barrier(uint32_t *sync, uint32_t nblocks, uint32_t &epoch, int32_t *status) {
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);  // this thread's published stores are complete
    __syncthreads();
    const uint32_t target = epoch + 1u;
    uint32_t *rel = sync + size_t(nblocks) * FLAG_STRIDE;
    if (threadIdx.x == 0) {
        s_ok = 1;
        st_dev(&sync[size_t(blockIdx.x) * FLAG_STRIDE], target);
    }
    if (blockIdx.x == 0) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nblocks; i += blockDim.x) {
            unsigned spins = 0;
            while (ld_dev(&sync[size_t(i) * FLAG_STRIDE]) != target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > SPIN_LIMIT || ld_dev(&status[4]) != 0) {
                    st_dev(&status[4], 1);
                    s_ok = 0;
                    break;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < N_RELEASE && s_ok) st_dev(&rel[threadIdx.x * FLAG_STRIDE], target);
    } else if (threadIdx.x == 0) {
        const uint32_t *r = &rel[(blockIdx.x % N_RELEASE) * FLAG_STRIDE];
        unsigned spins = 0;
        while (ld_dev(r) != target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT || ld_dev(&status[4]) != 0) {
                st_dev(&status[4], 1);
                s_ok = 0;
                break;
            }
        }
    }
    __syncthreads();
    epoch = target;
    return s_ok != 0;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// copies <- caller arrays (both state vectors at once when src1 != null)
template <typename T>
__global__ void k_scatter_in(const int32_t *__restrict__ cnode, int n_copies, const T *__restrict__ src0,
                             const T *__restrict__ src1, T *__restrict__ d0, T *__restrict__ d1) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_copies) return;
    const int n = cnode[l];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        d0[int64_t(k) * n_copies + l] = src0[3 * n + k];
        if (src1) d1[int64_t(k) * n_copies + l] = src1[3 * n + k];
    }
}

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
constexpr int KMAX = 32;  // chunks per workgroup

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC>
__global__ void __launch_bounds__(BLOCK) k_step(DevTopo tp, StepArgs a) {
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
    for (int k = threadIdx.x; k < nmine; k += BLOCK) s_ch[k] = tp.chunks[blockIdx.x + k * G];
    __syncthreads();
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
            sp.pp[k] = part + ((s & 1) * 3 + k) * NPART;
            sp.ru[k] = ru ? ru + k * L : nullptr;
        }
        sp.flags = a.flags;
        sp.acoef = static_cast<const T *>(tp.acoef);
        sp.bprime = T(a.bprime);
        sp.sval = T(ramp_value(a.ramp, double(n + 1) * a.dt, a.t_ramp));
        sp.want_res = check;
        sp.fout = nullptr;
        PhaseOut po{0.0, 0.0, 0, -1};
        for (int k = 0; k < nmine; k++) C::template element_phase<1>(tp, s_ch[k], sp, smem, po);
        // round A of the first batch of shared copies, in flight during the barrier
        SharedRegs<T, KB> sr;
        C::template shared_load<1, KB>(tp, s_ch, min(KB, nmine), 0, sp, sr);
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
        for (int k0 = 0; k0 < nmine; k0 += KB)
            C::template shared_batch<1, KB>(tp, s_ch + k0, min(KB, nmine - k0), k0 == 0 ? 1 : 0, sp, po);
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
                const double r = sy > 0.0 ? sqrt(sx) / sqrt(sy) : (sx > 0.0 ? INFINITY : 0.0);
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
    for (int k = 0; k < nmine; k++) {
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

// ---------------------------------------------------------------------------
// Pre-computation (Algorithm 1) in FP64, one thread per element
// ---------------------------------------------------------------------------
__device__ __forceinline__ double det3d(const double m[3][3]) {
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

__device__ __forceinline__ double tri_area(const double *p, const double *q, const double *r) {
    const double u0 = q[0] - p[0], u1 = q[1] - p[1], u2 = q[2] - p[2];
    const double v0 = r[0] - p[0], v1 = r[1] - p[1], v2 = r[2] - p[2];
    const double w0 = u1 * v2 - u2 * v1, w1 = u2 * v0 - u0 * v2, w2 = u0 * v1 - u1 * v0;
    return 0.5 * sqrt(w0 * w0 + w1 * w1 + w2 * w2);
}

template <typename T, int NE, int MODEL>
__global__ void k_precompute(const double *__restrict__ X, const int32_t *__restrict__ conn, int E,
                             const double *__restrict__ Ein, const double *__restrict__ nuin,
                             const double *__restrict__ etar, const double *__restrict__ fib, double hg_kappa,
                             double rho, T *__restrict__ planes, int64_t es, double *__restrict__ V64,
                             double *__restrict__ jinv64, unsigned long long *__restrict__ dtmin,
                             int32_t *__restrict__ bad) {
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
    double eta = 0.0;
    if (MODEL == DJ_TI) {
        double a0 = fib[3 * int64_t(e)], a1 = fib[3 * int64_t(e) + 1], a2 = fib[3 * int64_t(e) + 2];
        const double nrm = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        if (!(nrm > 0.0)) {
            atomicAdd(bad, 1);
            return;
        }
        eta = etar[e] * mu;
        planes[(P::FIB + 0) * es + e] = T(a0 / nrm);
        planes[(P::FIB + 1) * es + e] = T(a1 / nrm);
        planes[(P::FIB + 2) * es + e] = T(a2 / nrm);
        planes[P::ETAV * es + e] = T(eta * V);
    }
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
        planes[P::KHG * es + e] = T(hg_kappa * (ka + 4.0 * mu / 3.0) * V * sb / 8.0);
        L = 1.0 / sqrt(2.0 * sb);
    }
    const double cw = sqrt((ka + 4.0 * mu / 3.0 + 4.0 * eta) / rho);
    const double dte = L / cw;
    // positive doubles order like their bit patterns
    atomicMin(dtmin, __double_as_longlong(dte));
}

__global__ void k_node_mass(const int32_t *__restrict__ off, const int32_t *__restrict__ lst, int n_nodes, int ne,
                            double rho, const double *__restrict__ V64, double *__restrict__ mass) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    double m = 0.0;
    for (int j = off[n]; j < off[n + 1]; j++) m += rho * V64[lst[j]] / ne;
    mass[n] = m;
}

template <typename T>
__global__ void k_acoef(const int32_t *__restrict__ inode, int n_copies, const double *__restrict__ mass, double c2,
                        T *__restrict__ acoef) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_copies) return;
    acoef[l] = T(c2 / mass[inode[l]]);
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

// clears the barrier flags and the status words before a persistent launch
// (a kernel rather than a memset, so that the sequence can be graph-captured)
__global__ void k_reset_sync(uint32_t *sync, int n_sync, int32_t *status) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_sync; i += gridDim.x * blockDim.x) sync[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x < 8) status[threadIdx.x] = threadIdx.x == 2 ? -1 : 0;
}

// ---------------------------------------------------------------------------
// Dispatch over (precision, element type, model, variant)
// ---------------------------------------------------------------------------

template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC>
struct Inst {
    using C = Chunk<T, NE, MODEL, BLOCK, EPT, MC>;
    static hipError_t occ(int *bpc, size_t *lds) {
        *lds = C::LDS;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(bpc, k_step<T, NE, MODEL, BLOCK, EPT, MC>, BLOCK, C::LDS);
    }
    static hipError_t forces(Ctx &c, const void *u, void *f, hipStream_t s) {
        const int L = c.topo.n_copies, B = 256;
        T *u0 = static_cast<T *>(c.d_ubuf[0]);
        hipLaunchKernelGGL(k_scatter_in<T>, dim3((L + B - 1) / B), dim3(B), 0, s, c.topo.cnode, L,
                           static_cast<const T *>(u), static_cast<const T *>(nullptr), u0, static_cast<T *>(nullptr));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        StepPtrs<T> sp{};
        T *part = static_cast<T *>(c.d_part);
        for (int k = 0; k < 3; k++) {
            sp.uc[k] = u0 + int64_t(k) * L;
            sp.up[k] = nullptr;
            sp.un[k] = nullptr;
            sp.pp[k] = part + int64_t(k) * std::max(c.topo.n_part, 1);
            sp.ru[k] = nullptr;
        }
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
    static hipError_t step(Ctx &c, const StepArgs &a, const void *u_cur_in, const void *u_prev_in, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
        const int L = c.topo.n_copies, B = 256;
        const int n_sync = (c.grid + N_RELEASE) * FLAG_STRIDE;
        hipLaunchKernelGGL(k_reset_sync, dim3((n_sync + 255) / 256), dim3(256), 0, s, c.d_bar, n_sync, c.d_status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        T *dcur = static_cast<T *>(c.d_ubuf[a.cur0]);
        T *dprev = static_cast<T *>(c.d_ubuf[(a.cur0 + 2) % 3]);
        hipLaunchKernelGGL(k_scatter_in<T>, dim3((L + B - 1) / B), dim3(B), 0, s, c.topo.cnode, L,
                           static_cast<const T *>(u_cur_in), static_cast<const T *>(u_prev_in), dcur, dprev);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        DevTopo tp = c.topo;
        StepArgs aa = a;
        void *args[] = {&tp, &aa};
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_step<T, NE, MODEL, BLOCK, EPT, MC>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(C::LDS));
        if (e != hipSuccess) return e;
        if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return e;
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_step<T, NE, MODEL, BLOCK, EPT, MC>),
                                       dim3(c.grid), dim3(BLOCK), args, C::LDS, s);
        if (e != hipSuccess) return e;
        if (ev1) e = hipEventRecord(ev1, s);
        return e;
    }
};

// Kernel variants per (precision, element type): {threads, elements per thread, copies per thread}
constexpr Variant VAR_T4F[4] = {{256, 4, 2}, {256, 2, 2}, {512, 2, 2}, {128, 4, 2}};
constexpr Variant VAR_H8F[4] = {{256, 2, 4}, {256, 1, 4}, {512, 1, 3}, {128, 2, 4}};
constexpr Variant VAR_T4D[4] = {{256, 2, 2}, {256, 1, 2}, {512, 1, 2}, {128, 2, 2}};
constexpr Variant VAR_H8D[4] = {{256, 1, 4}, {128, 1, 4}, {512, 1, 3}, {128, 2, 4}};

template <typename T, int NE>
constexpr const Variant *var_table() {
    return sizeof(T) == 4 ? (NE == 4 ? VAR_T4F : VAR_H8F) : (NE == 4 ? VAR_T4D : VAR_H8D);
}

template <typename T, int NE, int MODEL, int V>
using InstV = Inst<T, NE, MODEL, var_table<T, NE>()[V].block, var_table<T, NE>()[V].ept, var_table<T, NE>()[V].mcopy>;

template <typename T, int NE, int MODEL, typename F>
static hipError_t with_variant(int v, F &&f) {
    switch (v) {
        case 0: return f(InstV<T, NE, MODEL, 0>());
        case 1: return f(InstV<T, NE, MODEL, 1>());
        case 2: return f(InstV<T, NE, MODEL, 2>());
        case 3: return f(InstV<T, NE, MODEL, 3>());
        default: return hipErrorInvalidValue;
    }
}

template <typename F>
static hipError_t dispatch(int prec, int ne, int model, int v, F &&f) {
    if (prec == DJ_FP32) {
        if (ne == 4) return model == DJ_NH ? with_variant<float, 4, DJ_NH>(v, f) : with_variant<float, 4, DJ_TI>(v, f);
        return model == DJ_NH ? with_variant<float, 8, DJ_NH>(v, f) : with_variant<float, 8, DJ_TI>(v, f);
    }
    if (ne == 4) return model == DJ_NH ? with_variant<double, 4, DJ_NH>(v, f) : with_variant<double, 4, DJ_TI>(v, f);
    return model == DJ_NH ? with_variant<double, 8, DJ_NH>(v, f) : with_variant<double, 8, DJ_TI>(v, f);
}

const std::vector<Variant> &variants(int ne, int prec) {
    static const std::vector<Variant> t4f(VAR_T4F, VAR_T4F + 4), h8f(VAR_H8F, VAR_H8F + 4);
    static const std::vector<Variant> t4d(VAR_T4D, VAR_T4D + 4), h8d(VAR_H8D, VAR_H8D + 4);
    if (prec == DJ_FP32) return ne == 4 ? t4f : h8f;
    return ne == 4 ? t4d : h8d;
}

hipError_t occupancy(int ne, int model, int prec, int variant, int *blocks_per_cu, size_t *lds_bytes) {
    return dispatch(prec, ne, model, variant, [&](auto inst) { return decltype(inst)::occ(blocks_per_cu, lds_bytes); });
}

hipError_t launch_forces(Ctx &c, const void *u, void *f, hipStream_t s) {
    return dispatch(c.prec, c.ne, c.model, c.variant, [&](auto inst) { return decltype(inst)::forces(c, u, f, s); });
}

hipError_t launch_step(Ctx &c, const StepArgs &a, const void *u_cur_in, const void *u_prev_in, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
    return dispatch(c.prec, c.ne, c.model, c.variant,
                    [&](auto inst) { return decltype(inst)::step(c, a, u_cur_in, u_prev_in, s, ev0, ev1); });
}

template <typename T>
static hipError_t precompute_t(Ctx &c, const double *dX, const int32_t *dconn, const double *dE, const double *dnu,
                               const double *deta, const double *dfib, double *d_dtmin, int32_t *d_bad, hipStream_t s) {
    const int B = 256, G = (c.n_elems + B - 1) / B;
    T *planes = static_cast<T *>(c.d_elem);
    auto *dtm = reinterpret_cast<unsigned long long *>(d_dtmin);
    const int64_t es = c.topo.estride;
    if (c.ne == 4 && c.model == DJ_NH)
        hipLaunchKernelGGL((k_precompute<T, 4, DJ_NH>), dim3(G), dim3(B), 0, s, dX, dconn, c.n_elems, dE, dnu, deta,
                           dfib, c.hg_kappa, c.rho, planes, es, c.d_V64, c.d_jinv64, dtm, d_bad);
    else if (c.ne == 4)
        hipLaunchKernelGGL((k_precompute<T, 4, DJ_TI>), dim3(G), dim3(B), 0, s, dX, dconn, c.n_elems, dE, dnu, deta,
                           dfib, c.hg_kappa, c.rho, planes, es, c.d_V64, c.d_jinv64, dtm, d_bad);
    else if (c.model == DJ_NH)
        hipLaunchKernelGGL((k_precompute<T, 8, DJ_NH>), dim3(G), dim3(B), 0, s, dX, dconn, c.n_elems, dE, dnu, deta,
                           dfib, c.hg_kappa, c.rho, planes, es, c.d_V64, c.d_jinv64, dtm, d_bad);
    else
        hipLaunchKernelGGL((k_precompute<T, 8, DJ_TI>), dim3(G), dim3(B), 0, s, dX, dconn, c.n_elems, dE, dnu, deta,
                           dfib, c.hg_kappa, c.rho, planes, es, c.d_V64, c.d_jinv64, dtm, d_bad);
    return hipGetLastError();
}

hipError_t launch_precompute(Ctx &c, const double *dX, const int32_t *dconn, const double *dE, const double *dnu,
                             const double *deta, const double *dfib, double *d_dtmin, int32_t *d_bad, hipStream_t s) {
    if (c.prec == DJ_FP32) return precompute_t<float>(c, dX, dconn, dE, dnu, deta, dfib, d_dtmin, d_bad, s);
    return precompute_t<double>(c, dX, dconn, dE, dnu, deta, dfib, d_dtmin, d_bad, s);
}

hipError_t launch_mass_acoef(Ctx &c, const int32_t *d_ne_off, const int32_t *d_ne_list, hipStream_t s) {
    const int B = 256;
    hipLaunchKernelGGL(k_node_mass, dim3((c.n_nodes + B - 1) / B), dim3(B), 0, s, d_ne_off, d_ne_list, c.n_nodes, c.ne,
                       c.rho, c.d_V64, c.d_mass64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double c2 = 2.0 * c.dt * c.dt / (2.0 + c.alpha * c.dt);
    const int G = (c.topo.n_copies + B - 1) / B;
    if (c.prec == DJ_FP32)
        hipLaunchKernelGGL(k_acoef<float>, dim3(G), dim3(B), 0, s, c.d_inode, c.topo.n_copies, c.d_mass64, c2,
                           static_cast<float *>(c.d_acoef));
    else
        hipLaunchKernelGGL(k_acoef<double>, dim3(G), dim3(B), 0, s, c.d_inode, c.topo.n_copies, c.d_mass64, c2,
                           static_cast<double *>(c.d_acoef));
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
