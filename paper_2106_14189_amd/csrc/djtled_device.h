// Device code shared by the DJ-TLED kernel translation units: element force,
// chunk phases, node update, grid barrier.
//
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
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "djtled_internal.h"

namespace dj {

// Sub-phase timers of the step kernels, compiled only into a separate
// instrumented build (-DDJ_INSTR): thread 0 of each workgroup adds wall-clock
// ticks (100 MHz) of each phase into its 16 counters.
#ifdef DJ_INSTR
static __device__ unsigned long long *dj_instr_buf;
__device__ __forceinline__ void instr_add(int k, unsigned long long v) {
    if (threadIdx.x == 0 && dj_instr_buf) dj_instr_buf[blockIdx.x * 16 + k] += v;
}
#define INSTR_T(x) const unsigned long long x = wall_clock64()
#else
#define INSTR_T(x)
#endif

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

__device__ __forceinline__ double det3d(const double m[3][3]) {
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

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

// cache-policy bit of a buffer access for device-scope coherence (gfx950: SC1)
constexpr int CPOL_SC1 = 16;

// Partial node forces of single meshes: three planes (x, y, z) over the
// partial entries of one step parity; each component is published and read
// with a device-scope access.  Entries of neighbouring nodes are adjacent in
// each plane, so a wave's stores of one component fall on few cache lines.
// (One 16-byte entry per partial, read as two 64-bit words, measured no
// faster.)
template <typename T>
__device__ __forceinline__ void put_partial(T *const (&pp)[3], int q, const T (&f)[3]) {
#pragma unroll
    for (int k = 0; k < 3; k++) st_dev(&pp[k][q], f[k]);
}
template <typename T>
__device__ __forceinline__ void get_partial(T *const (&pp)[3], int q, T (&f)[3]) {
#pragma unroll
    for (int k = 0; k < 3; k++) f[k] = ld_dev(&pp[k][q]);
}

// Batches keep a partial entry's three components together (pp[0] = the
// parity's first entry, component k of entry q at 3 q + k).  In FP32 one
// 12-byte buffer access with the same cache policy as the device-scope
// relaxed atomics (sc1: through to the coherence point) moves an entry.
template <bool AOS, typename T>
__device__ __forceinline__ void put_partial3(T *const (&pp)[3], int q, const T (&f)[3]) {
    if constexpr (AOS && sizeof(T) == 4) {
        typedef float f3v __attribute__((ext_vector_type(3)));
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(pp[0], 0, 0xffffffff, 0x00020000);
        f3v v;
        v.x = f[0];
        v.y = f[1];
        v.z = f[2];
        __builtin_amdgcn_raw_buffer_store_b96(v, r, 12 * q, 0, CPOL_SC1);
    } else if constexpr (AOS) {
#pragma unroll
        for (int k = 0; k < 3; k++) st_dev(&pp[0][3 * int64_t(q) + k], f[k]);
    } else {
        put_partial(pp, q, f);
    }
}
template <bool AOS, typename T>
__device__ __forceinline__ void get_partial3(T *const (&pp)[3], int q, T (&f)[3]) {
    if constexpr (AOS && sizeof(T) == 4) {
        typedef float f3v __attribute__((ext_vector_type(3)));
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(pp[0], 0, 0xffffffff, 0x00020000);
        const f3v v = __builtin_amdgcn_raw_buffer_load_b96(r, 12 * q, 0, CPOL_SC1);
        f[0] = v.x;
        f[1] = v.y;
        f[2] = v.z;
    } else if constexpr (AOS) {
#pragma unroll
        for (int k = 0; k < 3; k++) f[k] = ld_dev(&pp[0][3 * int64_t(q) + k]);
    } else {
        get_partial(pp, q, f);
    }
}

// Displacement of copy l in one of the rotating state buffers.  Single meshes
// keep three planes (p[k] = plane k); batches keep the three components of a
// copy together (p[0] = buffer start, component k of copy l at 3 l + k), so
// that one 12-byte access moves a copy's vector.
template <bool AOS, typename T>
__device__ __forceinline__ void ld_u3(const T *const (&p)[3], int l, T (&v)[3]) {
    if constexpr (AOS) {
        const T *q = p[0] + 3 * int64_t(l);
#pragma unroll
        for (int k = 0; k < 3; k++) v[k] = q[k];
    } else {
#pragma unroll
        for (int k = 0; k < 3; k++) v[k] = p[k][l];
    }
}
template <bool AOS, typename T>
__device__ __forceinline__ void st_u3(T *const (&p)[3], int l, const T (&v)[3]) {
    if constexpr (AOS) {
        T *q = p[0] + 3 * int64_t(l);
#pragma unroll
        for (int k = 0; k < 3; k++) q[k] = v[k];
    } else {
#pragma unroll
        for (int k = 0; k < 3; k++) p[k][l] = v[k];
    }
}

// ---------------------------------------------------------------------------
// element force (register-resident).  cst: the element's planes.  u: nodal
// displacements.  F: nodal forces.  Returns J.
// ---------------------------------------------------------------------------
// Classical TLED (Eq. 4 with the second Piola-Kirchhoff stress of each
// model), for comparison with the Table 3 force: deformation gradient
// X = I + D^T, C = X^T X, C^-1 from its cofactors, the invariants of Table 1,
// S 0V from the decoupled strain energies of Table 3, and M = X S 0V 0J^-1.
// Evaluated literally: its O(1) terms cancel to an O(strain) force.
template <typename T, int NE, int MD>
__device__ __forceinline__ T tled_stress_m(const T *__restrict__ cst, const T (&D)[3][3], T (&M)[3][3]) {
    using P = Planes<NE, MD>;
    T X[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) X[i][j] = (i == j ? T(1) : T(0)) + D[j][i];
    const T J = X[0][0] * (X[1][1] * X[2][2] - X[1][2] * X[2][1]) - X[0][1] * (X[1][0] * X[2][2] - X[1][2] * X[2][0]) +
                X[0][2] * (X[1][0] * X[2][1] - X[1][1] * X[2][0]);
    T C[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) C[i][j] = X[0][i] * X[0][j] + X[1][i] * X[1][j] + X[2][i] * X[2][j];
    T Ci[3][3];  // adj(C) / det C
    Ci[0][0] = C[1][1] * C[2][2] - C[1][2] * C[2][1];
    Ci[0][1] = C[0][2] * C[2][1] - C[0][1] * C[2][2];
    Ci[0][2] = C[0][1] * C[1][2] - C[0][2] * C[1][1];
    Ci[1][0] = C[1][2] * C[2][0] - C[1][0] * C[2][2];
    Ci[1][1] = C[0][0] * C[2][2] - C[0][2] * C[2][0];
    Ci[1][2] = C[0][2] * C[1][0] - C[0][0] * C[1][2];
    Ci[2][0] = C[1][0] * C[2][1] - C[1][1] * C[2][0];
    Ci[2][1] = C[0][1] * C[2][0] - C[0][0] * C[2][1];
    Ci[2][2] = C[0][0] * C[1][1] - C[0][1] * C[1][0];
    const T rdet = dj_rcp(C[0][0] * Ci[0][0] + C[0][1] * Ci[1][0] + C[0][2] * Ci[2][0]);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) Ci[i][j] *= rdet;
    const T I1 = C[0][0] + C[1][1] + C[2][2];
    const T c = dj_cbrt(J);
    const T Jm23 = dj_rcp(c * c);
    const T muV = cst[P::MUV], kaV = cst[P::KAV];
    // S 0V = J^-2/3 (mu I + 2 d4 a a^T + 2 d6 b b^T) + 2 C01 J^-4/3 (I1 I - C) + p C^-1
    T W[3][3];  // the part multiplying J^-2/3
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) W[i][j] = (i == j ? muV : T(0));
    T pV = -(muV * T(1.0 / 3.0)) * Jm23 * I1 + kaV * J * (J - T(1));
    auto fibre = [&](const T *fv, T etaV) {
        const T f[3] = {fv[0], fv[1], fv[2]};
        T Cf[3];
#pragma unroll
        for (int i = 0; i < 3; i++) Cf[i] = C[i][0] * f[0] + C[i][1] * f[1] + C[i][2] * f[2];
        const T Ib = Jm23 * (f[0] * Cf[0] + f[1] * Cf[1] + f[2] * Cf[2]);
        const T dV = etaV * (Ib - T(1));
        pV -= T(2.0 / 3.0) * dV * Ib;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) W[i][j] += T(2) * dV * f[i] * f[j];
    };
    if constexpr (MD == DJ_TI || MD == DJ_OT) fibre(cst + P::FIB, cst[P::ETAV]);
    if constexpr (MD == DJ_OT) fibre(cst + P::FIBB, cst[P::ETABV]);
    T SV[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) SV[i][j] = Jm23 * W[i][j];
    if constexpr (MD == DJ_MR) {
        const T c01V = cst[P::C01V], Jm43 = Jm23 * Jm23;
        T trC2 = 0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) trC2 += C[i][j] * C[j][i];
        const T I2 = T(0.5) * (I1 * I1 - trC2);
        pV -= T(4.0 / 3.0) * c01V * Jm43 * I2;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) SV[i][j] += T(2) * c01V * Jm43 * ((i == j ? I1 : T(0)) - C[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) SV[i][j] += pV * Ci[i][j];
    const T *Ji = cst + P::JINV;
    T Q[3][3];  // X S 0V
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int j = 0; j < 3; j++) Q[k][j] = X[k][0] * SV[0][j] + X[k][1] * SV[1][j] + X[k][2] * SV[2][j];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) M[i][j] = Q[i][0] * Ji[j] + Q[i][1] * Ji[3 + j] + Q[i][2] * Ji[6 + j];
    return J;
}

// J - 1 of an element at displacement u (Eq. 12 in the increment form used by
// element_force: D = 0J^-1 H_xi Ue, J - 1 = tr D + (tr^2 D - tr D^2) / 2 + det D)
template <typename T, int NE, int MODEL>
__device__ __forceinline__ T element_jm1(const T *__restrict__ cst, const T (&u)[NE][3]) {
    using P = Planes<NE, MODEL>;
    T dJ[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            if constexpr (NE == 4) {
                dJ[i][k] = u[i + 1][k] - u[0][k];
            } else {
                T s = 0;
#pragma unroll
                for (int a = 1; a < 8; a++) s += (h8s(a, i) > 0) ? (u[a][k] - u[0][k]) : -(u[a][k] - u[0][k]);
                dJ[i][k] = s * T(0.125);
            }
        }
    const T *Ji = cst + P::JINV;
    T D[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) D[i][k] = Ji[3 * i] * dJ[0][k] + Ji[3 * i + 1] * dJ[1][k] + Ji[3 * i + 2] * dJ[2][k];
    const T trD = D[0][0] + D[1][1] + D[2][2];
    T trD2 = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) trD2 += D[i][j] * D[j][i];
    const T detD = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) - D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                   D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    return trD + T(0.5) * (trD * trD - trD2) + detD;
}

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
    constexpr int MD = base_model(MODEL);
    T M[3][3];
    T J;
    if constexpr ((MODEL & DJ_FORM_TLED) != 0) {
        J = tled_stress_m<T, NE, MD>(cst, D, M);
    } else {
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
        J = T(1) + Jm1;
        const T I1m3 = T(2) * trD + nD2;                          // I1 - 3 (Eq. 27)
        const T c = dj_cbrt(J);
        const T Jm23 = dj_rcp(c * c);                             // J^-2/3
        const T muV = cst[P::MUV], kaV = cst[P::KAV];
        // (mu J^-2/3 + p) 0V; with ANP the kappa plane holds pbar 0V, pbar = dPsi_vol/dJ
        T c0 = -(muV * T(1.0 / 3.0)) * Jm23 * I1m3 + ((MODEL & DJ_FORM_ANP) ? J * kaV : kaV * J * Jm1);
        T ciso = muV * Jm23;                                          // the O(1) identity part of c0 - p 0V
        T Q[3][3];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) Q[i][k] = muV * Jm23 * D[k][i];
        // fibre terms (TI: a; OT: a and b): 2 J^-2/3 psi 0V (f + D^T f) f^T, psi = eta (Ibar - 1)
        auto fibre_term = [&](const T *fv, T etaV) {
            const T f[3] = {fv[0], fv[1], fv[2]};
            T Dtf[3];
#pragma unroll
            for (int k = 0; k < 3; k++) Dtf[k] = D[0][k] * f[0] + D[1][k] * f[1] + D[2][k] * f[2];
            const T fDf = f[0] * Dtf[0] + f[1] * Dtf[1] + f[2] * Dtf[2];
            const T Im1 = T(2) * fDf + Dtf[0] * Dtf[0] + Dtf[1] * Dtf[1] + Dtf[2] * Dtf[2];  // I4 - 1 (Eq. 31, 32)
            const T Jm23m1 = -Jm1 * (c + T(1)) * dj_rcp(c * c * (c * c + c + T(1)));     // J^-2/3 - 1
            const T Ibm1 = Jm23 * Im1 + Jm23m1;                                             // Ibar - 1
            const T psiV = etaV * Ibm1;
            c0 -= T(2.0 / 3.0) * psiV * (T(1) + Ibm1);
            const T w = T(2) * Jm23 * psiV;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int k = 0; k < 3; k++) Q[i][k] += w * (f[i] + Dtf[i]) * f[k];
        };
        if constexpr (MD == DJ_TI || MD == DJ_OT) fibre_term(cst + P::FIB, cst[P::ETAV]);
        if constexpr (MD == DJ_OT) fibre_term(cst + P::FIBB, cst[P::ETABV]);
        if constexpr (MD == DJ_MR) {
            // C01 term: 2 C01 0V J^-4/3 (I + D^T)(I1 I - C) with C = I + G, G = D + D^T + D D^T;
            // its identity part 4 C01 0V J^-4/3 joins c0, the rest is O(strain)
            const T c01V = cst[P::C01V];
            const T Jm43 = Jm23 * Jm23;
            T G[3][3];
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    G[i][j] = D[i][j] + D[j][i] + D[i][0] * D[j][0] + D[i][1] * D[j][1] + D[i][2] * D[j][2];
            T trG2 = 0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) trG2 += G[i][j] * G[i][j];
            const T I2m3 = T(2) * I1m3 + T(0.5) * (I1m3 * I1m3 - trG2);  // I2 - 3 (Eq. 28)
            const T w = T(2) * c01V * Jm43;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const T DtG = D[0][i] * G[0][k] + D[1][i] * G[1][k] + D[2][i] * G[2][k];
                    Q[i][k] += w * (T(2) * D[k][i] + I1m3 * ((i == k ? T(1) : T(0)) + D[k][i]) - G[i][k] - DtG);
                }
            c0 -= T(4.0 / 3.0) * c01V * Jm43 * I2m3;  // p_MR 0V + 4 C01 0V J^-4/3
            ciso += T(4) * c01V * Jm43;
        }
        const T pJ = (c0 - ciso) * dj_rcp(J);  // p 0V / J
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
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) M[i][j] = Q[i][0] * Ji[j] + Q[i][1] * Ji[3 + j] + Q[i][2] * Ji[6 + j];

    }
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
    // batches (per-copy coefficients): B' per copy, ramp rate per loaded copy
    const T *bpc;
    const T *rrate;
    T n1;             // n + 1
    // average nodal pressure step: per-copy nodal pressure p_n (force pass; null otherwise)
    const T *pn;
};

struct PhaseOut {
    double num, den;  // residual partial sums over canonical copies
    int bad;          // 0, DJ_ERR_INVERTED or DJ_ERR_NONFINITE
    int bad_elem;     // internal element index; -2 - copy for a node-level error
};

// Ramp value of a batch instance at step n + 1 from its rate q = dt / t_ramp
// stored with the ramp kind in the sign (+ smooth, - linear; 0: no ramp).
// Same polynomial as ramp_value.
template <typename T>
__device__ __forceinline__ T ramp_rate(T q, T n1) {
    if (q == T(0)) return T(1);
    const T tau = (q < T(0) ? -q : q) * n1;
    if (tau >= T(1)) return T(1);
    if (q < T(0)) return tau;
    return tau * tau * tau * (T(10) - T(15) * tau + T(6) * tau * tau);
}

// u^{n+1} = u^n + B'(u^n - u^{n-1}) + A (R - F); prescribed components = s(t) target
template <typename T>
__device__ __forceinline__ void node_value(int l, uint32_t fl, const T (&f)[3], const T (&uc)[3], const T (&up)[3],
                                           T A, T bp, T sv, const T (&rv)[3], const StepPtrs<T> &sp, PhaseOut &po,
                                           T (&un)[3]) {
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const bool pres = (fl >> k) & 1u;
        if (pres) {
            un[k] = sv * rv[k];
            if (sp.want_res && (fl & FLAG_CANON)) po.den += double(f[k]) * double(f[k]);
        } else {
            un[k] = uc[k] + bp * (uc[k] - up[k]) + A * (rv[k] - f[k]);
            if (sp.want_res && (fl & FLAG_CANON)) {
                const double d = double(f[k]) - double(rv[k]);
                po.num += d * d;
            }
        }
        fin = fin && isfinite(un[k]);
    }
    if (!fin && po.bad == 0) {
        po.bad = DJ_ERR_NONFINITE;
        po.bad_elem = -2 - l;  // node-level error: the copy
    }
}
template <typename T, bool AOS = false>
__device__ __forceinline__ void node_update(int l, uint32_t fl, const T (&f)[3], const T (&uc)[3], const T (&up)[3],
                                            T A, T bp, T sv, const T (&rv)[3], const StepPtrs<T> &sp,
                                            PhaseOut &po) {
    T un[3];
    node_value<T>(l, fl, f, uc, up, A, bp, sv, rv, sp, po, un);
    st_u3<AOS>(sp.un, l, un);
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
    T uc[KB][3], up[KB][3], rv[KB][3], A[KB], bp[KB], rr[KB];
};

struct NoOp {
    __device__ void operator()() const {}
};
struct NoOpJ {
    __device__ void operator()(int) const {}
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// PC: per-copy B' and ramp rates (batches of instances with their own steps).
// PF: the chunk's element planes and slot positions are staged in LDS by
// direct global -> LDS loads issued while the previous chunk is summed
// (prefetch), instead of being loaded into registers at the chunk's start.
template <typename T, int NE, int MODEL, int BLOCK, int EPT, int MC, bool PC = false, bool PF = false>
struct Chunk {
    static constexpr int CMAX = BLOCK * EPT;
    static constexpr int NP = Planes<NE, MODEL>::N;
    // slot plane: the chunk's NE x CMAX incidences and up to one padding slot
    // per copy (each copy's range starts an odd distance after the previous
    // one, so the copies of a wave walk their ranges on distinct LDS banks)
    static constexpr int SP = NE * CMAX + MC * BLOCK;
    static constexpr bool ANPM = (MODEL & DJ_FORM_ANP) != 0;
    // FP32 (not the average-nodal-pressure passes): a slot's x, y, z side by
    // side in one 16-byte entry, so a gather, a scatter or a sum step is one
    // 12-byte LDS access; otherwise three planes of SP slots
    static constexpr bool L4 = sizeof(T) == 4 && !ANPM;
    static constexpr size_t SLOTS = (L4 ? size_t(4) : size_t(3)) * SP * sizeof(T);
    static constexpr int PDW = CMAX * int(sizeof(T)) / 4;  // dwords of one staged plane
    static constexpr int WDW = CMAX / 2 + 2;               // dwords of one staged slot-position plane
    static constexpr size_t STAGE = PF ? size_t(4) * (size_t(NP) * PDW + size_t(NE) * WDW) : 0;
    static constexpr size_t LDS = SLOTS + STAGE;

    // LDS-DMA loads of one chunk's element planes and slot positions into the
    // staging area (dword granularity; each wave takes 64-dword pieces).
    // Completion: s_waitcnt vmcnt + a workgroup barrier before the reads.
    __device__ static void prefetch(const DevTopo &tp, const ChunkDesc &ch, unsigned char *smem) {
        if constexpr (PF) {
            constexpr int NW = BLOCK / 64;
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            uint32_t *stage = reinterpret_cast<uint32_t *>(smem + SLOTS);
            uint32_t *wstage = stage + NP * PDW;
            const int64_t es = tp.estride;
            const int ndw = ch.elem_count * int(sizeof(T)) / 4;
            const uint32_t *src = reinterpret_cast<const uint32_t *>(static_cast<const T *>(tp.elem) + ch.elem_begin);
            const int64_t pstride = es * int64_t(sizeof(T)) / 4;  // dwords between planes
#pragma unroll 1
            for (int q = 0; q < NP; q++, src += pstride) {
#pragma unroll 1
                for (int i = w * 64; i < ndw; i += NW * 64)
                    if (i + lane < ndw)
                        __builtin_amdgcn_global_load_lds((glb_void_t *)(src + i + lane), (lds_void_t *)(stage + q * PDW + i),
                                                         4, 0, 0);
            }
            const int e0 = ch.elem_begin & ~1;
            const int nw = (ch.elem_begin + ch.elem_count - e0 + 1) / 2;
            const uint32_t *wsrc = reinterpret_cast<const uint32_t *>(tp.wpos + e0);
#pragma unroll 1
            for (int a = 0; a < NE; a++, wsrc += es / 2) {
#pragma unroll 1
                for (int i = w * 64; i < nw; i += NW * 64)
                    if (i + lane < nw)
                        __builtin_amdgcn_global_load_lds((glb_void_t *)(wsrc + i + lane), (lds_void_t *)(wstage + a * WDW + i),
                                                         4, 0, 0);
            }
        }
    }

    // Registers of one chunk's element data and of its node copies, so that
    // the loads of the next chunk can be issued while this one is summed.
    struct ElemRegs {
        T cst[EPT][NP];
        int wp[EPT][NE];
    };
    struct CopyRegs {
        uint32_t cr[MC], fl[MC];
        int pb[MC];
        T ux[MC][3], upv[MC][3], A[MC], Bp[MC], rr[MC], rv[MC][3];
        T pn[MC];  // average-nodal-pressure step: the copy's nodal pressure
    };
    // LDS of the average-nodal-pressure step: a fourth slot plane carries p_n
    static constexpr size_t LDS_ANP = LDS + size_t(SP) * sizeof(T);

    // FP32 contexts read the interleaved element copy (elem4): NP + NE / 2
    // words per element in 16-byte loads; the slot positions stay packed two
    // to a word in wp[j][2i] until they are used (slot(), after the chunk's
    // wait).  The average-nodal-pressure step and forces read the planes (the
    // force pass takes a modified kappa plane).
    static constexpr bool PK = !PF && sizeof(T) == 4 && !ANPM;
    static constexpr bool AOS = PC;  // batches: copy displacements as 3-vectors (ld_u3)
    // batches: a copy's (A, B') side by side, and its (load x, y, z, ramp rate)
    struct alignas(2 * sizeof(T)) ABPair {
        T a, b;
    };
    struct alignas(4 * sizeof(T)) RQuad {
        T x, y, z, r;
    };
    __device__ static void ld_ab(const StepPtrs<T> &sp, int l, T &A, T &Bp) {
        const ABPair p = reinterpret_cast<const ABPair *>(sp.acoef)[l];
        A = p.a;
        Bp = p.b;
    }
    __device__ static void ld_rq(const StepPtrs<T> &sp, int l, T (&rv)[3], T &rr) {
        const RQuad q = reinterpret_cast<const RQuad *>(sp.ru[0])[l];
        rv[0] = q.x;
        rv[1] = q.y;
        rv[2] = q.z;
        rr = q.r;
    }
    __device__ static int slot(const ElemRegs &er, int j, int a) {
        if constexpr (PK) return int((uint32_t(er.wp[j][a & ~1]) >> (16 * (a & 1))) & 0xffffu);
        else return er.wp[j][a];
    }

    // Element planes and slot positions (register path).  Lanes past the
    // chunk's end load its last element again: the loads are unconditional, so
    // no lane keeps an older value and nothing waits on them before use.
    __device__ static void load_elem(const DevTopo &tp, const ChunkDesc &ch, ElemRegs &er, int j) {
        if constexpr (PK) {
            constexpr int D = NP + NE / 2, G = D / 4, R = D % 4;
            const int64_t es = tp.estride;
            const int64_t e = ch.elem_begin + min(int(threadIdx.x) + j * BLOCK, ch.elem_count - 1);
            const uint4 *__restrict__ g4 = static_cast<const uint4 *>(tp.elem4);
            const uint32_t *__restrict__ g1 = static_cast<const uint32_t *>(tp.elem4) + 4 * G * es;
            uint32_t w[D];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const uint4 v = g4[g * es + e];
                w[4 * g] = v.x;
                w[4 * g + 1] = v.y;
                w[4 * g + 2] = v.z;
                w[4 * g + 3] = v.w;
            }
#pragma unroll
            for (int r = 0; r < R; r++) w[4 * G + r] = g1[r * es + e];
#pragma unroll
            for (int q = 0; q < NP; q++) er.cst[j][q] = __uint_as_float(w[q]);
#pragma unroll
            for (int a = 0; a < NE; a += 2) er.wp[j][a] = int(w[NP + a / 2]);
        } else if constexpr (!PF) {
            const T *__restrict__ ep = static_cast<const T *>(tp.elem);
            const int64_t es = tp.estride;
            const int e = min(int(threadIdx.x) + j * BLOCK, ch.elem_count - 1);
            const T *src = ep + ch.elem_begin + e;
#pragma unroll
            for (int q = 0; q < NP; q++) er.cst[j][q] = src[q * es];
            const uint16_t *w = tp.wpos + ch.elem_begin + e;
#pragma unroll
            for (int a = 0; a < NE; a++) er.wp[j][a] = w[a * es];
        }
    }
    __device__ static void load_elems(const DevTopo &tp, const ChunkDesc &ch, ElemRegs &er) {
#pragma unroll
        for (int j = 0; j < EPT; j++) load_elem(tp, ch, er, j);
    }

    // Per-copy data of the chunk's node copies (MODE 1 adds what the update
    // needs, except the load values, which load_rv fetches once the flags are
    // in).  Range, flags and u^n as in load_elems (clamped, unconditional).
    template <int MODE>
    __device__ static void load_copies(const DevTopo &tp, const ChunkDesc &ch, const StepPtrs<T> &sp, CopyRegs &c) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            const int l = ch.copy_begin + min(i, ch.copy_count - 1);
            c.cr[m] = tp.crange[l];
            c.fl[m] = sp.flags[l];
            ld_u3<AOS>(sp.uc, l, c.ux[m]);
            if constexpr (ANPM) c.pn[m] = sp.pn ? sp.pn[l] : T(0);
            if (i < ch.copy_count) {
                if (i >= ch.n_interior) {
                    c.pb[m] = tp.pidx[l];
                } else if (MODE == 1) {
                    ld_u3<AOS>(sp.up, l, c.upv[m]);
                    if constexpr (PC) ld_ab(sp, l, c.A[m], c.Bp[m]);
                    else c.A[m] = sp.acoef[l];
                }
            }
        }
    }

    // loads (BC targets / forces) of interior copies, needed only at the update
    template <int MODE>
    __device__ static void load_rv(const ChunkDesc &ch, const StepPtrs<T> &sp, CopyRegs &c) {
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = threadIdx.x + m * BLOCK;
#pragma unroll
            for (int k = 0; k < 3; k++) c.rv[m][k] = T(0);
            if constexpr (PC) c.rr[m] = T(0);
            if (MODE == 1 && i < ch.n_interior && (c.fl[m] & FLAG_RU)) {
                const int l = ch.copy_begin + i;
                if constexpr (PC) {
                    ld_rq(sp, l, c.rv[m], c.rr[m]);
                } else {
#pragma unroll
                    for (int k = 0; k < 3; k++) c.rv[m][k] = sp.ru[k][l];
                }
            }
        }
    }

    // MODE 0: forces to the caller array; MODE 1: time-step update.  `after`
    // runs once the element forces are in LDS (PF: issues the next prefetch).
    template <int MODE, typename After = NoOp>
    __device__ static void element_phase(const DevTopo &tp, const ChunkDesc &ch, const StepPtrs<T> &sp,
                                         unsigned char *smem, PhaseOut &po, After after = After()) {
        ElemRegs er;
        CopyRegs cp;
        load_elems(tp, ch, er);
        load_copies<MODE>(tp, ch, sp, cp);
        load_rv<MODE>(ch, sp, cp);
        process<MODE, false>(tp, ch, sp, smem, po, er, cp, after);
    }

    struct alignas(16) Slot4 {  // 12 bytes used of 16
        float x, y, z;
    };
    __device__ static void slot_put(T *lx, int q, T a, T b, T c) {
        if constexpr (L4) {
            reinterpret_cast<Slot4 *>(lx)[q] = Slot4{a, b, c};
        } else {
            lx[q] = a;
            lx[SP + q] = b;
            lx[2 * SP + q] = c;
        }
    }
    __device__ static void slot_get(const T *lx, int q, T &a, T &b, T &c) {
        if constexpr (L4) {
            const Slot4 v = reinterpret_cast<const Slot4 *>(lx)[q];
            a = v.x;
            b = v.y;
            c = v.z;
        } else {
            a = lx[q];
            b = lx[SP + q];
            c = lx[2 * SP + q];
        }
    }

    // u^n (and the nodal pressure of the average-nodal-pressure step) of each
    // copy over its contiguous incidence range
    __device__ static void scatter_u(const ChunkDesc &ch, const StepPtrs<T> &sp, T *lx, const CopyRegs &cin) {
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = int(threadIdx.x) + m * BLOCK;
            if (i < ch.copy_count) {
                const int b = cin.cr[m] & 0xffffu, n = cin.cr[m] >> 16;
                for (int q = b; q < b + n; q++) slot_put(lx, q, cin.ux[m][0], cin.ux[m][1], cin.ux[m][2]);
                if constexpr (ANPM)
                    if (sp.pn)
                        for (int q = b; q < b + n; q++) lx[3 * SP + q] = cin.pn[m];
            }
        }
    }

    // element forces from the slots, written back over the element's own positions;
    // done(j) runs once element slot j's registers are consumed
    template <typename Done = NoOpJ>
    __device__ static void forces(const ChunkDesc &ch, const StepPtrs<T> &sp, T *lx, PhaseOut &po, ElemRegs &er,
                                  Done done = Done()) {
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            const int e = int(threadIdx.x) + j * BLOCK;
            if (e < ch.elem_count) {
                T u[NE][3], F[NE][3];
#pragma unroll
                for (int a = 0; a < NE; a++) slot_get(lx, slot(er, j, a), u[a][0], u[a][1], u[a][2]);
                T J;
                if constexpr (ANPM) {
                    // average nodal pressure: with sp.pn the kappa plane holds 0V and the
                    // element pressure is the mean of its nodes' pressures; without it
                    // the plane already holds that mean times 0V
                    T cst[NP];
#pragma unroll
                    for (int q = 0; q < NP; q++) cst[q] = er.cst[j][q];
                    if (sp.pn) {
                        T pb = 0;
#pragma unroll
                        for (int a = 0; a < NE; a++) pb += lx[3 * SP + slot(er, j, a)];
                        cst[Planes<NE, MODEL>::KAV] *= pb * T(1.0 / NE);
                    }
                    J = element_force<T, NE, MODEL>(cst, u, F);
                } else {
                    J = element_force<T, NE, MODEL>(er.cst[j], u, F);
                }
                // an inverted (or non-finite) element stops the run; its force is
                // left out so that the error is reported at the element itself
                const bool ok = J > T(0);
#pragma unroll
                for (int a = 0; a < NE; a++)
                    slot_put(lx, slot(er, j, a), ok ? F[a][0] : T(0), ok ? F[a][1] : T(0), ok ? F[a][2] : T(0));
                if (!isfinite(J)) {
                    po.bad = DJ_ERR_NONFINITE;
                    po.bad_elem = ch.elem_begin + e;
                } else if (!(J > T(0)) && po.bad == 0) {
                    po.bad = DJ_ERR_INVERTED;
                    po.bad_elem = ch.elem_begin + e;
                }
            }
            done(j);
        }
    }

    // node sum of the thread's copy m over its range, in fixed order
    __device__ static void copy_sum(const CopyRegs &c, int m, const T *lx, T (&f)[3]) {
        const int b = c.cr[m] & 0xffffu, n = c.cr[m] >> 16;
        f[0] = f[1] = f[2] = T(0);
        // four slots' reads in flight per round, added in slot order (the same sums)
        int q = b;
        for (; q + 4 <= b + n; q += 4) {
            T x[4], y[4], z[4];
#pragma unroll
            for (int t = 0; t < 4; t++) slot_get(lx, q + t, x[t], y[t], z[t]);
#pragma unroll
            for (int t = 0; t < 4; t++) {
                f[0] += x[t];
                f[1] += y[t];
                f[2] += z[t];
            }
        }
        for (; q < b + n; q++) {
            T x, y, z;
            slot_get(lx, q, x, y, z);
            f[0] += x;
            f[1] += y;
            f[2] += z;
        }
    }

    // One chunk from registers loaded beforehand (RV: fetch the load values
    // here, after the scatter).  `after` runs once the element forces are in
    // LDS and the chunk's registers are consumed or copied, so it may reload
    // `er` and `cin` with the next chunk's data.
    template <int MODE, bool RV, typename After>
    __device__ static void process(const DevTopo &tp, const ChunkDesc &ch, const StepPtrs<T> &sp, unsigned char *smem,
                                   PhaseOut &po, ElemRegs &er, CopyRegs &cin, After after) {
        const int tid = threadIdx.x;
        INSTR_T(i0);
        T *lx = reinterpret_cast<T *>(smem);
        scatter_u(ch, sp, lx, cin);
        if constexpr (RV) load_rv<MODE>(ch, sp, cin);
        if constexpr (PF) __builtin_amdgcn_s_waitcnt(0);  // this thread's staged loads have landed
        __syncthreads();
        INSTR_T(i1);
        if constexpr (PF) {
            const T *stage = reinterpret_cast<const T *>(smem + SLOTS);
            const uint16_t *wstage = reinterpret_cast<const uint16_t *>(smem + SLOTS) + 2 * NP * PDW + (ch.elem_begin & 1);
#pragma unroll
            for (int j = 0; j < EPT; j++) {
                const int e = tid + j * BLOCK;
                if (e < ch.elem_count) {
#pragma unroll
                    for (int q = 0; q < NP; q++) er.cst[j][q] = stage[q * CMAX + e];
#pragma unroll
                    for (int a = 0; a < NE; a++) er.wp[j][a] = wstage[a * 2 * WDW + e];
                }
            }
        }
        forces(ch, sp, lx, po, er);
        __syncthreads();
        INSTR_T(i2);
        const CopyRegs c = cin;
        after();
        // ---- node sums over each copy's range, in fixed order
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            if (i < ch.copy_count) {
                T f[3];
                copy_sum(c, m, lx, f);
                const int l = ch.copy_begin + i;
                if (i >= ch.n_interior) {
                    const int q = c.pb[m] + int((c.fl[m] >> FLAG_RANK_SHIFT) & 255u);
                    put_partial3<AOS>(sp.pp, q, f);
                    if (!(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2])) && po.bad == 0) {
                        po.bad = DJ_ERR_NONFINITE;
                        po.bad_elem = -2 - l;
                    }
                } else if constexpr (MODE == 0) {
                    const int nd = tp.cnode[l];
                    sp.fout[3 * nd] = f[0];
                    sp.fout[3 * nd + 1] = f[1];
                    sp.fout[3 * nd + 2] = f[2];
                } else if constexpr (PC) {
                    node_update<T, AOS>(l, c.fl[m], f, c.ux[m], c.upv[m], c.A[m], c.Bp[m], ramp_rate(c.rr[m], sp.n1), c.rv[m],
                                   sp, po);
                } else {
                    node_update<T, AOS>(l, c.fl[m], f, c.ux[m], c.upv[m], c.A[m], sp.bprime, sp.sval, c.rv[m], sp, po);
                }
            }
        }
        __syncthreads();  // LDS is reused by the next chunk
#ifdef DJ_INSTR
        INSTR_T(i3);
        instr_add(3, i1 - i0);
        instr_add(4, i2 - i1);
        instr_add(5, i3 - i2);
        instr_add(6, 1);
#endif
    }

    // The node results of one chunk, kept in registers until the next chunk
    // has waited for its loads: copy index (< 0: none), partial entry (>= 0 for
    // a shared copy's force sum, else the copy's new displacement), values.
    struct Held {
        int l[MC], q[MC];
        T v[MC][3];
    };
    __device__ static void held_clear(Held &h) {
#pragma unroll
        for (int m = 0; m < MC; m++) h.l[m] = -1;
    }
    __device__ static void held_store(const Held &h, const StepPtrs<T> &sp) {
#pragma unroll
        for (int m = 0; m < MC; m++) {
            if (h.l[m] < 0) continue;
            if (h.q[m] >= 0) {
                put_partial3<AOS>(sp.pp, h.q[m], h.v[m]);
            } else {
                st_u3<AOS>(sp.un, h.l[m], h.v[m]);
            }
        }
    }

    // Time-step chunk (register path, per-copy coefficients) with one wait for
    // memory per phase.  gfx950 counts vector loads and stores on one counter,
    // so waiting for a load while stores are in flight waits for every access
    // in flight.  Here a chunk waits for everything once at its start (its
    // element and copy data, loaded during the previous chunk, and that chunk's
    // stores are then complete), requests its load values, scatters, computes
    // the element forces while requesting the next chunk's element data
    // (`reload(j)` after slot j), waits for those loads, issues the next
    // chunk's copy loads (`after`) and then the previous chunk's stores, and
    // keeps its own node results in `held` for the next chunk to store.
    template <typename Reload, typename After>
    __device__ static void process_held(const ChunkDesc &ch, const StepPtrs<T> &sp, unsigned char *smem, PhaseOut &po,
                                        ElemRegs &er, CopyRegs &cin, Held &held, Reload reload, After after) {
        static_assert(PC && !PF, "batch register path");
        const int tid = threadIdx.x;
        INSTR_T(i0);
        T *lx = reinterpret_cast<T *>(smem);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_sched_barrier(0);
        load_rv<1>(ch, sp, cin);
        scatter_u(ch, sp, lx, cin);
        __syncthreads();
        INSTR_T(i1);
        forces(ch, sp, lx, po, er, reload);  // the next chunk's element data is requested slot by slot
        __syncthreads();
        INSTR_T(i2);
        __builtin_amdgcn_s_waitcnt(0);  // the load values and the next element data
        __builtin_amdgcn_sched_barrier(0);
        INSTR_T(ia);
        const CopyRegs c = cin;
        after();
        held_store(held, sp);
        __builtin_amdgcn_sched_barrier(0);
        INSTR_T(ib);
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            held.l[m] = -1;
            if (i < ch.copy_count) {
                T f[3];
                copy_sum(c, m, lx, f);
                const int l = ch.copy_begin + i;
                held.l[m] = l;
                if (i >= ch.n_interior) {
                    held.q[m] = c.pb[m] + int((c.fl[m] >> FLAG_RANK_SHIFT) & 255u);
#pragma unroll
                    for (int k = 0; k < 3; k++) held.v[m][k] = f[k];
                    if (!(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2])) && po.bad == 0) {
                        po.bad = DJ_ERR_NONFINITE;
                        po.bad_elem = -2 - l;
                    }
                } else {
                    held.q[m] = -1;
                    node_value<T>(l, c.fl[m], f, c.ux[m], c.upv[m], c.A[m], c.Bp[m], ramp_rate(c.rr[m], sp.n1), c.rv[m],
                                  sp, po, held.v[m]);
                }
            }
        }
        INSTR_T(ic);
        __syncthreads();  // LDS is reused by the next chunk
#ifdef DJ_INSTR
        INSTR_T(i3);
        instr_add(3, i1 - i0);
        instr_add(4, i2 - i1);
        instr_add(5, i3 - i2);
        instr_add(6, 1);
        instr_add(9, ia - i2);
        instr_add(10, ib - ia);
        instr_add(11, ic - ib);
        instr_add(12, i3 - ic);
#endif
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
                        ld_u3<AOS>(sp.uc, l, r.uc[kb]);
                        ld_u3<AOS>(sp.up, l, r.up[kb]);
                        if constexpr (PC) {
                            ld_ab(sp, l, r.A[kb], r.bp[kb]);
#pragma unroll
                            for (int k = 0; k < 3; k++) r.rv[kb][k] = T(0);
                            r.rr[kb] = T(0);
                            if (sp.ru[0]) ld_rq(sp, l, r.rv[kb], r.rr[kb]);
                        } else {
                            r.A[kb] = sp.acoef[l];
#pragma unroll
                            for (int k = 0; k < 3; k++) r.rv[kb][k] = sp.ru[0] ? sp.ru[k][l] : T(0);
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
                    if (q < cnt) get_partial3<AOS>(sp.pp, r.pb[kb] + q, px[kb][q]);
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
            for (int q = UNR; q < cnt; q++) {
                T g[3];
                get_partial3<AOS>(sp.pp, r.pb[kb] + q, g);
#pragma unroll
                for (int k = 0; k < 3; k++) f[k] += g[k];
            }
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
                if constexpr (PC)
                    node_update<T, AOS>(l, r.fl[kb], f, r.uc[kb], r.up[kb], r.A[kb], r.bp[kb],
                                   ramp_rate((r.fl[kb] & FLAG_RU) ? r.rr[kb] : T(0), sp.n1), r.rv[kb], sp, po);
                else
                    node_update<T, AOS>(l, r.fl[kb], f, r.uc[kb], r.up[kb], r.A[kb], sp.bprime, sp.sval, r.rv[kb], sp,
                                   po);
            }
        }
    }

    // Average-nodal-pressure J pass over one chunk: every element adds
    // 0V / n_e (J_e - 1) (the kappa plane holds 0V) to its nodes' slots; each
    // copy sums its range into S.  Interior copies finish the nodal pressure
    // p_n = c_n S_n at once, with c_n = kappa_n / V_n per copy; shared copies
    // publish S into their node's group (one plane).  Errors are left to the
    // force pass, which evaluates the same elements at the same u.
    __device__ static void anp_j_phase(const DevTopo &tp, const ChunkDesc &ch, const StepPtrs<T> &sp, T *jpart,
                                       const T *cn, T *pn, unsigned char *smem) {
        const int tid = threadIdx.x;
        ElemRegs er;
        CopyRegs cp;
        load_elems(tp, ch, er);
        load_copies<0>(tp, ch, sp, cp);
        T *lx = reinterpret_cast<T *>(smem);
        T *ly = lx + SP;
        T *lz = lx + 2 * SP;
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            if (i < ch.copy_count) {
                const int b = cp.cr[m] & 0xffffu, n = cp.cr[m] >> 16;
                for (int q = b; q < b + n; q++) {
                    lx[q] = cp.ux[m][0];
                    ly[q] = cp.ux[m][1];
                    lz[q] = cp.ux[m][2];
                }
            }
        }
        __syncthreads();
        // each element reads and then overwrites only its own incidence slots
#pragma unroll
        for (int j = 0; j < EPT; j++) {
            const int e = tid + j * BLOCK;
            if (e < ch.elem_count) {
                T u[NE][3];
#pragma unroll
                for (int a = 0; a < NE; a++) {
                    u[a][0] = lx[slot(er, j, a)];
                    u[a][1] = ly[slot(er, j, a)];
                    u[a][2] = lz[slot(er, j, a)];
                }
                const T jw = er.cst[j][Planes<NE, MODEL>::KAV] * T(1.0 / NE) * element_jm1<T, NE, MODEL>(er.cst[j], u);
#pragma unroll
                for (int a = 0; a < NE; a++) lx[slot(er, j, a)] = jw;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MC; m++) {
            const int i = tid + m * BLOCK;
            if (i < ch.copy_count) {
                const int b = cp.cr[m] & 0xffffu, n = cp.cr[m] >> 16;
                T S = T(0);
                for (int q = b; q < b + n; q++) S += lx[q];
                const int l = ch.copy_begin + i;
                if (i >= ch.n_interior) st_dev(&jpart[cp.pb[m] + int((cp.fl[m] >> FLAG_RANK_SHIFT) & 255u)], S);
                else pn[l] = cn[l] * S;
            }
        }
        __syncthreads();  // LDS is reused by the next chunk
    }

    // After the J barrier: the nodal pressure of every shared copy of one
    // chunk from its node's group of J sums (summed in rank order).
    __device__ static void anp_j_shared(const DevTopo &tp, const ChunkDesc &ch, const StepPtrs<T> &sp,
                                        const T *jpart, const T *cn, T *pn) {
        for (int i = ch.n_interior + threadIdx.x; i < ch.copy_count; i += BLOCK) {
            const int l = ch.copy_begin + i;
            const uint32_t fl = sp.flags[l];
            const int cnt = (fl >> FLAG_NCOPY_SHIFT) & 255u, q0 = tp.pidx[l];
            T S = T(0);
            for (int q = 0; q < cnt; q++) S += ld_dev(&jpart[q0 + q]);
            pn[l] = cn[l] * S;
        }
    }

    // Shared-node phase of the batch path with one memory round per round of
    // copies.  The index round is only what the partial loads need (flags and
    // partial-group index per shared copy); every other value of a copy is
    // addressed by its copy index and is loaded together with the partials.
    // So the kernel issues, in one round, the state and partials of round r,
    // the indices of round r + 1 and the stores of round r - 1 (the results
    // wait in registers, SharedHeld).
    static constexpr int SUNR = 8;  // partials per copy loaded with the state (more are read on the spot)
    template <int KB>
    struct SharedIdx {
        uint32_t fl[KB];
        int pb[KB];
    };
    template <int KB>
    struct SharedPart {
        T px[KB][SUNR][3];
    };
    template <int KB>
    struct SharedHeld {
        int l[KB];  // < 0: nothing to store
        T v[KB][3];
    };
    // the same two loads by copy index (l < 0: no copy in this slot)
    template <int KB>
    __device__ static void shared_idx_l(const DevTopo &tp, const StepPtrs<T> &sp, const int (&ls)[KB], SharedIdx<KB> &x) {
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            x.fl[kb] = 0u;
            x.pb[kb] = 0;
            if (ls[kb] >= 0) {
                x.fl[kb] = sp.flags[ls[kb]];
                x.pb[kb] = tp.pidx[ls[kb]];
            }
        }
    }
    // state and partials by copy index; the load values only for loaded copies
    template <int KB>
    __device__ static void shared_fetch_l(const StepPtrs<T> &sp, const int (&ls)[KB], const SharedIdx<KB> &x,
                                          SharedRegs<T, KB> &r, SharedPart<KB> &pt) {
        static_assert(PC, "batch path");
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            r.ok[kb] = ls[kb] >= 0;
            if (ls[kb] >= 0) {
                const int l = ls[kb];
                r.li[kb] = l;
                r.fl[kb] = x.fl[kb];
                r.pb[kb] = x.pb[kb];
                ld_ab(sp, l, r.A[kb], r.bp[kb]);
                ld_u3<AOS>(sp.uc, l, r.uc[kb]);
                ld_u3<AOS>(sp.up, l, r.up[kb]);
#pragma unroll
                for (int k = 0; k < 3; k++) r.rv[kb][k] = T(0);
                r.rr[kb] = T(0);
                if ((x.fl[kb] & FLAG_RU) && sp.ru[0]) ld_rq(sp, l, r.rv[kb], r.rr[kb]);
                const int cnt = (x.fl[kb] >> FLAG_NCOPY_SHIFT) & 255u;
#pragma unroll
                for (int q = 0; q < SUNR; q++)
                    if (q < cnt) get_partial3<AOS>(sp.pp, x.pb[kb] + q, pt.px[kb][q]);
            }
        }
    }
    template <int KB>
    __device__ static void shared_values(SharedRegs<T, KB> &r, const SharedPart<KB> &pt, const StepPtrs<T> &sp,
                                         PhaseOut &po, SharedHeld<KB> &h) {
        static_assert(PC, "batch path");
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            h.l[kb] = -1;
            if (!r.ok[kb]) continue;
            const int cnt = (r.fl[kb] >> FLAG_NCOPY_SHIFT) & 255u;
            T f[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < SUNR; q++)
                if (q < cnt)
#pragma unroll
                    for (int k = 0; k < 3; k++) f[k] += pt.px[kb][q][k];
            for (int q = SUNR; q < cnt; q++) {  // nodes in more than SUNR chunks
                T g[3];
                get_partial3<AOS>(sp.pp, r.pb[kb] + q, g);
#pragma unroll
                for (int k = 0; k < 3; k++) f[k] += g[k];
            }
            if (!(r.fl[kb] & FLAG_RU))
#pragma unroll
                for (int k = 0; k < 3; k++) r.rv[kb][k] = T(0);
            node_value<T>(r.li[kb], r.fl[kb], f, r.uc[kb], r.up[kb], r.A[kb], r.bp[kb],
                          ramp_rate((r.fl[kb] & FLAG_RU) ? r.rr[kb] : T(0), sp.n1), r.rv[kb], sp, po, h.v[kb]);
            h.l[kb] = r.li[kb];
        }
    }

    // all passes of one batch of chunks (round A, then the partial groups and the update)
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

// A node-level error raised in the shared-node phase of step s (a non-finite
// u^{n+1} at a copy of a node shared by several chunks) is found after that
// step's grid barrier, when the other workgroups have moved on.  It goes to
// the error word of parity s + 1: every workgroup reads that word after the
// next barrier and stops there with step s counted as done (its state holds
// the non-finite value); after a launch's last step the host reads the word.
// No workgroup reads parity s + 1 between the two barriers, so the word is free.
__device__ __forceinline__ void publish_late_error(int32_t *status, int s, int code, int32_t where, int32_t step_word,
                                                   int32_t case_word = -1) {
    if (atomicCAS(&status[5 + ((s + 1) & 1)], 0, code) == 0) {
        status[2] = where;
        status[3] = step_word;
        if (case_word >= 0) status[7] = case_word;
    }
}

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
// copies <- caller arrays (both state vectors at once when src1 != null);
// AOS: the batches' copy-major state layout
template <typename T, bool AOS = false>
__global__ void k_scatter_in(const int32_t *__restrict__ cnode, int n_copies, const T *__restrict__ src0,
                             const T *__restrict__ src1, T *__restrict__ d0, T *__restrict__ d1) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_copies) return;
    const int n = cnode[l];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int64_t o = AOS ? 3 * int64_t(l) + k : int64_t(k) * n_copies + l;
        d0[o] = src0[3 * n + k];
        if (src1) d1[o] = src1[3 * n + k];
    }
}

// Kernel variants per (precision, element type): {threads, elements per thread, copies per thread}
// Variants 4 and 5 trade register spills for a third wave per SIMD.
constexpr Variant VAR_T4F[N_VARIANTS] = {{256, 4, 2, 1}, {256, 2, 2, 1}, {512, 2, 2, 1},
                                         {128, 4, 2, 1}, {256, 4, 2, 3}, {256, 2, 2, 3}};
constexpr Variant VAR_H8F[N_VARIANTS] = {{256, 2, 4, 1}, {256, 1, 4, 1}, {512, 1, 3, 1},
                                         {128, 2, 4, 1}, {256, 1, 4, 3}, {512, 1, 3, 3}};
constexpr Variant VAR_T4D[N_VARIANTS] = {{256, 2, 2, 1}, {256, 1, 2, 1}, {512, 1, 2, 1},
                                         {128, 2, 2, 1}, {256, 2, 2, 1}, {256, 2, 2, 1}};
constexpr Variant VAR_H8D[N_VARIANTS] = {{256, 1, 4, 1}, {128, 1, 4, 1}, {512, 1, 3, 1},
                                         {128, 2, 4, 1}, {256, 1, 4, 1}, {256, 1, 4, 1}};

template <typename T, int NE>
constexpr const Variant *var_table() {
    return sizeof(T) == 4 ? (NE == 4 ? VAR_T4F : VAR_H8F) : (NE == 4 ? VAR_T4D : VAR_H8D);
}

}  // namespace dj
