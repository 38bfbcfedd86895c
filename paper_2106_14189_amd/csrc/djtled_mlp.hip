// Surrogate MLP for the learned warm start: p (n_in) -> relu(W1) -> relu(W2)
// -> W3 -> u (n_out), trained with mean-squared error and Adam.  All dense
// products run on a BF16 MFMA GEMM for gfx950 (v_mfma_f32_32x32x16_bf16, FP32
// accumulation) with fused epilogues (bias + ReLU, loss + output gradient,
// ReLU masks, split-K partials); small reductions and Adam are elementwise
// kernels.  GEMM operands are BF16; master weights, gradients and Adam moments
// are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <type_traits>

#include "../../include/djtled_mlp.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ---------------------------------------------------------------------------
// GEMM  C[M x N] = sum_k A(m, k) B(k, n), BF16 in, FP32 accumulate.
//   A(m, k) = A[m * lda + k]  (AK: K contiguous)  or  A[k * lda + m]  (M contiguous)
//   B(k, n) = B[n * ldb + k]  (BK: K contiguous)  or  B[k * ldb + n]  (N contiguous)
// Tile 128 x 128 x 32, 256 threads = 4 waves of 64 x 64 (2 x 2 MFMA 32x32x16).
// LDS holds both tiles K-contiguous ([row][k], padded) so every MFMA operand
// is one 16-byte LDS read.  gridDim.z splits K.
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BKT = 32, LDK = BKT + 8;  // LDS row: 40 bf16 = 80 bytes

enum Epi : int {
    EPI_F32 = 0,        // C (FP32) = acc
    EPI_BIAS_RELU = 1,  // Cb (BF16) = relu(acc + bias[n])
    EPI_BIAS_F32 = 2,   // C (FP32) = acc + bias[n]
    EPI_LOSS = 3,       // d = acc + bias[n] - U[m, n] (n < n_valid else 0): Cb = bf16(d * gscale), loss += d^2
    EPI_MASK = 4,       // Cb (BF16) = acc if aux[m, n] > 0 else 0   (ReLU backward)
    EPI_SPLITK = 5      // C[z][m][n] (FP32) = acc of split z
};

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;
    int64_t lda;
    const uint16_t *B;
    int64_t ldb;
    float *C;
    uint16_t *Cb;
    int64_t ldc;
    const float *bias;
    const float *U;        // EPI_LOSS targets (ldc)
    const uint16_t *aux;   // EPI_MASK activations (ldc)
    int n_valid;           // EPI_LOSS: columns that carry a loss
    float gscale;          // EPI_LOSS: output-gradient scale
    double *loss_part;     // EPI_LOSS: one partial per workgroup
    int k_per_split;       // multiple of BKT
};

// One 128 x 32 tile per operand: 512 vectors of 8 elements, two per thread.
// fetch: global -> registers (zero outside the matrix or beyond kend);
// stash: registers -> the K-contiguous LDS tile.
struct TileRegs {
    uint4 v[2];
};

template <bool KC>
__device__ __forceinline__ void fetch_tile(const uint16_t *__restrict__ G, int64_t ld, int r0, int k0, int R, int kend,
                                           TileRegs &t) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int v = threadIdx.x + h * 256;
        uint16_t e[8];
        if (KC) {
            const int gr = r0 + (v >> 2), gk = k0 + (v & 3) * 8;
            if (gr < R && gk + 8 <= kend) {
                t.v[h] = *reinterpret_cast<const uint4 *>(G + int64_t(gr) * ld + gk);
                continue;
            }
#pragma unroll
            for (int i = 0; i < 8; i++) e[i] = (gr < R && gk + i < kend) ? G[int64_t(gr) * ld + gk + i] : 0;
        } else {
            const int gk = k0 + (v >> 4), gr = r0 + (v & 15) * 8;
            if (gk < kend && gr + 8 <= R) {
                t.v[h] = *reinterpret_cast<const uint4 *>(G + int64_t(gk) * ld + gr);
                continue;
            }
#pragma unroll
            for (int i = 0; i < 8; i++) e[i] = (gk < kend && gr + i < R) ? G[int64_t(gk) * ld + gr + i] : 0;
        }
        t.v[h] = *reinterpret_cast<const uint4 *>(e);
    }
}

template <bool KC>
__device__ __forceinline__ void stash_tile(const TileRegs &t, uint16_t (*S)[LDK]) {
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int v = threadIdx.x + h * 256;
        if (KC) {
            *reinterpret_cast<uint4 *>(&S[v >> 2][(v & 3) * 8]) = t.v[h];
        } else {
            const int k = v >> 4, rq = (v & 15) * 8;
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&t.v[h]);
#pragma unroll
            for (int i = 0; i < 8; i++) S[rq + i][k] = e[i];
        }
    }
}

template <bool AK, bool BK, int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    // two LDS stages: the tiles of step k + 1 are fetched into registers while
    // step k multiplies, then stored into the other stage; one barrier per step
    __shared__ __align__(16) uint16_t As[2][BM][LDK];
    __shared__ __align__(16) uint16_t Bs[2][BN][LDK];
    __shared__ double s_loss[4];
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kbeg = blockIdx.z * g.k_per_split;
    const int kend = min(g.K, kbeg + g.k_per_split);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][j][r] = 0.0f;
    TileRegs ra, rb;
    if (kbeg < kend) {
        fetch_tile<AK>(g.A, g.lda, m0, kbeg, g.M, kend, ra);
        fetch_tile<BK>(g.B, g.ldb, n0, kbeg, g.N, kend, rb);
    }
    int st = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BKT, st ^= 1) {
        stash_tile<AK>(ra, As[st]);
        stash_tile<BK>(rb, Bs[st]);
        __syncthreads();
        if (k0 + BKT < kend) {
            fetch_tile<AK>(g.A, g.lda, m0, k0 + BKT, g.M, kend, ra);
            fetch_tile<BK>(g.B, g.ldb, n0, k0 + BKT, g.N, kend, rb);
        }
#pragma unroll
        for (int kk = 0; kk < BKT; kk += 16) {
            const int kq = kk + 8 * (lane >> 5);
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; i++) a[i] = *reinterpret_cast<const bf16x8 *>(&As[st][wm + 32 * i + (lane & 31)][kq]);
#pragma unroll
            for (int j = 0; j < 2; j++) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[st][wn + 32 * j + (lane & 31)][kq]);
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // epilogue: acc[i][j][r] -> row wm + 32 i + 8 (r / 4) + 4 (lane / 32) + r % 4, col wn + 32 j + lane % 32
    double lsum = 0.0;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int m = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int n = n0 + wn + 32 * j + (lane & 31);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                const int64_t o = int64_t(m) * g.ldc + n;
                if constexpr (EPI == EPI_F32) {
                    g.C[o] = v;
                } else if constexpr (EPI == EPI_BIAS_RELU) {
                    g.Cb[o] = f2bf(fmaxf(v + g.bias[n], 0.0f));
                } else if constexpr (EPI == EPI_BIAS_F32) {
                    g.C[o] = v + g.bias[n];
                } else if constexpr (EPI == EPI_LOSS) {
                    float d = 0.0f;
                    if (n < g.n_valid) d = v + g.bias[n] - g.U[o];
                    g.Cb[o] = f2bf(d * g.gscale);
                    lsum += double(d) * double(d);
                } else if constexpr (EPI == EPI_MASK) {
                    g.Cb[o] = bf2f(g.aux[o]) > 0.0f ? f2bf(v) : uint16_t(0);
                } else {
                    g.C[int64_t(blockIdx.z) * g.M * g.ldc + o] = v;
                }
            }
    if constexpr (EPI == EPI_LOSS) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (lane == 0) s_loss[wave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0)
            g.loss_part[blockIdx.y * gridDim.x + blockIdx.x] = (s_loss[0] + s_loss[1]) + (s_loss[2] + s_loss[3]);
    }
}

// ---------------------------------------------------------------------------
// The products with W3 (n_out x H, ~0.65 GB at full size) at batch B <= 256,
// H <= 512, H % 16 == 0.  Persistent workgroups of 8 waves keep the whole
// batch's H2 in registers as MFMA operands and stream the wide matrix once,
// in panels of 32 rows (W3) or 32 columns (dY) staged through LDS:
//   k_w3_fwd: wave w holds rows 32 w .. 32 w + 31 of H2 (all of K) as A
//     operands; per W3 panel it forms its 32 x 32 block of H2 W3^T and runs
//     the epilogue on it (bias; or loss, output gradient and its column sums
//     db3);
//   k_w3_dw: wave w holds columns 64 w .. 64 w + 63 of H2 (all B rows as K)
//     as B operands; per 32-column panel of dY, staged transposed, it forms
//     32 rows x 64 columns of dW3 = dY^T H2;
//   k_w3_dh: partial sums of dH2 = dY W3 over runs of W3 rows (below).
// dY is stored tiled by panel, [ceil(O / 32)][B][32]: a panel's 32 columns of
// every row are one contiguous 16 KB block (B = 256), so each wave writes
// whole 128-byte lines and the readers stream tiles in order.
// Every byte of W3, U, dY and dW3 crosses HBM once; H2 is read once per
// workgroup.  A panel is fetched into registers while the previous one is
// multiplied, then stored to LDS between two barriers.  Operands past B or H
// are zero, so every MFMA loop runs its full length.
// ---------------------------------------------------------------------------
constexpr int PNL = 32, KSMAX = 32, HMAX = 512, LDP = HMAX + 8, BMAX = 256, LDT = BMAX + 8;

struct W3Args {
    int B, H, N, O;             // batch, hidden width, columns written (<= O), rows of W3 = columns of U and dY
    const uint16_t *H2;         // [B x H]
    const uint16_t *W3;         // [O x H]
    const float *bias;          // [O]
    float *Y;                   // EPI_BIAS_F32: [B x O]
    const float *U;             // EPI_LOSS: targets [B x O]
    uint16_t *dY;               // EPI_LOSS: output gradient, tiled [ceil(O / 32)][B][32]
    float *db3;                 // EPI_LOSS: column sums of dY [O]
    int n_valid;                // EPI_LOSS: columns that carry a loss
    float gscale;               // EPI_LOSS: output-gradient scale
    double *loss_part;          // EPI_LOSS: one partial per workgroup
};

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// One wait per panel.  gfx950 counts vector loads and stores on one counter,
// and a load result needed while stores are in flight can only be waited for
// with a full wait.  So each panel starts with one full wait, and everything it
// consumes was issued one panel earlier: its tile of the wide operand, its
// targets and bias; the stores of the panel before it are issued from
// registers only after this panel's tile is in LDS.  Loads use clamped
// addresses and a select instead of a branch, and the last panel's prefetch
// reloads itself, so every panel issues the same accesses.
__device__ __forceinline__ void wait_all() { __builtin_amdgcn_s_waitcnt(0); }

template <int EPI>
__global__ void __launch_bounds__(512) k_w3_fwd(W3Args g) {
    constexpr int PPT = PNL * (HMAX / 8) / 512;  // 16-byte pieces of a panel per thread
    __shared__ __align__(16) uint16_t Ws[PNL + 1][LDP];
    __shared__ float s_db[8][32];
    __shared__ double s_loss[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int npc = g.H / 8, nact = min(8, (g.B + 31) / 32);
    const bool active = wave < nact;
    // columns past H stay zero: the panel stores below never reach them
    for (int i = threadIdx.x; i < (PNL + 1) * LDP / 8; i += 512)
        reinterpret_cast<uint4 *>(&Ws[0][0])[i] = make_uint4(0, 0, 0, 0);
    uint4 a[KSMAX];
    {
        const int row = wave * 32 + (lane & 31);
#pragma unroll
        for (int ks = 0; ks < KSMAX; ks++) {
            const int k = 16 * ks + 8 * (lane >> 5);
            a[ks] = make_uint4(0, 0, 0, 0);
            if (k < g.H && row < g.B) a[ks] = *reinterpret_cast<const uint4 *>(g.H2 + int64_t(row) * g.H + k);
        }
    }
    int pr[PPT], pc[PPT];  // panel row and 8-column group of each piece this thread moves
#pragma unroll
    for (int h = 0; h < PPT; h++) {
        const int v = threadIdx.x + 512 * h;
        pr[h] = min(v / npc, PNL);  // row PNL of Ws takes the pieces past the panel (H < 512)
        pc[h] = v / npc < PNL ? (v - (v / npc) * npc) * 8 : 0;
    }
    // raw loads from clamped addresses; the pieces past the panel or past O are zeroed when stored
    // (a select right after a load would wait for it at once)
    auto fetch = [&](int p, uint4 (&pf)[PPT]) {
#pragma unroll
        for (int h = 0; h < PPT; h++) {
            const int r = min(pr[h], min(PNL, g.O - p * PNL) - 1);
            pf[h] = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(g.W3 + int64_t(p) * PNL * g.H) +
                                                     2u * uint32_t(r * g.H + pc[h]));
        }
    };
    // element (m, n) of U and Y ([B x O]) sits at the uniform offset (8 (r / 4) + r % 4) O + 32 p
    // plus the lane's own, (32 wave + 4 (lane / 32)) O + lane % 32, for m = 32 wave + 4 (lane / 32)
    // + 8 (r / 4) + r % 4 and n = 32 p + lane % 32; the lane's part is kept as a 32-bit byte offset
    const uint32_t L4 = 4u * (uint32_t(wave * 32 + 4 * (lane >> 5)) * uint32_t(g.O) + uint32_t(lane & 31));
    // dY is tiled by panel ([O / 32][B][32]): the lane's byte offset within a tile
    const uint32_t LT = 2u * uint32_t((wave * 32 + 4 * (lane >> 5)) * PNL + (lane & 31));
    auto roff = [&](int r, uint32_t esz) { return esz * uint32_t(8 * (r >> 2) + (r & 3)) * uint32_t(g.O); };
    // the compiler would otherwise keep one offset per row live across the panel loop
    auto opaque = [](uint32_t x) {
        asm volatile("" : "+v"(x));
        return x;
    };
    // raw loads; rows past B and columns past n_valid read element (0, 32 p) instead, and the
    // epilogue never uses them
    auto fetch_u = [&](int p, float (&u)[16]) {
        const int n = p * PNL + (lane & 31);
        const uint32_t l4 = opaque(L4);
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int m = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const uint32_t o = m < g.B && n < g.n_valid ? l4 + roff(r, 4u) : 0u;
            u[r] = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(g.U + int64_t(p) * PNL) + o);
        }
    };
    auto fetch_bias = [&](int p) { return g.bias[min(p * PNL + (lane & 31), g.O - 1)]; };
    // db3 of panel pp from the per-wave column sums
    auto flush_db3 = [&](int pp) {
        if (EPI == EPI_LOSS && threadIdx.x < 32 && pp * PNL + int(threadIdx.x) < g.O) {
            float t = 0.0f;
            for (int w = 0; w < nact; w++) t += s_db[w][threadIdx.x];
            g.db3[pp * PNL + threadIdx.x] = t;
        }
    };
    // the outputs of panel ph, held in registers until the next panel's tile is in LDS
    float yh[16];
    uint32_t qh[8];
    int ph = -1;
    auto store_held = [&]() {
        if (ph < 0 || !active) return;
        const int n = ph * PNL + (lane & 31);
        const uint32_t l4 = opaque(L4), lt = opaque(LT);
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int m = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (m >= g.B || n >= g.N) continue;
            if constexpr (EPI == EPI_BIAS_F32) {
                *reinterpret_cast<float *>(reinterpret_cast<char *>(g.Y + int64_t(ph) * PNL) + (l4 + roff(r, 4u))) = yh[r];
            } else {
                *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(g.dY + int64_t(ph) * PNL * g.B) +
                                              (lt + 64u * uint32_t(8 * (r >> 2) + (r & 3)))) =
                    uint16_t(r & 1 ? qh[r >> 1] >> 16 : qh[r >> 1] & 0xffffu);
            }
        }
    };
    // each workgroup takes a contiguous run of panels
    const int npan = (g.O + PNL - 1) / PNL, per = (npan + gridDim.x - 1) / gridDim.x;
    const int p_beg = min(npan, int(blockIdx.x) * per), p_end = min(npan, p_beg + per);
    uint4 pf[PPT];
    float u[16], un[16], bn = 0.0f, bnn = 0.0f;
    double lsum = 0.0;
    if (p_beg < p_end) {
        fetch(p_beg, pf);
        if (EPI == EPI_LOSS && active) fetch_u(p_beg, un);
        bnn = fetch_bias(p_beg);
    }
    for (int p = p_beg; p < p_end; p++) {
        wait_all();
        __syncthreads();  // the previous panel's tile and column sums have been read and written
        if (p > p_beg) flush_db3(p - 1);
#pragma unroll
        for (int h = 0; h < PPT; h++)
            *reinterpret_cast<uint4 *>(&Ws[pr[h]][pc[h]]) =
                pr[h] < min(PNL, g.O - p * PNL) ? pf[h] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 16; r++) u[r] = un[r];
        bn = bnn;
        __syncthreads();
        store_held();
        const int pn = min(p + 1, p_end - 1);
        fetch(pn, pf);
        if (EPI == EPI_LOSS && active) fetch_u(pn, un);
        bnn = fetch_bias(pn);
        ph = p;
        if (!active) continue;
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; r++) acc[r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < KSMAX; ks++) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Ws[lane & 31][16 * ks + 8 * (lane >> 5)]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a[ks]), b, acc, 0, 0, 0);
        }
        // acc[r]: row 32 wave + 8 (r / 4) + 4 (lane / 32) + r % 4, column 32 p + lane % 32
        if constexpr (EPI == EPI_BIAS_F32) {
#pragma unroll
            for (int r = 0; r < 16; r++) yh[r] = acc[r] + bn;
        } else {
            const int n = p * PNL + (lane & 31);
            float csum = 0.0f, ls = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                float d[2];
#pragma unroll
                for (int t = 0; t < 2; t++) {
                    const int m = wave * 32 + 8 * ((r + t) >> 2) + 4 * (lane >> 5) + ((r + t) & 3);
                    d[t] = (m < g.B && n < g.n_valid) ? acc[r + t] + bn - u[r + t] : 0.0f;
                    ls += d[t] * d[t];
                }
                // two BF16 roundings (to nearest even) in one conversion
                const f32x2 sd = {d[0] * g.gscale, d[1] * g.gscale};
                const uint32_t q2 = __builtin_bit_cast(uint32_t, __builtin_convertvector(sd, bf16x2));
                csum += __uint_as_float(q2 << 16) + __uint_as_float(q2 & 0xffff0000u);
                qh[r >> 1] = q2;
            }
            lsum += double(ls);  // 16 squares per lane and panel in FP32, the running sum in FP64
            csum += __shfl_xor(csum, 32, 64);
            if (lane < 32) s_db[wave][lane] = csum;
        }
    }
    wait_all();
    __syncthreads();
    if (p_end > p_beg) flush_db3(p_end - 1);
    store_held();
    if constexpr (EPI == EPI_LOSS) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (lane == 0) s_loss[wave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < 8; w++) t += s_loss[w];
            g.loss_part[blockIdx.x] = t;
        }
    }
}

__global__ void __launch_bounds__(512) k_w3_dw(int B, int H, int O, const uint16_t *__restrict__ H2,
                                               const uint16_t *__restrict__ dY, float *__restrict__ dW3) {
    constexpr int KS = BMAX / 16;
    __shared__ __align__(16) uint16_t Ts[PNL][LDT];  // the dY panel transposed: [column][batch row]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // b[ks][j]: H2 rows 16 ks + 8 (lane / 32) + 0..7 at column 64 wave + 32 j + lane % 32
    uint4 b[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int h = 64 * wave + 32 * j + (lane & 31), m0 = 16 * ks + 8 * (lane >> 5);
            const int hc = min(h, H - 1);
            uint32_t e[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int ma = m0 + 2 * i, mb = ma + 1;
                const uint32_t lo = H2[int64_t(min(ma, B - 1)) * H + hc], hi = H2[int64_t(min(mb, B - 1)) * H + hc];
                e[i] = (ma < B && h < H ? lo : 0u) | (mb < B && h < H ? hi << 16 : 0u);
            }
            b[ks][j] = make_uint4(e[0], e[1], e[2], e[3]);
        }
        __builtin_amdgcn_sched_barrier(0);  // bounds the 16-bit loads in flight
    }
    // each thread moves rows 2 mp, 2 mp + 1 of one 8-column group of a dY tile
    const int cg = (threadIdx.x & 3) * 8, mp = threadIdx.x >> 2;
    // raw loads from clamped addresses, zeroed when stored (see k_w3_fwd)
    auto fetch = [&](int p, uint4 &r0, uint4 &r1) {
        const uint16_t *tile = dY + int64_t(p) * PNL * B + (p * PNL + cg < O ? cg : 0);
        r0 = *reinterpret_cast<const uint4 *>(tile + min(2 * mp, B - 1) * PNL);
        r1 = *reinterpret_cast<const uint4 *>(tile + min(2 * mp + 1, B - 1) * PNL);
    };
    // acc of panel ph is stored only after the next panel's tile is in LDS (one wait per panel, as in k_w3_fwd)
    f32x16 acc[2];
    int ph = -1;
    auto store_held = [&]() {
        if (ph < 0 || 64 * wave >= H) return;
        const int n0 = ph * PNL;
        char *base = reinterpret_cast<char *>(dW3 + int64_t(n0) * H);
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int h = 64 * wave + 32 * j + (lane & 31);
            const uint32_t lo = 4u * uint32_t(4 * (lane >> 5) * H + h);
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int n = n0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (n < O && h < H)
                    *reinterpret_cast<float *>(base + (lo + 4u * uint32_t((8 * (r >> 2) + (r & 3)) * H))) = acc[j][r];
            }
        }
    };
    // contiguous runs of panels: consecutive dY tiles
    const int npan = (O + PNL - 1) / PNL, per = (npan + gridDim.x - 1) / gridDim.x;
    const int p_beg = min(npan, int(blockIdx.x) * per), p_end = min(npan, p_beg + per);
    uint4 r0, r1;
    if (p_beg < p_end) fetch(p_beg, r0, r1);
    for (int p = p_beg; p < p_end; p++) {
        wait_all();
        __syncthreads();
        {
            const bool okc = p * PNL + cg < O;
            const uint4 z4 = make_uint4(0, 0, 0, 0);
            const uint4 s0 = okc && 2 * mp < B ? r0 : z4, s1 = okc && 2 * mp + 1 < B ? r1 : z4;
            const uint32_t x0[4] = {s0.x, s0.y, s0.z, s0.w}, x1[4] = {s1.x, s1.y, s1.z, s1.w};
#pragma unroll
            for (int i = 0; i < 4; i++) {
                *reinterpret_cast<uint32_t *>(&Ts[cg + 2 * i][2 * mp]) = (x0[i] & 0xffffu) | (x1[i] << 16);
                *reinterpret_cast<uint32_t *>(&Ts[cg + 2 * i + 1][2 * mp]) = (x0[i] >> 16) | (x1[i] & 0xffff0000u);
            }
        }
        __syncthreads();
        store_held();
        fetch(min(p + 1, p_end - 1), r0, r1);
        ph = p;
        if (64 * wave >= H) continue;
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[j][r] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&Ts[lane & 31][16 * ks + 8 * (lane >> 5)]);
#pragma unroll
            for (int j = 0; j < 2; j++)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf16x8(b[ks][j]), acc[j], 0, 0, 0);
        }
    }
    wait_all();
    store_held();
}

// dH2 partial sums over runs of W3 rows: part[z][m][h] = sum over the n of run z of dY[m][n] W3[n][h].
// Workgroup b takes run z and the 128-column slice sl of H; the slices of one run share b % 8 (one
// XCD), so the dY tiles they all read meet in its L2.  Wave w owns rows 32 w .. 32 w + 31 and the
// slice's four 32-column blocks.  dY operands come straight from the tiles (8 consecutive n of a row
// are 16 contiguous bytes); 128 rows of W3 at a time are staged transposed ([h][n]) in LDS.  Nothing
// is stored inside the loop, so the compiler's waits count loads precisely: the loads of the next two
// chunks stay in flight while this chunk multiplies.
constexpr int DHN = 128, DHS = 128, LDH = DHN + 8, DKS = DHN / 16;

__global__ void __launch_bounds__(512) k_w3_dh(int B, int H, int O, int nsplit, const uint16_t *__restrict__ dY,
                                               const uint16_t *__restrict__ W3, float *__restrict__ part) {
    __shared__ __align__(16) uint16_t Wt[DHS][LDH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nhs = (H + DHS - 1) / DHS, b = blockIdx.x;
    const int z = nsplit % 8 == 0 ? (b / (8 * nhs)) * 8 + b % 8 : b / nhs;
    const int sl = nsplit % 8 == 0 ? (b / 8) % nhs : b % nhs;
    const int h0 = sl * DHS;
    const int nch = (O + DHN - 1) / DHN, per = (nch + nsplit - 1) / nsplit;
    const int c_beg = min(nch, z * per), c_end = min(nch, c_beg + per);
    const bool active = 32 * wave < B;
    const int m = 32 * wave + (lane & 31);
    // W3 staging: rows 2 q, 2 q + 1 and 64 + 2 q, 65 + 2 q of the chunk, 8 columns from hq
    const int q = threadIdx.x >> 4, hq = (threadIdx.x & 15) * 8;
    // raw loads from clamped addresses, zeroed when used (a select right after a load would wait for it)
    auto fetch_w = [&](int c, uint4 (&w)[4]) {
        const int h = h0 + hq, hc = h < H ? h : 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int n = c * DHN + 64 * (i >> 1) + 2 * q + (i & 1);
            w[i] = *reinterpret_cast<const uint4 *>(W3 + int64_t(min(n, O - 1)) * H + hc);
        }
    };
    // dY operands of chunk c: k-step ks covers n = 128 c + 16 ks + 8 (lane / 32) + 0..7
    auto a_ok = [&](int c, int ks) {
        const int p = 4 * c + (ks >> 1), k = 16 * (ks & 1) + 8 * (lane >> 5);
        return m < B && p * PNL + k < O;
    };
    auto fetch_a = [&](int c, uint4 (&a)[DKS]) {
#pragma unroll
        for (int ks = 0; ks < DKS; ks++) {
            const int p = 4 * c + (ks >> 1), k = 16 * (ks & 1) + 8 * (lane >> 5);
            a[ks] = *reinterpret_cast<const uint4 *>(dY + (a_ok(c, ks) ? (int64_t(p) * B + m) * PNL + k : 0));
        }
    };
    f32x16 acc[4];
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[j][r] = 0.0f;
    // two register sets, two chunks ahead; an odd run ends with chunk nch, past the matrix, which adds zeros
    auto chunk = [&](int c, uint4 (&w)[4], uint4 (&a)[DKS]) __attribute__((always_inline)) {
        __syncthreads();  // the previous chunk's tile has been read
        {
            const int h = h0 + hq;
            const uint4 z4 = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int pr = 0; pr < 2; pr++) {
                const int n = c * DHN + 64 * pr + 2 * q;
                const uint4 s0 = h < H && n < O ? w[2 * pr] : z4;
                const uint4 s1 = h < H && n + 1 < O ? w[2 * pr + 1] : z4;
                const uint32_t x0[4] = {s0.x, s0.y, s0.z, s0.w}, x1[4] = {s1.x, s1.y, s1.z, s1.w};
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    *reinterpret_cast<uint32_t *>(&Wt[hq + 2 * i][64 * pr + 2 * q]) = (x0[i] & 0xffffu) | (x1[i] << 16);
                    *reinterpret_cast<uint32_t *>(&Wt[hq + 2 * i + 1][64 * pr + 2 * q]) =
                        (x0[i] >> 16) | (x1[i] & 0xffff0000u);
                }
            }
        }
        uint4 ac[DKS];
#pragma unroll
        for (int ks = 0; ks < DKS; ks++) ac[ks] = a_ok(c, ks) ? a[ks] : make_uint4(0, 0, 0, 0);
        __syncthreads();
        const int cn = min(c + 2, c_end - 1);
        fetch_w(cn, w);
        fetch_a(cn, a);
        if (!active) return;
#pragma unroll
        for (int ks = 0; ks < DKS; ks++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(&Wt[32 * j + (lane & 31)][16 * ks + 8 * (lane >> 5)]);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ac[ks]), bw, acc[j], 0, 0, 0);
            }
    };
    uint4 wA[4], aA[DKS], wB[4], aB[DKS];
    if (c_beg < c_end) {
        fetch_w(c_beg, wA);
        fetch_a(c_beg, aA);
        fetch_w(min(c_beg + 1, c_end - 1), wB);
        fetch_a(min(c_beg + 1, c_end - 1), aB);
    }
    for (int c = c_beg; c < c_end; c += 2) {
        chunk(c, wA, aA);
        chunk(c + 1 < c_end ? c + 1 : nch, wB, aB);
    }
    if (!active) return;
    // acc[j][r]: row 32 wave + 8 (r / 4) + 4 (lane / 32) + r % 4, column h0 + 32 j + lane % 32
    float *out = part + int64_t(z) * B * H;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int h = h0 + 32 * j + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int mr = 32 * wave + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (mr < B && h < H) out[int64_t(mr) * H + h] = acc[j][r];
        }
    }
}

// ---------------------------------------------------------------------------
// The hidden layers at batch MM <= 2: Y[m, n] = bf16(relu(sum_k x[m, k] W[k, n]
// + bias[n])) with W [K x N] (N contiguous) and x BF16 (or FP32 rounded to
// BF16 on load).  256 threads per 64 columns: 8 groups of 8 columns (one
// 16-byte piece of a W row) x 32 slices of K, summed through LDS in a fixed
// order.
// ---------------------------------------------------------------------------
template <int MM, bool XF32>
__global__ void __launch_bounds__(256) k_gemv_kn(const void *__restrict__ X, int64_t ldx, int K,
                                                 const uint16_t *__restrict__ W, int N, const float *__restrict__ bias,
                                                 uint16_t *__restrict__ Y, int64_t ldy) {
    __shared__ float red[32][MM][65];
    const int c8 = threadIdx.x & 7, sl = threadIdx.x >> 3;
    const int n = blockIdx.x * 64 + c8 * 8;
    float acc[MM][8];
#pragma unroll
    for (int m = 0; m < MM; m++)
#pragma unroll
        for (int i = 0; i < 8; i++) acc[m][i] = 0.0f;
    if (n < N) {
        for (int k = sl; k < K; k += 32) {
            const uint4 w = *reinterpret_cast<const uint4 *>(W + int64_t(k) * N + n);
            const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
            float x[MM];
#pragma unroll
            for (int m = 0; m < MM; m++)
                x[m] = XF32 ? bf2f(f2bf(static_cast<const float *>(X)[int64_t(m) * ldx + k]))
                            : bf2f(static_cast<const uint16_t *>(X)[int64_t(m) * ldx + k]);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const float lo = __uint_as_float(ww[i] << 16), hi = __uint_as_float(ww[i] & 0xffff0000u);
#pragma unroll
                for (int m = 0; m < MM; m++) {
                    acc[m][2 * i] += x[m] * lo;
                    acc[m][2 * i + 1] += x[m] * hi;
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < MM; m++)
#pragma unroll
        for (int i = 0; i < 8; i++) red[sl][m][c8 * 8 + i] = acc[m][i];
    __syncthreads();
    if (threadIdx.x < 64 * MM) {
        const int m = threadIdx.x >> 6, c = threadIdx.x & 63, nn = blockIdx.x * 64 + c;
        float s = 0.0f;
        for (int q = 0; q < 32; q++) s += red[q][m][c];
        if (nn < N) Y[int64_t(m) * ldy + nn] = f2bf(fmaxf(s + bias[nn], 0.0f));
    }
}

// ---------------------------------------------------------------------------
// Y[m, n] = sum_k X[m, k] W[n, k] + bias[n] for MM <= 2 rows (inference of the
// output layer): a streaming product over W (n_out x K, K contiguous).  Each
// wave takes 64 rows of W; per row every lane loads 16-byte pieces (a 1 KB row
// is one wave-wide load when K = 512) and keeps a partial dot per row; a
// butterfly of shuffles then halves the rows held per lane five times over,
// leaving lane l with the fixed-order sum of row l.
// ---------------------------------------------------------------------------
template <int MM, int T>
__global__ void __launch_bounds__(256) k_gemv(const uint16_t *__restrict__ X, int64_t ldx, int K,
                                              const uint16_t *__restrict__ W, int64_t ldw, int N,
                                              const float *__restrict__ bias, float *__restrict__ Y, int64_t ldy) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 4 + wave) * 64;
    if (r0 >= N) return;
    const int nc = K / 8;  // 16-byte pieces per row
    float x[MM][T][8];
#pragma unroll
    for (int m = 0; m < MM; m++)
#pragma unroll
        for (int t = 0; t < T; t++) {
            const int c = lane + 64 * t;
#pragma unroll
            for (int i = 0; i < 8; i++) x[m][t][i] = c < nc ? bf2f(X[int64_t(m) * ldx + c * 8 + i]) : 0.0f;
        }
    float p[MM][64];
#pragma unroll
    for (int j = 0; j < 64; j++) {
        const int row = min(r0 + j, N - 1);  // rows past the end are computed and dropped
#pragma unroll
        for (int m = 0; m < MM; m++) p[m][j] = 0.0f;
#pragma unroll
        for (int t = 0; t < T; t++) {
            const int c = lane + 64 * t;
            if (c < nc) {
                const uint4 w = *reinterpret_cast<const uint4 *>(W + int64_t(row) * ldw + c * 8);
                const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const float lo = __uint_as_float(ww[i] << 16), hi = __uint_as_float(ww[i] & 0xffff0000u);
#pragma unroll
                    for (int m = 0; m < MM; m++) p[m][j] += lo * x[m][t][2 * i] + hi * x[m][t][2 * i + 1];
                }
            }
        }
    }
    // butterfly: after the step of offset o each lane keeps half of its rows
#pragma unroll
    for (int o = 32, h = 32; o > 0; o >>= 1, h >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int j = 0; j < 32; j++) {
            if (j < h) {
#pragma unroll
                for (int m = 0; m < MM; m++) {
                    const float send = up ? p[m][j] : p[m][j + h];
                    const float keep = up ? p[m][j + h] : p[m][j];
                    p[m][j] = keep + __shfl_xor(send, o, 64);
                }
            }
        }
    }
    const int n = r0 + lane;
    if (n < N)
#pragma unroll
        for (int m = 0; m < MM; m++) Y[int64_t(m) * ldy + n] = p[m][0] + bias[n];
}

// split-K reduction with the ReLU mask: out = bf16(sum_z part[z]) where act > 0
__global__ void k_splitk_mask(const float *__restrict__ part, int splits, int64_t mn, const uint16_t *__restrict__ act,
                              uint16_t *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= mn) return;
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += part[int64_t(z) * mn + i];
    out[i] = bf2f(act[i]) > 0.0f ? f2bf(s) : uint16_t(0);
}

// column sums of a BF16 matrix [M x N] (bias gradients), fixed order
__global__ void __launch_bounds__(256) k_colsum(const uint16_t *__restrict__ X, int M, int N, int64_t ld,
                                                float *__restrict__ out) {
    // 32 columns x 8 row slices per block; the slices' sums are added in slice order
    __shared__ float part[8][33];
    const int c = threadIdx.x & 31, sl = threadIdx.x >> 5, n = blockIdx.x * 32 + c;
    float s = 0.0f;
    if (n < N) {
        const int m0 = sl * ((M + 7) / 8), m1 = min(M, m0 + (M + 7) / 8);
#pragma unroll 8
        for (int m = m0; m < m1; m++) s += bf2f(X[int64_t(m) * ld + n]);
    }
    part[sl][c] = s;
    __syncthreads();
    if (sl == 0 && n < N) {
        float t = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; q++) t += part[q][c];
        out[n] = t;
    }
}

// FP32 [M x K] -> BF16 [M x ldo] (columns K..ldo zero)
__global__ void k_to_bf16(const float *__restrict__ x, int M, int K, uint16_t *__restrict__ y, int ldo) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(M) * ldo) return;
    const int m = int(i / ldo), k = int(i % ldo);
    y[i] = k < K ? f2bf(x[int64_t(m) * K + k]) : uint16_t(0);
}

__global__ void k_sum_parts(const double *__restrict__ p, int n, double scale, double *__restrict__ out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += p[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * scale;
}

// Adam on one tensor; refreshes the BF16 copy when given
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ gr, float *__restrict__ m, float *__restrict__ v,
                       uint16_t *__restrict__ wb, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
}

__global__ void k_refresh_bf16(const float *__restrict__ w, uint16_t *__restrict__ wb, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

thread_local std::string g_mlp_err;

int mfail(int code, const std::string &m) {
    g_mlp_err = m;
    return code;
}

#define MLP_HIP(call)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) return mfail(DJ_MLP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <bool AK, bool BK, int EPI>
hipError_t gemm(GemmArgs a, int splits, hipStream_t s) {
    dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, splits);
    hipLaunchKernelGGL((k_gemm<AK, BK, EPI>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// the streaming W3 kernels: batch and width they hold in registers; a lane's byte offset into a
// [B x O] FP32 matrix fits 32 bits
bool w3_stream(int B, int H, int64_t O) {
    return B <= BMAX && H <= HMAX && H % 16 == 0 && int64_t(BMAX) * O * 4 < (int64_t(1) << 32);
}
constexpr int MAX_PERSIST = 4096;  // loss partials the workspace holds

// persistent grid: the resident workgroups of the device, at most `work`
template <typename Kern>
int persistent_grid(Kern kern, int slot, int work) {
    static std::atomic<int> cache[3][64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int n = cache[slot][dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        int cus = 0, occ = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 512, 0) != hipSuccess || occ <= 0) occ = 1;
        n = std::min(cus * occ, MAX_PERSIST);
        cache[slot][dev].store(n, std::memory_order_relaxed);
    }
    return std::max(1, std::min(n, work));
}

GemmArgs ga(int M, int N, int K, const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb) {
    GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.k_per_split = (K + BKT - 1) / BKT * BKT;
    return g;
}

int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// workspace carve-up
struct WS {
    uint16_t *Pb, *H1, *H2, *dY, *dZ2, *dZ1;
    float *part;
    double *loss_part, *loss;
    int splits;
};

int carve(const djtled_mlp *m, int B, void *base, size_t bytes, WS &w, size_t *need) {
    const int64_t H = m->n_hidden, O = m->ld_out;
    const int splits = int(std::min<int64_t>(64, std::max<int64_t>(1, (m->n_out + 8191) / 8192)));
    const int64_t tiles = ((O + BN - 1) / BN) * ((B + BM - 1) / BM);
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off += rup(int64_t(n), 256);
        return o;
    };
    const size_t oPb = take(size_t(B) * 32 * 2), oH1 = take(size_t(B) * H * 2), oH2 = take(size_t(B) * H * 2);
    const size_t odY = take(size_t(B) * rup(O, 32) * 2), odZ2 = take(size_t(B) * H * 2), odZ1 = take(size_t(B) * H * 2);
    const size_t opart = take(size_t(splits) * B * H * 4);
    const size_t olp = take(size_t(std::max<int64_t>(tiles, MAX_PERSIST)) * 8), ol = take(8);
    if (need) *need = off;
    if (!base) return DJ_MLP_OK;
    if (bytes < off) return mfail(DJ_MLP_ERR_ARG, "workspace too small");
    char *b = static_cast<char *>(base);
    w.Pb = reinterpret_cast<uint16_t *>(b + oPb);
    w.H1 = reinterpret_cast<uint16_t *>(b + oH1);
    w.H2 = reinterpret_cast<uint16_t *>(b + oH2);
    w.dY = reinterpret_cast<uint16_t *>(b + odY);
    w.dZ2 = reinterpret_cast<uint16_t *>(b + odZ2);
    w.dZ1 = reinterpret_cast<uint16_t *>(b + odZ1);
    w.part = reinterpret_cast<float *>(b + opart);
    w.loss_part = reinterpret_cast<double *>(b + olp);
    w.loss = reinterpret_cast<double *>(b + ol);
    w.splits = splits;
    return DJ_MLP_OK;
}

int check(const djtled_mlp *m, int B) {
    if (!m) return mfail(DJ_MLP_ERR_ARG, "null MLP");
    if (m->n_in <= 0 || m->n_in > 32 || m->n_hidden <= 0 || m->n_hidden % 8 || m->n_out <= 0 || m->ld_out < m->n_out ||
        m->ld_out % 8)
        return mfail(DJ_MLP_ERR_ARG, "need 0 < n_in <= 32, n_hidden % 8 == 0, ld_out >= n_out, ld_out % 8 == 0");
    if (B <= 0) return mfail(DJ_MLP_ERR_ARG, "batch must be > 0");
    if (!m->W1_bf16 || !m->W2_bf16 || !m->W3_bf16 || !m->b1 || !m->b2 || !m->b3)
        return mfail(DJ_MLP_ERR_ARG, "null parameter pointer");
    return DJ_MLP_OK;
}

// forward through the hidden layers: Pb, H1, H2
hipError_t hidden_forward(const djtled_mlp *m, int B, const float *P, WS &w, hipStream_t s) {
    const int H = m->n_hidden;
    hipLaunchKernelGGL(k_to_bf16, dim3((B * 32 + 255) / 256), dim3(256), 0, s, P, B, m->n_in, w.Pb, 32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // H1 = relu(P W1 + b1): W1 is [n_in x H] (N contiguous)
    GemmArgs g = ga(B, H, m->n_in, w.Pb, 32, m->W1_bf16, H);
    g.Cb = w.H1;
    g.ldc = H;
    g.bias = m->b1;
    if ((e = gemm<true, false, EPI_BIAS_RELU>(g, 1, s)) != hipSuccess) return e;
    // H2 = relu(H1 W2 + b2): W2 is [H x H] (N contiguous)
    g = ga(B, H, H, w.H1, H, m->W2_bf16, H);
    g.Cb = w.H2;
    g.ldc = H;
    g.bias = m->b2;
    return gemm<true, false, EPI_BIAS_RELU>(g, 1, s);
}

}  // namespace

extern "C" {

const char *djtled_mlp_last_error(void) { return g_mlp_err.c_str(); }

int djtled_mlp_workspace_size(const djtled_mlp *m, int32_t batch, size_t *bytes) {
    int rc = check(m, batch);
    if (rc != DJ_MLP_OK) return rc;
    if (!bytes) return mfail(DJ_MLP_ERR_ARG, "null output");
    WS w;
    return carve(m, batch, nullptr, 0, w, bytes);
}

int djtled_mlp_forward(const djtled_mlp *m, int32_t batch, const float *P, float *Y, void *ws, size_t ws_bytes,
                       void *stream) {
    int rc = check(m, batch);
    if (rc != DJ_MLP_OK) return rc;
    if (!P || !Y || !ws) return mfail(DJ_MLP_ERR_ARG, "null argument");
    WS w;
    if ((rc = carve(m, batch, ws, ws_bytes, w, nullptr)) != DJ_MLP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int H = m->n_hidden;
    if (batch <= 2 && H <= 2048) {
        // inference: streaming products, one launch per layer
        const dim3 gh(unsigned((H + 63) / 64));
        if (batch == 1) {
            hipLaunchKernelGGL((k_gemv_kn<1, true>), gh, dim3(256), 0, s, P, int64_t(m->n_in), m->n_in, m->W1_bf16, H,
                               m->b1, w.H1, int64_t(H));
            hipLaunchKernelGGL((k_gemv_kn<1, false>), gh, dim3(256), 0, s, w.H1, int64_t(H), H, m->W2_bf16, H, m->b2,
                               w.H2, int64_t(H));
        } else {
            hipLaunchKernelGGL((k_gemv_kn<2, true>), gh, dim3(256), 0, s, P, int64_t(m->n_in), m->n_in, m->W1_bf16, H,
                               m->b1, w.H1, int64_t(H));
            hipLaunchKernelGGL((k_gemv_kn<2, false>), gh, dim3(256), 0, s, w.H1, int64_t(H), H, m->W2_bf16, H, m->b2,
                               w.H2, int64_t(H));
        }
        MLP_HIP(hipGetLastError());
        // Y = H2 W3^T + b3: W3 is [ld_out x H] (K contiguous)
        const dim3 grid(unsigned((m->n_out + 255) / 256));
        const int T = (H / 8 + 63) / 64;
        auto run = [&](auto mm, auto tt) {
            hipLaunchKernelGGL((k_gemv<decltype(mm)::value, decltype(tt)::value>), grid, dim3(256), 0, s, w.H2,
                               int64_t(H), H, m->W3_bf16, int64_t(H), m->n_out, m->b3, Y, int64_t(m->ld_out));
        };
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        if (batch == 1) {
            if (T == 1) run(I1(), I1()); else if (T == 2) run(I1(), I2()); else if (T == 3) run(I1(), I3()); else run(I1(), I4());
        } else {
            if (T == 1) run(I2(), I1()); else if (T == 2) run(I2(), I2()); else if (T == 3) run(I2(), I3()); else run(I2(), I4());
        }
        MLP_HIP(hipGetLastError());
        return DJ_MLP_OK;
    }
    MLP_HIP(hidden_forward(m, batch, P, w, s));
    if (w3_stream(batch, H, m->ld_out)) {
        W3Args a{};
        a.B = batch;
        a.H = H;
        a.N = m->n_out;
        a.O = m->ld_out;
        a.H2 = w.H2;
        a.W3 = m->W3_bf16;
        a.bias = m->b3;
        a.Y = Y;
        const int grid = persistent_grid(k_w3_fwd<EPI_BIAS_F32>, 0, (a.O + PNL - 1) / PNL);
        hipLaunchKernelGGL(k_w3_fwd<EPI_BIAS_F32>, dim3(grid), dim3(512), 0, s, a);
        MLP_HIP(hipGetLastError());
        return DJ_MLP_OK;
    }
    // Y = H2 W3^T + b3: W3 is [ld_out x H] (K contiguous)
    GemmArgs g = ga(batch, m->n_out, H, w.H2, H, m->W3_bf16, H);
    g.C = Y;
    g.ldc = m->ld_out;
    g.bias = m->b3;
    MLP_HIP((gemm<true, true, EPI_BIAS_F32>(g, 1, s)));
    return DJ_MLP_OK;
}

int djtled_mlp_loss_grad(const djtled_mlp *m, int32_t batch, const float *P, const float *U, djtled_mlp_grads *gr,
                         double *loss, void *ws, size_t ws_bytes, void *stream) {
    int rc = check(m, batch);
    if (rc != DJ_MLP_OK) return rc;
    if (!P || !U || !gr || !ws || !gr->W1 || !gr->W2 || !gr->W3 || !gr->b1 || !gr->b2 || !gr->b3)
        return mfail(DJ_MLP_ERR_ARG, "null argument");
    WS w;
    if ((rc = carve(m, batch, ws, ws_bytes, w, nullptr)) != DJ_MLP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int B = batch, H = m->n_hidden, O = m->ld_out, NI = m->n_in;
    MLP_HIP(hidden_forward(m, B, P, w, s));
    // loss = mean over (batch, n_out) of (Y - U)^2; dY = 2 (Y - U) / (B n_out)
    const float gscale = float(2.0 / (double(B) * m->n_out));
    GemmArgs g;
    if (w3_stream(B, H, O)) {
        W3Args a{};
        a.B = B;
        a.H = H;
        a.N = O;
        a.O = O;
        a.H2 = w.H2;
        a.W3 = m->W3_bf16;
        a.bias = m->b3;
        a.U = U;
        a.dY = w.dY;
        a.n_valid = m->n_out;
        a.gscale = gscale;
        a.loss_part = w.loss_part;
        a.db3 = gr->b3;
        const int grid = persistent_grid(k_w3_fwd<EPI_LOSS>, 1, (O + PNL - 1) / PNL);
        hipLaunchKernelGGL(k_w3_fwd<EPI_LOSS>, dim3(grid), dim3(512), 0, s, a);
        MLP_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, w.loss_part, grid, 1.0 / (double(B) * m->n_out),
                           w.loss);
        MLP_HIP(hipGetLastError());
        // dW3 [O x H] = dY^T H2 (db3 came with dY)
        const int gd = persistent_grid(k_w3_dw, 2, (O + PNL - 1) / PNL);
        hipLaunchKernelGGL(k_w3_dw, dim3(gd), dim3(512), 0, s, B, H, O, w.H2, w.dY, gr->W3);
        MLP_HIP(hipGetLastError());
        // dH2 [B x H] = dY W3 as partial sums over runs of W3 rows; then their sum under the ReLU mask of H2
        const int nsplit = int(std::min<int64_t>(w.splits, (O + DHN - 1) / DHN));
        hipLaunchKernelGGL(k_w3_dh, dim3(unsigned(nsplit * ((H + DHS - 1) / DHS))), dim3(512), 0, s, B, H, O, nsplit,
                           w.dY, m->W3_bf16, w.part);
        MLP_HIP(hipGetLastError());
        const int64_t bh = int64_t(B) * H;
        hipLaunchKernelGGL(k_splitk_mask, dim3(unsigned((bh + 255) / 256)), dim3(256), 0, s, w.part, nsplit, bh, w.H2,
                           w.dZ2);
        MLP_HIP(hipGetLastError());
    } else {
        g = ga(B, O, H, w.H2, H, m->W3_bf16, H);
        g.Cb = w.dY;
        g.ldc = O;
        g.bias = m->b3;
        g.U = U;
        g.n_valid = m->n_out;
        g.gscale = gscale;
        g.loss_part = w.loss_part;
        MLP_HIP((gemm<true, true, EPI_LOSS>(g, 1, s)));
        const int tiles = ((O + BN - 1) / BN) * ((B + BM - 1) / BM);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, w.loss_part, tiles, 1.0 / (double(B) * m->n_out),
                           w.loss);
        MLP_HIP(hipGetLastError());
        // dW3 [O x H] = dY^T H2  (A = dY: M contiguous; B = H2: N contiguous)
        g = ga(O, H, B, w.dY, O, w.H2, H);
        g.C = gr->W3;
        g.ldc = H;
        MLP_HIP((gemm<false, false, EPI_F32>(g, 1, s)));
        hipLaunchKernelGGL(k_colsum, dim3((O + 31) / 32), dim3(256), 0, s, w.dY, B, O, int64_t(O), gr->b3);
        MLP_HIP(hipGetLastError());
        // dH2 [B x H] = dY W3 (B operand W3 [O x H]: N contiguous), split over K = O; then the ReLU mask of H2
        g = ga(B, H, O, w.dY, O, m->W3_bf16, H);
        g.k_per_split = int(rup((O + w.splits - 1) / w.splits, BKT));
        const int splits = (O + g.k_per_split - 1) / g.k_per_split;
        g.C = w.part;
        g.ldc = H;
        MLP_HIP((gemm<true, false, EPI_SPLITK>(g, splits, s)));
        const int64_t bh = int64_t(B) * H;
        hipLaunchKernelGGL(k_splitk_mask, dim3(unsigned((bh + 255) / 256)), dim3(256), 0, s, w.part, splits, bh, w.H2,
                           w.dZ2);
        MLP_HIP(hipGetLastError());
    }
    // dW2 [H x H] = H1^T dZ2 ; db2
    g = ga(H, H, B, w.H1, H, w.dZ2, H);
    g.C = gr->W2;
    g.ldc = H;
    MLP_HIP((gemm<false, false, EPI_F32>(g, 1, s)));
    hipLaunchKernelGGL(k_colsum, dim3((H + 31) / 32), dim3(256), 0, s, w.dZ2, B, H, int64_t(H), gr->b2);
    MLP_HIP(hipGetLastError());
    // dZ1 [B x H] = (dZ2 W2^T) masked by H1 (B operand W2^T: K contiguous rows of W2)
    g = ga(B, H, H, w.dZ2, H, m->W2_bf16, H);
    g.Cb = w.dZ1;
    g.ldc = H;
    g.aux = w.H1;
    MLP_HIP((gemm<true, true, EPI_MASK>(g, 1, s)));
    // dW1 [n_in x H] = P^T dZ1 ; db1
    g = ga(NI, H, B, w.Pb, 32, w.dZ1, H);
    g.C = gr->W1;
    g.ldc = H;
    MLP_HIP((gemm<false, false, EPI_F32>(g, 1, s)));
    hipLaunchKernelGGL(k_colsum, dim3((H + 31) / 32), dim3(256), 0, s, w.dZ1, B, H, int64_t(H), gr->b1);
    MLP_HIP(hipGetLastError());
    if (loss) {
        MLP_HIP(hipMemcpyAsync(loss, w.loss, sizeof(double), hipMemcpyDeviceToHost, s));
        MLP_HIP(hipStreamSynchronize(s));
    }
    return DJ_MLP_OK;
}

int djtled_mlp_adam(djtled_mlp *m, const djtled_mlp_grads *g, djtled_mlp_grads *mom1, djtled_mlp_grads *mom2,
                    int32_t t, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!m || !g || !mom1 || !mom2 || t < 1) return mfail(DJ_MLP_ERR_ARG, "null argument or t < 1");
    if (!m->W1 || !m->W2 || !m->W3) return mfail(DJ_MLP_ERR_ARG, "null FP32 master weights");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float c1 = float(1.0 - std::pow(double(beta1), t)), c2 = float(1.0 - std::pow(double(beta2), t));
    const int64_t H = m->n_hidden;
    struct T {
        float *w, *g, *m, *v;
        uint16_t *wb;
        int64_t n;
    } ts[6] = {{m->W1, g->W1, mom1->W1, mom2->W1, m->W1_bf16, int64_t(m->n_in) * H},
               {m->b1, g->b1, mom1->b1, mom2->b1, nullptr, H},
               {m->W2, g->W2, mom1->W2, mom2->W2, m->W2_bf16, H * H},
               {m->b2, g->b2, mom1->b2, mom2->b2, nullptr, H},
               {m->W3, g->W3, mom1->W3, mom2->W3, m->W3_bf16, int64_t(m->ld_out) * H},
               {m->b3, g->b3, mom1->b3, mom2->b3, nullptr, int64_t(m->ld_out)}};
    for (const T &x : ts) {
        if (!x.w || !x.g || !x.m || !x.v) return mfail(DJ_MLP_ERR_ARG, "null tensor in Adam");
        hipLaunchKernelGGL(k_adam, dim3(unsigned((x.n + 255) / 256)), dim3(256), 0, s, x.w, x.g, x.m, x.v, x.wb, x.n,
                           lr, beta1, beta2, eps, c1, c2);
        MLP_HIP(hipGetLastError());
    }
    return DJ_MLP_OK;
}

int djtled_mlp_sync_bf16(djtled_mlp *m, void *stream) {
    if (!m || !m->W1 || !m->W2 || !m->W3 || !m->W1_bf16 || !m->W2_bf16 || !m->W3_bf16)
        return mfail(DJ_MLP_ERR_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t H = m->n_hidden;
    const int64_t n[3] = {int64_t(m->n_in) * H, H * H, int64_t(m->ld_out) * H};
    float *w[3] = {m->W1, m->W2, m->W3};
    uint16_t *b[3] = {m->W1_bf16, m->W2_bf16, m->W3_bf16};
    for (int i = 0; i < 3; i++) {
        hipLaunchKernelGGL(k_refresh_bf16, dim3(unsigned((n[i] + 255) / 256)), dim3(256), 0, s, w[i], b[i], n[i]);
        MLP_HIP(hipGetLastError());
    }
    return DJ_MLP_OK;
}

int djtled_mlp_gemm_test(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t lda, int32_t a_kcont,
                         const uint16_t *B, int64_t ldb, int32_t b_kcont, float *C, int64_t ldc, int32_t splits,
                         void *stream) {
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C || splits < 1) return mfail(DJ_MLP_ERR_ARG, "bad GEMM arguments");
    if (lda % 8 || ldb % 8) return mfail(DJ_MLP_ERR_ARG, "leading dimensions must be multiples of 8");
    hipStream_t s = static_cast<hipStream_t>(stream);
    GemmArgs g = ga(M, N, K, A, lda, B, ldb);
    g.C = C;
    g.ldc = ldc;
    g.k_per_split = int(rup((K + splits - 1) / splits, BKT));
    const int z = (K + g.k_per_split - 1) / g.k_per_split;
    hipError_t e;
    if (a_kcont && b_kcont) e = gemm<true, true, EPI_SPLITK>(g, z, s);
    else if (a_kcont) e = gemm<true, false, EPI_SPLITK>(g, z, s);
    else if (b_kcont) e = gemm<false, true, EPI_SPLITK>(g, z, s);
    else e = gemm<false, false, EPI_SPLITK>(g, z, s);
    MLP_HIP(e);
    return z;
}

}  // extern "C"
