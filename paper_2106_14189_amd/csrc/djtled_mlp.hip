// Surrogate MLP for the learned warm start: p (n_in) -> relu(W1) -> relu(W2)
// -> W3 -> u (n_out), trained with mean-squared error and Adam.  All dense
// products run on a BF16 MFMA GEMM for gfx950 (v_mfma_f32_32x32x16_bf16, FP32
// accumulation) with fused epilogues (bias + ReLU, loss + output gradient,
// ReLU masks, split-K partials); small reductions and Adam are elementwise
// kernels.  GEMM operands are BF16; master weights, gradients and Adam moments
// are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/djtled_mlp.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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
__global__ void k_colsum(const uint16_t *__restrict__ X, int M, int N, int64_t ld, float *__restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int m = 0; m < M; m++) s += bf2f(X[int64_t(m) * ld + n]);
    out[n] = s;
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
    const size_t odY = take(size_t(B) * O * 2), odZ2 = take(size_t(B) * H * 2), odZ1 = take(size_t(B) * H * 2);
    const size_t opart = take(size_t(splits) * B * H * 4), olp = take(size_t(tiles) * 8), ol = take(8);
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
    MLP_HIP(hidden_forward(m, batch, P, w, s));
    // Y = H2 W3^T + b3: W3 is [ld_out x H] (K contiguous)
    GemmArgs g = ga(batch, m->n_out, m->n_hidden, w.H2, m->n_hidden, m->W3_bf16, m->n_hidden);
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
    GemmArgs g = ga(B, O, H, w.H2, H, m->W3_bf16, H);
    g.Cb = w.dY;
    g.ldc = O;
    g.bias = m->b3;
    g.U = U;
    g.n_valid = m->n_out;
    g.gscale = float(2.0 / (double(B) * m->n_out));
    g.loss_part = w.loss_part;
    MLP_HIP((gemm<true, true, EPI_LOSS>(g, 1, s)));
    const int tiles = ((O + BN - 1) / BN) * ((B + BM - 1) / BM);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, w.loss_part, tiles, 1.0 / (double(B) * m->n_out), w.loss);
    MLP_HIP(hipGetLastError());
    // dW3 [O x H] = dY^T H2  (A = dY: M contiguous; B = H2: N contiguous)
    g = ga(O, H, B, w.dY, O, w.H2, H);
    g.C = gr->W3;
    g.ldc = H;
    MLP_HIP((gemm<false, false, EPI_F32>(g, 1, s)));
    hipLaunchKernelGGL(k_colsum, dim3((O + 255) / 256), dim3(256), 0, s, w.dY, B, O, int64_t(O), gr->b3);
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
    // dW2 [H x H] = H1^T dZ2 ; db2
    g = ga(H, H, B, w.H1, H, w.dZ2, H);
    g.C = gr->W2;
    g.ldc = H;
    MLP_HIP((gemm<false, false, EPI_F32>(g, 1, s)));
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, w.dZ2, B, H, int64_t(H), gr->b2);
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
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, w.dZ1, B, H, int64_t(H), gr->b1);
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
