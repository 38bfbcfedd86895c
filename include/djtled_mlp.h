/*
 * djtled_mlp.h -- C ABI of the learned warm start's surrogate network
 * (libdjtled.so).
 *
 * The paper names data-driven acceleration of the explicit solve as future
 * work (Sec. 8) and gives no network; this one maps a load-parameter vector p
 * (n_in values) to a displacement field u (n_out values):
 *     H1 = relu(p W1 + b1),  H2 = relu(H1 W2 + b2),  u = H2 W3^T + b3,
 * trained with the mean-squared error against steady states of the plain
 * DJ-TLED dynamic relaxation (djtled_step in RELAX mode) and Adam.  Its
 * prediction seeds u^0 = u^{-1} of a relaxation that still runs to
 * convergence, so the network never decides the final answer.
 *
 * Every dense product runs on the library's BF16 MFMA GEMM (gfx950, FP32
 * accumulation); activations and output gradients are kept in BF16, master
 * weights, gradients and Adam moments in FP32.
 *
 * Conventions: all pointers are device memory owned by the caller; matrices
 * are row-major; `stream` is a hipStream_t passed as void*.  Return codes:
 * DJ_MLP_OK (0) or a negative DJ_MLP_ERR_*; djtled_mlp_last_error() gives a
 * thread-local message.  BF16 tensors are uint16_t bit patterns.
 */
#ifndef DJTLED_MLP_H
#define DJTLED_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DJ_MLP_OK 0
#define DJ_MLP_ERR_ARG (-1)   /* invalid argument or size */
#define DJ_MLP_ERR_HIP (-7)   /* a HIP runtime call failed */

typedef struct {
    int32_t n_in;             /* input width, 1..32 */
    int32_t n_hidden;         /* hidden width, multiple of 8 */
    int32_t n_out;            /* output width */
    int32_t ld_out;           /* padded output width (>= n_out, multiple of 8; a multiple of 64 keeps FP32
                                 rows 256-byte aligned, which the output-layer kernels read whole lines of):
                                 row length of W3^T rows, b3, Y, U */
    float *W1, *b1;           /* FP32 masters: W1 [n_in x n_hidden], b1 [n_hidden] */
    float *W2, *b2;           /* W2 [n_hidden x n_hidden], b2 [n_hidden] */
    float *W3, *b3;           /* W3 [ld_out x n_hidden] (one row per output), b3 [ld_out] */
    uint16_t *W1_bf16, *W2_bf16, *W3_bf16;  /* BF16 copies used by the products (same layouts) */
} djtled_mlp;

/* Gradients, or Adam moments: FP32 tensors of the shapes of the masters. */
typedef struct {
    float *W1, *b1, *W2, *b2, *W3, *b3;
} djtled_mlp_grads;

/* Bytes of device workspace djtled_mlp_forward / djtled_mlp_loss_grad need for `batch` rows. */
int djtled_mlp_workspace_size(const djtled_mlp *m, int32_t batch, size_t *bytes);

/*
 * djtled_mlp_forward -- Y [batch x ld_out] (FP32, columns < n_out written) =
 * the network applied to P [batch x n_in] (FP32).  Uses the BF16 weights.
 * Asynchronous on stream.
 */
int djtled_mlp_forward(const djtled_mlp *m, int32_t batch, const float *P, float *Y, void *workspace,
                       size_t workspace_bytes, void *stream);

/*
 * djtled_mlp_loss_grad -- forward pass, loss = mean over (row, column < n_out)
 * of (Y - U)^2 for targets U [batch x ld_out] (FP32), and the gradients of the
 * loss with respect to every parameter (FP32, overwritten).  *loss (host, may
 * be NULL) receives the loss; when given, the call synchronises the stream.
 */
int djtled_mlp_loss_grad(const djtled_mlp *m, int32_t batch, const float *P, const float *U, djtled_mlp_grads *grads,
                         double *loss, void *workspace, size_t workspace_bytes, void *stream);

/*
 * djtled_mlp_adam -- one Adam step (bias-corrected, step number t >= 1) on
 * every FP32 master from grads and the moments m1, m2 (updated in place),
 * then refreshes the BF16 copies.  Asynchronous on stream.
 */
int djtled_mlp_adam(djtled_mlp *m, const djtled_mlp_grads *grads, djtled_mlp_grads *m1, djtled_mlp_grads *m2,
                    int32_t t, float lr, float beta1, float beta2, float eps, void *stream);

/* BF16 copies <- FP32 masters (after the caller initialises the masters). */
int djtled_mlp_sync_bf16(djtled_mlp *m, void *stream);

/*
 * djtled_mlp_gemm_test -- the library's BF16 MFMA product on its own, for
 * tests: C[z][M x N] (FP32, ldc) = sum over the K slice z of A(m, k) B(k, n),
 * with A(m, k) = A[m lda + k] if a_kcont else A[k lda + m], and B(k, n) =
 * B[n ldb + k] if b_kcont else B[k ldb + n]; K split into `splits` slices of
 * a multiple of 32.  Returns the number of slices written (>= 1) or an error.
 */
int djtled_mlp_gemm_test(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t lda, int32_t a_kcont,
                         const uint16_t *B, int64_t ldb, int32_t b_kcont, float *C, int64_t ldc, int32_t splits,
                         void *stream);

const char *djtled_mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DJTLED_MLP_H */
