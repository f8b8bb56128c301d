/*
 * rad_warmstart.h — C-ABI of librad's warm start for the radiosity solve:
 * a POD basis of solution snapshots and a small perceptron that maps a sun
 * direction to POD coefficients, both on one AMD Instinct MI355X.
 *
 * The paper (Potter et al., arXiv 2209.07632) solves B = E + diag(rho) F B by
 * Jacobi relaxation (section 3 and 5.1), which accepts any starting guess; it
 * has no learned component.  This extension predicts the scattered part
 * B - E of a new sun's solution from solves of earlier suns, so that the
 * solve starts at B^0 = E + Phi c instead of B^0 = E.  rad_solve's warm
 * option (rad.h) judges the guess against the cold start column by column.
 *
 * Conventions are those of rad.h (status codes, rad_last_error, caller-owned
 * pointers, hip_stream may be NULL).  Facet-indexed arrays here are
 * row-major "facet-major" blocks: element (t, c) of an N x R block sits at
 * X[t * ld + c], the layout of rad.h's RAD_ORDER_TREE_RMAJOR; any fixed facet
 * order works as long as every array uses the same one.
 */
#ifndef RAD_WARMSTART_H
#define RAD_WARMSTART_H

#include "rad.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ POD */

/*
 * POD modes of the snapshot block S by the method of snapshots: Gram matrix
 * G = S^T S accumulated in FP64 on the device, its eigenpairs on the host
 * (one-sided Jacobi, FP64), modes Phi = S W Lambda^{-1/2} formed in FP64 and
 * re-orthonormalised by classical Gram-Schmidt applied twice, stored FP32.
 *   S      device, N x M facet-major FP32 (ld lds >= M); one snapshot per column
 *   Phi    device, N x m facet-major FP32 (ld ldp >= m); output
 *   sigma  host, m doubles: singular values of S, decreasing; output
 * 1 <= m <= M <= 1024.  Errors: RAD_EINVAL for bad sizes, null pointers,
 * non-finite snapshots, or snapshots of rank below m; RAD_ENOMEM; RAD_EDEVICE.
 * Synchronises hip_stream.
 */
rad_status rad_pod_build(const float *S, int64_t N, int64_t M, int64_t lds, int32_t m, float *Phi, int64_t ldp,
                         double *sigma, int32_t device, void *hip_stream);

/*
 * Coefficients C[c * m + j] = scale_j * sum_t Phi[t, j] (B[t, c] - E[t, c])
 * for R columns (FP64 accumulation, FP32 result).  E and scale may be NULL
 * (no subtraction, unit scale).  B and E share the leading dimension ldb.
 *   Phi device N x m (ldp); B, E device N x R (ldb); scale device m; C device R x m.
 * Errors: RAD_EINVAL, RAD_EDEVICE.  Enqueued on hip_stream.
 */
rad_status rad_pod_project(const float *Phi, int64_t N, int32_t m, int64_t ldp, const float *B, const float *E,
                           int64_t R, int64_t ldb, const float *scale, float *C, void *hip_stream);

/*
 * Field B[t, c] = E[t, c] + sum_j Phi[t, j] scale_j C[c * m + j] for R
 * columns (E and scale may be NULL).  B must not overlap Phi or C; B == E is
 * allowed.  Errors: RAD_EINVAL, RAD_EDEVICE.  Enqueued on hip_stream.
 */
rad_status rad_pod_expand(const float *Phi, int64_t N, int32_t m, int64_t ldp, const float *C, const float *scale,
                          const float *E, int64_t R, int64_t ldb, float *B, void *hip_stream);

/* ------------------------------------------------------------ perceptron */

typedef struct rad_mlp rad_mlp;

/*
 * Perceptron with layer widths sizes[0..nsizes-1] (2 <= nsizes <= 8, widths
 * 1..1024): hidden layers h = tanh(W h_prev + b), linear output layer.
 * params (host, FP32) packs, layer by layer, W (out x in, row-major) then b;
 * its length is sum over layers of out * in + out.  compute is RAD_F32
 * (FP32 products) or RAD_BF16 (operands rounded to BF16 on the matrix cores,
 * FP32 accumulation, FP32 master parameters and optimizer state).
 * max_batch bounds B in every later call.  Errors: RAD_EINVAL, RAD_ENOMEM,
 * RAD_EDEVICE.  *out is NULL on error.
 */
rad_status rad_mlp_create(const int32_t *sizes, int32_t nsizes, const float *params, int32_t compute,
                          int32_t max_batch, int32_t device, rad_mlp **out);

/* Number of packed parameters (-1 for NULL). */
int64_t rad_mlp_param_count(const rad_mlp *net);

/* Copies the packed parameters to host memory (FP32), or replaces them and
 * resets the optimizer state (set). */
rad_status rad_mlp_get_params(const rad_mlp *net, float *params);
rad_status rad_mlp_set_params(rad_mlp *net, const float *params);

/*
 * Y (device, B x sizes[last], row-major) = network(X) for X (device,
 * B x sizes[0], row-major), 1 <= B <= max_batch.  Enqueued on hip_stream.
 */
rad_status rad_mlp_forward(rad_mlp *net, const float *X, int64_t B, float *Y, void *hip_stream);

/*
 * Loss L = (1 / 2B) sum_b sum_j w_j (y_bj - t_bj)^2 over the batch (X, T
 * device row-major, w device of length sizes[last]) and its gradient by
 * backpropagation, kept in the network for rad_mlp_adam_step.  loss (host)
 * and grad (host, param_count floats) may be NULL.  Synchronises hip_stream
 * when either is requested.
 */
rad_status rad_mlp_loss_grad(rad_mlp *net, const float *X, const float *T, const float *w, int64_t B, double *loss,
                             float *grad, void *hip_stream);

/*
 * One Adam step (Kingma and Ba) on the gradient of the last rad_mlp_loss_grad:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t counting
 * steps since create or set_params.  Enqueued on hip_stream.
 */
rad_status rad_mlp_adam_step(rad_mlp *net, double lr, double beta1, double beta2, double eps, void *hip_stream);

/*
 * steps full-batch training steps (loss/gradient then Adam) on (X, T, w),
 * replayed from one captured HIP graph.  loss_hist (host, steps doubles,
 * may be NULL) receives the loss before each step.  Synchronises hip_stream.
 */
rad_status rad_mlp_train(rad_mlp *net, const float *X, const float *T, const float *w, int64_t B, int32_t steps,
                         double lr, double beta1, double beta2, double eps, double *loss_hist, void *hip_stream);

/* Releases the network.  NULL is allowed. */
void rad_mlp_free(rad_mlp *net);

#ifdef __cplusplus
}
#endif

#endif /* RAD_WARMSTART_H */
