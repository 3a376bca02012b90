/*
 * pts_no.h - C ABI of the learned initial space-time iterate for the BDF1 Newton solver.
 *
 * A spectral neural operator maps the initial condition u^0 of a periodic problem to a
 * prediction of the whole space-time solution U = [u^1 .. u^nt]; the Newton iteration
 * of pts_solve then starts from it. The network (all arithmetic in the library's HIP
 * kernels, matrix products on BF16 MFMA with FP32 accumulation):
 *
 *   v_0 = lift_w * u^0 + lift_b                          (pointwise, 1 -> width)
 *   v_{l+1} = GELU(W_l v_l + b_l + K_l v_l),  l = 0..layers-1
 *   c_k = sum_c proj_w[k][c] v_L[c] + proj_b[k]          (pointwise, width -> K = tmodes)
 *   U_pred^n = u^0 + sum_k Phi[n][k] c_k                 (float32 synthesis, K -> nt levels)
 *
 * K_l is the Fourier neural operator's truncated spectral convolution: every complex Fourier
 * mode exp(2 pi i (kx x + ky y)) with |kx|, |ky| < m of every channel is multiplied by a
 * complex width x width matrix W = alpha + i beta. Fields are held in the real basis
 * phi_k(x) = cos(2 pi k x) for k = 0..m-1 and phi_{m-1+k}(x) = sin(2 pi k x) for k = 1..m-1
 * (x = i / nx on the periodic unit square, likewise in y), 2m - 1 functions per direction:
 *   vhat[c][a][b] = (1/(nx ny)) sum_{j,i} v[c][j][i] phi_a(y_j) phi_b(x_i),
 *   what = the mode-wise complex mixing of vhat,
 *   (K_l v)[c'][j][i] = sum_{a,b} what[c'][a][b] phi_a(y_j) phi_b(x_i).
 * For kx, ky >= 1 the coefficients A (cos y cos x), B (cos y sin x), C (sin y cos x),
 * D (sin y sin x) carry the amplitudes z+ = (A - D)/2 - i (B + C)/2 of exp(i(x + y)) and
 * z- = (A + D)/2 - i (B - C)/2 of exp(i(x - y)); z+ is multiplied by
 * alpha+ + i beta+ = R[cos ky][cos kx] + i R[cos ky][sin kx], z- by
 * alpha- + i beta- = R[sin ky][cos kx] + i R[sin ky][sin kx]. With one zero frequency the
 * (cos, sin) pair carries z = cos-coefficient - i sin-coefficient, multiplied by
 * R[cos] + i R[sin]; the mean is multiplied by R[0][0].
 * GELU(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
 *
 * Phi [nt][K] is the temporal basis: the Gram-Schmidt orthonormalisation (in order, over
 * the nt levels) of s_k(n) = sin(pi (k - 1/2) n / nt), n = 1..nt, k = 1..K. Its columns are
 * smooth in time and vanish at t = 0, so a prediction is continuous with u^0 and its error
 * varies smoothly from level to level; orthonormality makes the mean-squared error over
 * the levels equal to |c - c_true|^2 / (nt nx ny) plus a term independent of the network,
 * with c_true = Phi^T (U_true - u^0) (pts_no_encode). Training can therefore keep the
 * encoded targets (K fields per sample instead of nt) resident in device memory.
 *
 * Parameters are one float32 device array in this order:
 *   lift_w[width], lift_b[width],
 *   per layer: W[width][width] (row = output channel), b[width],
 *              R[(2m-1)*(2m-1)][width][width] (basis pair a * (2m-1) + b, then output, input channel),
 *   proj_w[tmodes][width], proj_b[tmodes].
 *
 * Conventions of pts.h apply (device pointers, stream ordering, return codes,
 * pts_last_error).
 */
#ifndef PTS_NO_H
#define PTS_NO_H

#include <stddef.h>
#include <stdint.h>

#include "pts.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pts_no_config {
  int32_t nx, ny;  /* periodic grid of u^0 (the problem's grid)                     */
  int32_t nt;      /* predicted levels                                            */
  int32_t width;   /* channels, multiple of 16, <= 64                             */
  int32_t modes;   /* m: frequencies |k| < m per direction (2m - 1 basis functions),
                      1..32 and 2m <= min(nx, ny)                                  */
  int32_t layers;  /* spectral layers, 1..8                                       */
  int32_t tmodes;  /* K: temporal modes, 1..64 and <= nt                          */
} pts_no_config;

/* Judge of pts_no_initial_iterate: the norm in which the Newton residual R of the two
   candidates is compared. */
#define PTS_NO_JUDGE_RESIDUAL 0    /* max_{n,p} |R^n_p|                                     */
#define PTS_NO_JUDGE_ACCUMULATED 1 /* max_{n,p} |sum_{m<=n} R^m_p|: the Newton correction of
                                      the block forward substitution (Section 3, Eq. (7))
                                      with every diagonal block A_n replaced by I, a cheap
                                      estimate of the iterate's error                       */

/* Number of float32 parameters (layout above). 0 for an invalid configuration. */
size_t pts_no_param_count(const pts_no_config* cfg);

/* Device workspace for one sample: the spatial and temporal bases, activations kept for the
   backward pass, and scratch. */
size_t pts_no_workspace_bytes(const pts_no_config* cfg);

/* Fill the bases of a workspace (the trigonometric basis in x and y and Phi), once after it
   is allocated and before any other call uses it; the other calls read them and leave them
   intact. A workspace is tied to its configuration. */
int pts_no_prepare(const pts_no_config* cfg, void* workspace, size_t workspace_bytes, pts_stream_t stream);

/* U_pred [nt][ny][nx] (float64) from u0 [ny][nx] (float64). Keeps the activations and the
   coefficient fields in the workspace for a following pts_no_backward or
   pts_no_backward_coef on the same sample. U_pred may be NULL: then only the coefficient
   fields are formed (training in coefficient space). */
int pts_no_forward(const pts_no_config* cfg, const float* params, const double* u0, double* U_pred,
                   void* workspace, size_t workspace_bytes, pts_stream_t stream);

/* The forward pass of `batch` samples at once: U_pred[b] from u0[b] (device arrays, as
   pts_no_forward). The spectral transforms run over the channels of all samples together and
   the channel mixes as batched products, so the launches carry `batch` times the work. The
   workspace (pts_no_workspace_bytes_batched(cfg, batch) bytes) is prepared with pts_no_prepare
   like a one-sample workspace; its activations are not kept for a backward pass. */
size_t pts_no_workspace_bytes_batched(const pts_no_config* cfg, int batch);
int pts_no_forward_batched(const pts_no_config* cfg, const float* params, int batch, const double* const* u0,
                           double* const* U_pred, void* workspace, size_t workspace_bytes, pts_stream_t stream);

/* Mean-squared-error loss against U_true [nt][ny][nx] (float64) after pts_no_forward on the
   same sample and workspace: grads (float32, param_count) and loss (device double[1]) are
   ACCUMULATED into (the caller zeroes them before a batch). loss += mean((U_pred-U_true)^2),
   grads += its gradient. */
int pts_no_backward(const pts_no_config* cfg, const float* params, const double* u0, const double* U_pred,
                    const double* U_true, float* grads, double* loss, void* workspace, size_t workspace_bytes,
                    pts_stream_t stream);

/* Coefficient-space loss after pts_no_forward on the same sample and workspace: coef_true
   [tmodes][ny][nx] (float32, e.g. from pts_no_encode). loss += |c - c_true|^2 / (nt nx ny),
   grads += its gradient (accumulated like pts_no_backward; equal to pts_no_backward's for
   U_true = u0 + Phi c_true). */
int pts_no_backward_coef(const pts_no_config* cfg, const float* params, const double* u0, const float* coef_true,
                         float* grads, double* loss, void* workspace, size_t workspace_bytes, pts_stream_t stream);

/* coef [tmodes][ny][nx] (float32) = Phi^T (U - u0) for U [nt][ny][nx], u0 [ny][nx] (float64):
   the training target of a solved sample. Uses the network workspace for Phi. */
int pts_no_encode(const pts_no_config* cfg, const double* u0, const double* U, float* coef, void* workspace,
                  size_t workspace_bytes, pts_stream_t stream);

/* One Adam step (bias-corrected, step >= 1) on n float32 parameters with gradients scaled
   by grad_scale (e.g. 1/batch): m, v are the moment buffers. */
int pts_no_adam(size_t n, float* params, const float* grads, float* m, float* v, int step, float lr, float beta1,
                float beta2, float eps, float grad_scale, pts_stream_t stream);

/* Learned initial iterate with the Newton residual as the judge: U <- U_pred of the
   network if the residual of U_pred is smaller than that of the plain iterate u^n = u^0
   (in the norm `judge` selects, PTS_NO_JUDGE_*), else the plain iterate (the fallback);
   a non-finite prediction always falls back. p must be periodic with p->nx = cfg->nx,
   p->ny = cfg->ny, p->nt = cfg->nt. chosen (host int, may be NULL) receives 1 for the
   prediction, 0 for the fallback; res_pred / res_plain (host doubles, may be NULL)
   receive both norms. The decision is taken on the device: with all three NULL the call
   only enqueues work on the stream; otherwise it synchronises the stream to report them.
   solver_ws is a pts_workspace_bytes(p) workspace (its residual buffer is overwritten). */
int pts_no_initial_iterate(const pts_problem* p, const pts_no_config* cfg, const float* params, const double* u0,
                           double* U, void* no_ws, size_t no_ws_bytes, void* solver_ws, size_t solver_ws_bytes,
                           int judge, int* chosen, double* res_pred, double* res_plain, pts_stream_t stream);

/* pts_no_initial_iterate for `batch` initial conditions of the problem p: one batched
   forward pass (no_ws: a pts_no_workspace_bytes_batched(cfg, batch) workspace), then the judge
   of each instance in turn on solver_ws. chosen (host int[batch], may be NULL) as for the
   one-sample call (then the stream is synchronised). */
int pts_no_initial_iterate_batched(const pts_problem* p, const pts_no_config* cfg, const float* params, int batch,
                                   const double* const* u0, double* const* U, void* no_ws, size_t no_ws_bytes,
                                   void* solver_ws, size_t solver_ws_bytes, int judge, int* chosen,
                                   pts_stream_t stream);

/* Strided batched GEMM used by the network, exposed for testing: for b in [0, batch)
     C_b[m][n] = alpha * sum_k A_b[m][k] B_b[k][n] + beta * C_b[m][n]
   with A_b[m][k] = A[b*bsa + m*sam + k*sak] (likewise B, C), operands rounded to bfloat16
   (nearest even) and products accumulated in float32. */
int pts_no_gemm(int M, int N, int K, float alpha, const float* A, long sam, long sak, long bsa, const float* B,
                long sbk, long sbn, long bsb, float beta, float* C, long scm, long scn, long bsc, int batch,
                pts_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PTS_NO_H */
