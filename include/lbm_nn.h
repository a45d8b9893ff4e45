/*
 * lbm_nn.h - C ABI of the learned coarse-grid corrector of liblbm.so: a small
 * stack of 3x3x3 periodic convolutions trained on the GPU by the library's
 * own forward and backward kernels (bf16 matrix cores, FP32 accumulation)
 * and applied to the macroscopic fields of a coarse lattice Boltzmann run
 * every few steps.  The corrector is not part of the paper: it corrects a
 * coarse run of the method of arXiv:2102.09512 toward box-filtered fine runs
 * of the same method.
 *
 * Network.  Layer l maps c[l] channels to c[l+1] channels:
 *   y[v][o] = b[o] + sum_{t < 27} sum_{i} x[v + s_t][i] W[t][i][o]
 * with s_t = (t%3 - 1, (t/3)%3 - 1, t/9 - 1) (x, y, z offsets, periodic wrap)
 * and a ReLU after every layer but the last.  Supported: c[0] <= 16, hidden
 * widths exactly 32, c[L] <= 32; nx a multiple of 32, ny and nz multiples of 4.
 *
 * Tensors at the ABI are FP32 and planar: x[c][z][y][x] (node = x + nx*(y +
 * ny*z), the node order of lbm.h), on the device (LBM_DEVICE) unless stated.
 * Parameters are one FP32 vector: for each layer W[27][c_in][c_out] then
 * b[c_out].
 *
 * Scaling.  The network sees normalised inputs (x_c - mean_c) / std_c and its
 * output is a normalised correction: the correction in physical units is
 * y_c * out_std_c (lbm_nn_set_scaling; c < c[0] for the input, c < c[L] for
 * the output; c[L] = c[0] for a corrector).
 *
 * Errors as in lbm.h (LBM_OK or a negative code, message in lbm_last_error).
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_nn_ctx* lbm_nn;

/* layers >= 1; channels[0..layers]; dims of the grid the network runs on.
   Allocates parameters, gradients, Adam moments and the activations of one
   sample (about 200 bytes per node). */
int lbm_nn_create(lbm_nn* out, int layers, const int* channels, const int64_t dims[3]);
int lbm_nn_destroy(lbm_nn net);
int lbm_nn_set_stream(lbm_nn net, void* hip_stream);
int64_t lbm_nn_param_count(lbm_nn net);
/* params: lbm_nn_param_count floats (host or device, see mem). */
int lbm_nn_set_params(lbm_nn net, const float* params, int mem);
int lbm_nn_get_params(lbm_nn net, float* params, int mem);
/* Accumulated gradients of the last lbm_nn_loss_backward calls since
   lbm_nn_zero_grad, same layout as the parameters. */
int lbm_nn_get_grads(lbm_nn net, float* grads, int mem);
int lbm_nn_zero_grad(lbm_nn net);
/* mean[c], std[c] (host arrays of c[0] values, std > 0) normalise the input;
   out_std[c] (host array of c[L] values, > 0) scales the output; out_std may
   be NULL, then out_std = std. */
int lbm_nn_set_scaling(lbm_nn net, const double* mean, const double* std, const double* out_std);
/* Output c of the network belongs to input field offset + c (loss and
   correction); offset + c[L] <= c[0].  Default 0.  E.g. offset 1 with
   c[L] = D: the network corrects the velocity only. */
int lbm_nn_set_output_offset(lbm_nn net, int offset);
/* lbm_nn_correct clips each normalised output to [-limit, limit] (so an
   increment is at most limit out_std_c); 0 (default) clips nothing. */
int lbm_nn_set_correction_limit(lbm_nn net, double limit);
/* y = network(normalised x): x is c[0] planes, y is c[L] planes (device). */
int lbm_nn_forward(lbm_nn net, const float* x, float* y);
/* Training loss of one sample and its gradients (accumulated):
     L = mean over nodes and c < c[L] of (y_c + (x_f - t_f) / out_std_c)^2,
   f = offset + c, y = network(normalised x), t the target fields (c[0]
   planes, device); the corrected field x_f + y_c out_std_c is compared with
   t_f in units of out_std_c.
   *loss (host) receives L, and the call is synchronous.  loss NULL: nothing
   waits for the GPU; L is added to a device-side running sum instead (see
   lbm_nn_take_loss). */
int lbm_nn_loss_backward(lbm_nn net, const float* x, const float* target, double* loss);
/* The running sum of the losses of the lbm_nn_loss_backward calls made with
   loss NULL since the last call of this function (*sum, host) and their
   number (*count, host, may be NULL); resets both.  Synchronous. */
int lbm_nn_take_loss(lbm_nn net, double* sum, int64_t* count);
/* One Adam step on the accumulated gradients (scaled by grad_scale), step
   count t >= 1 for the bias correction; then the bf16 weight copies are
   rebuilt. */
int lbm_nn_adam_step(lbm_nn net, double lr, double beta1, double beta2, double eps, double grad_scale, int64_t t);
/* FP64 fields (device) -> FP32 planes x[c][v] (device) for the network:
   c = 0 rho, 1..D u (u holds D planes of nodes values), D + 1 T.  nodes >= 1.
   Runs on hip_stream. */
int lbm_nn_fields_to_planes(int D, int64_t nodes, const double* rho, const double* u, const double* T, float* x,
                            void* hip_stream);
/* Applies the corrector to a lattice Boltzmann handle whose dims equal the
   network's: forms rho, u, T of the stored state, runs the network and adds
   the correction y_c out_std_c to field offset + c (the other fields get
   none) by re-equilibration, as lbm_fields_add does, all on the handle's
   stream and without host synchronisation.  Unlike lbm_fields_add the new
   fields are not validated: bound the correction with
   lbm_nn_set_correction_limit (a limit also turns a non-finite output into
   +-limit) and watch the run with lbm_diagnostics.  Requires c[0] = D + 2. */
int lbm_nn_correct(lbm_nn net, lbm_handle h);

#ifdef __cplusplus
}
#endif
#endif
