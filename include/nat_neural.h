/*
 * nat_neural.h -- C ABI of the neural acoustic transfer field in
 * libnat_bem.so: the network that the Monte-Carlo BEM's data trains
 * (arXiv 2506.06190, Section 3).
 *
 * The field maps a listener position around the object, in spherical
 * coordinates (theta, phi, r) about the scene centre, the object's
 * condition variables v and the frequency f to |p| (Section 3.2):
 *   x  = [ G(theta/pi, phi/(2 pi), (r - r_lo)/(r_hi - r_lo)) | P(v) | P(f) | 0 ]
 *   y  = MLP(x)
 * with (Sections 3.3 and 3.4)
 *  - G: four lattices over the unit cube with 8, 16, 32, 64 cells per axis,
 *    4 features per lattice vertex, trilinear interpolation inside a cell
 *    (coordinates clamped to [0, 1]); a lattice with more than 2^16
 *    vertices keeps them in a table of 2^16 entries addressed by the
 *    spatial hash (i * 1) ^ (j * 2654435761) ^ (k * 805459861) mod 2^16
 *    (unsigned 32-bit products), the others densely at (i n1 + j) n1 + k,
 *    n1 = cells + 1;
 *  - P: sin(2^m pi c), cos(2^m pi c) for m = 0..5 and every scalar c of v
 *    and f, in the order (c, m, sin/cos);
 *  - x padded with zeros to D = a multiple of 16 (D = 16 + 12 (n_v + 1)
 *    rounded up);
 *  - MLP: 4 hidden layers of 128 with ReLU, a linear output layer of
 *    n_out, weights and biases;
 *  - loss: mean squared error over the batch and the outputs;
 *  - Adam (beta1 0.9, beta2 0.999, eps 1e-8), learning rate 1e-3 times
 *    0.33 after each third of the run's steps.
 *
 * Precision: the MLP's inputs, weights, hidden activations and
 * back-propagated gradients are stored in bfloat16 (round to nearest even)
 * and multiplied on the matrix cores with FP32 accumulation; the grid
 * features, biases, the output, the loss and every parameter with its Adam
 * moments are FP32.  The grid-feature gradient is summed in 64-bit fixed
 * point (units of 2^-e, e chosen from the batch size and the largest
 * back-propagated grid feature so that no sum can overflow); every other
 * sum runs in a fixed order that depends only on the batch size, so a
 * gradient is the same on every run.
 *
 * Parameters (host arrays of nat_nf_set_params and friends) are one FP32
 * array in this order: for layer i = 0..4 the weights W_i [out_i][in_i]
 * then the biases b_i [out_i] (in_0 = D, out_0..3 = in_1..4 = 128,
 * out_4 = n_out); then for lattice l = 0..3 its table [size_l][4]
 * (size_l = min((8 * 2^l + 1)^3, 2^16)).
 *
 * Inputs (device) are FP32 rows [B][3 + n_v + 1] = (theta, phi, r,
 * v_0 .. v_{n_v-1}, f) with f already normalised to [0, 1]; targets
 * (device) are FP32 rows [B][n_out].  The conventions of nat_bem.h apply:
 * plain pointers, stream-ordered device work, NAT_E_INVALID before any
 * device work for a bad argument, NAT_E_HIP for a runtime failure, device
 * memory charged to the context's HBM budget.  A field's calls are made by
 * one host thread at a time, on one stream at a time.
 */
#ifndef NAT_NEURAL_H
#define NAT_NEURAL_H

#include <stdint.h>

#include "nat_bem.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nat_nf nat_nf;

/* A field with n_v condition variables (0..16) and n_out outputs (1..32)
 * over the training shell r_lo < r_hi, parameters initialised from seed
 * (Glorot-uniform weights from a counter-based generator, zero biases,
 * grid features uniform in +-1e-4) and Adam moments at zero.  The call
 * synchronises the device. */
nat_status nat_nf_create(nat_ctx* ctx, int32_t n_v, int32_t n_out, double r_lo, double r_hi,
                         uint64_t seed, nat_nf** out);
void nat_nf_destroy(nat_nf* nf);

/* Input width D and parameter count of the layout above. */
nat_status nat_nf_info(const nat_nf* nf, int32_t* input_dim, int64_t* n_params);

/* Host copies of all parameters (n = the parameter count).  set_params
 * also zeroes the Adam moments; get_grads returns the gradient of the last
 * nat_nf_loss_grad or nat_nf_train_step.  These calls synchronise the
 * device. */
nat_status nat_nf_set_params(nat_nf* nf, const float* params, int64_t n);
nat_status nat_nf_get_params(const nat_nf* nf, float* params, int64_t n);
nat_status nat_nf_get_grads(const nat_nf* nf, float* grads, int64_t n);

/* Loss and gradient of the parameters at one batch of B rows (1 .. 2^24),
 * without changing the parameters.  loss (host, may be NULL) receives the
 * mean squared error; when given, the call waits for the stream. */
nat_status nat_nf_loss_grad(nat_nf* nf, const float* inputs, const float* targets, int32_t B,
                            double* loss, void* stream);

/* One training step: loss and gradient as nat_nf_loss_grad, then the Adam
 * update of step `step` (0-based) of a run of total_steps, whose learning
 * rate is 1e-3 * 0.33^min(2, floor(3 step / total_steps)). */
nat_status nat_nf_train_step(nat_nf* nf, const float* inputs, const float* targets, int32_t B,
                             int32_t step, int32_t total_steps, double* loss, void* stream);

/* Field values out [B][n_out] (device, FP32) at B input rows.  Allocates
 * nothing: the whole forward pass runs in on-chip memory. */
nat_status nat_nf_infer(nat_nf* nf, const float* inputs, int32_t B, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NAT_NEURAL_H */
