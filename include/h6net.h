/*
 * h6net - learned correction to the helmholtz6 preconditioner (one MI355X, gfx950).
 *
 * The paper's preconditioner is the direct inverse of the 7-point operator
 * A_p (Section 3.3, eq. (3DAP)); its error against the 27-point operator A of
 * eq. (scheme) is what a Krylov method (Section 2) must remove.  This
 * library adds a small convolutional network that maps a residual r to a
 * correction c, used as  z = A_p^{-1} r + c(r)  inside flexible GMRES, with
 * the plain A_p^{-1} r as fallback and acceptance test.  The network is not part of the
 * paper.
 *
 * Network (fixed): three levels with 16 / 32 / 64 channels, zero-padded 3x3x3
 * convolutions with bias, ReLU after every convolution but the last, 2x2x2
 * average pooling (extent ceil(n/2), missing entries count as zero, divisor
 * 8), nearest-neighbour upsampling and channel concatenation [upsampled,
 * skip]:
 *     s1 = R(e1b(R(e1a(x))))  3->16->16      s2 = R(e2b(R(e2a(pool s1))))  16->32->32
 *     b3 = R(b3b(R(b3a(pool s2))))  32->64->64
 *     d2 = R(d2b(R(d2a([up b3, s2]))))  96->32->32
 *     d1 = R(d1b(R(d1a([up d2, s1]))))  48->16->16      y = out(d1)  16->2
 * Input features of a residual r: s = sqrt(mean |r|^2),
 * x = (Re r / s, Im r / s, kh) with kh = Re(k) h; correction c = s (y0 + i y1).
 * Activations and weights are BF16 on the device, every convolution
 * accumulates in FP32 on the matrix cores; master weights, gradients and the
 * Adam state are FP32.  Values stored in BF16: the input features, every
 * hidden layer's output after its ReLU and the pooled values (forward); the
 * output gradient, every convolution's input gradient, the upsampling
 * gradient and each skip gradient plus pooling gradient (training).  The last
 * layer's output is kept in FP32.  Training loss of a pair (r, t):
 * L = sum |c(r) - t|^2 / sum |t|^2.
 *
 * Parameters (host FP32, h6net_param_count() values): for each layer in the
 * order e1a e1b e2a e2b b3a b3b d2a d2b d1a d1b out, the weights W[co][ci][dz][dy][dx]
 * (dz, dy, dx = 0..2 for offsets -1..1) followed by the biases b[co].
 *
 * Vectors r, c, t: device complex128, the helmholtz6 layout (x fastest) on the
 * grid the net was created for.  All entry points are extern "C", never
 * throw, and only enqueue work on the given HIP stream except where stated.
 * Errors use the h6_status codes of helmholtz6.h.
 */
#ifndef H6NET_H
#define H6NET_H

#include "helmholtz6.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h6_net_s* h6_net;

/* Number of FP32 parameters (weights and biases of all layers). */
long long h6net_param_count(void);

/* Creates a network for grids of dims = {n'x, n'y, n'z} (each >= 1, with
 * 48 n'x n'y n'z < 2^31, i.e. up to about 350^3 unknowns: the convolutions
 * address activations with 32-bit offsets; H6_ERR_ARG beyond) and
 * allocates its inference buffers (training buffers on the first training
 * call).  Parameters start at zero; set them with h6net_set_params.
 * hip_stream: stream for the set-up work.  On failure *out is NULL. */
h6_status h6net_create(const int dims[3], void* hip_stream, h6_net* out);

/* Copies count = h6net_param_count() host FP32 values in / out (synchronous).
 * Setting parameters resets the Adam state. */
h6_status h6net_set_params(h6_net net, const float* params, long long count, void* hip_stream);
h6_status h6net_get_params(h6_net net, float* params, long long count, void* hip_stream);

/* c = correction of the residual r (device complex128; r and c must not
 * alias).  kh = Re(k) h of the problem.  A zero residual gives c = 0. */
h6_status h6net_forward(h6_net net, const void* r, double kh, void* c, void* hip_stream);

/* Loss and parameter gradients of one pair (r, t) without an update:
 * grads (host, h6net_param_count() values, parameter layout) and *loss are
 * written on return (synchronises hip_stream).  grads may be NULL. */
h6_status h6net_gradients(h6_net net, const void* r, double kh, const void* t, float* grads,
                          double* loss, void* hip_stream);

/* One Adam step (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, learning rate lr)
 * on the pair (r, t); *loss (host, may be NULL) is the loss before the step
 * (synchronises hip_stream when loss is not NULL). */
h6_status h6net_train_step(h6_net net, const void* r, double kh, const void* t, float lr,
                           double* loss, void* hip_stream);

/* Operator-weighted loss of a pair (r, t) on a plan's grid (the quantity the
 * solver's acceptance test measures: with t = e - A_p^{-1} r, A t = r - A A_p^{-1} r):
 *   L_A = sum |A (c(r) - t)|^2 / sum |A t|^2,  A = the plan's operator of
 * eq. (scheme) (helmholtz6_apply_A), kh = Re(k) h of the plan.  The gradient
 * takes the adjoint of A as conj(A conj(.)), exact for all-Dirichlet faces
 * (A complex symmetric); with Neumann or Sommerfeld faces this defines the
 * training gradient.  Same outputs and synchronisation as h6net_gradients /
 * h6net_train_step; the net must have been created for the plan's dims
 * (H6_ERR_ARG otherwise).  Three complex128 work vectors are allocated on
 * first use. */
h6_status h6net_gradients_op(h6_net net, h6_plan plan, const void* r, const void* t, float* grads,
                             double* loss, void* hip_stream);
h6_status h6net_train_step_op(h6_net net, h6_plan plan, const void* r, const void* t, float lr,
                              double* loss, void* hip_stream);

/* Training pair of the correction from an iterate U of a plain solve of
 * A U* = F on the plan's grid: the residual r = F - A U (eq. (scheme)'s
 * operator, FP64) and the target t = (U* - U) - A_p^{-1} r, the part of the
 * error e = U* - U that the plain preconditioner of eq. (3DAP) misses (A e = r;
 * A_p^{-1} in the plan's precision, complex64 arithmetic in H6_MIXED plans).
 * All six vectors are device complex128 on the plan's grid; r and t are
 * outputs and must not alias each other or the inputs.  Uses the plan's
 * preconditioner workspace and reduction buffer (do not overlap with other
 * work on the plan).  Enqueue only. */
h6_status h6net_training_pair(h6_plan plan, const void* F, const void* Ustar, const void* U, void* r,
                              void* t, void* hip_stream);

/* Attaches (net != NULL) or detaches (NULL) the network to a plan: flexible
 * GMRES solves of the plan then use z = A_p^{-1} q + c(q) for the Arnoldi
 * vectors of every restart cycle whose first step the correction does not
 * worsen (||q - A z|| against the plain z = A_p^{-1} q), and the plain
 * preconditioner for the other cycles.  The net must have been created for
 * the plan's dims; kh is taken from the plan.  The plan does not own the
 * net; keep it alive while attached. */
h6_status helmholtz6_attach_net(h6_plan plan, h6_net net);

/* A-applications of the last solve on the plan that used the correction. */
h6_status helmholtz6_learned_steps(h6_plan plan, int* steps);

void h6net_destroy(h6_net net);

#ifdef __cplusplus
}
#endif
#endif /* H6NET_H */
