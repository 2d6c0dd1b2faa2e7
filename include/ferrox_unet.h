/*
 * ferrox_unet.h -- C ABI of the learned warm start of the Poisson solve.
 *
 * A small 3D convolutional U-Net predicts, from the polarisation P_z, the
 * doping and the gate voltage V of a stack, a starting iterate for the
 * Newton-multigrid solve of eq. (Poisson) with eq. (rho): the network output
 * is the deviation of phi from phi_lin(V), the potential the layered stack
 * would carry with P = 0 and no carriers (a series capacitor).  Multigrid
 * to the stack's tolerance still judges the result: the prediction only
 * replaces the starting iterate (phi^n in the paper's Step 1b, or phi = 0 in
 * Step 0).  The network is trained on the GPU by this library's own forward
 * and backward kernels on (input, phi) snapshots the plain solver produces.
 *
 * Network (fixed): tensors (z, y, x, channel) over the device planes of a
 * stack, channel fastest, BF16 activations and weights with FP32
 * accumulation on the matrix cores.  Three levels with 16, 32 and 64
 * channels; two 3x3x3 convolutions, each followed by ReLU, per level on the
 * way down and on the way up; 2x2x2 average pooling; nearest-neighbour 2x
 * upsampling; skip connections by channel concatenation [upsampled | skip];
 * a 1x1x1 linear head.  Convolutions wrap periodically in x and y and see
 * zeros beyond the z-ends of the device slab.
 *
 * Input channels (16; channels 3..15 are zero): 0 P_z / 0.2 C m^-2,
 * 1 (N_d - N_a) / 1e24 m^-3 of the plane, 2 V / 2 V.  Output: (phi -
 * phi_lin(V)) / 1 V.
 *
 * Parameters: one flat FP32 vector, layers in the order e0a (16->16),
 * e0b (16->16), e1a (16->32), e1b (32->32), b2a (32->64), b2b (64->64),
 * d1a (96->32), d1b (32->32), d0a (48->16), d0b (16->16), each as
 * W[27][cout][cin] then b[cout], where tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)
 * reads the input at (z+dz, y+dy, x+dx); then the head w[16], b.
 * unet_num_params() gives the length (359761).
 *
 * Conventions as in ferrox.h: device pointers on the current device, all
 * work on the stream given to unet_init, fx_status results, last_error()
 * for the message.  The library allocates no device memory: the caller
 * passes the workspace.
 */
#ifndef FERROX_UNET_H
#define FERROX_UNET_H

#include <stddef.h>
#include "ferrox.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fx_unet fx_unet;

size_t unet_num_params(void);

/* Workspace for a network over device slabs of nx * ny * nzd cells (each a
 * multiple of 4, nzd >= 4); train = 1 adds the gradient and optimiser
 * buffers.  0 if the sizes are invalid. */
size_t unet_workspace_bytes(int nx, int ny, int nzd, int train);

/* d_ws: caller-owned device buffer of unet_workspace_bytes(...) bytes,
 * 256-byte aligned.  Parameters start at zero: set them with
 * unet_set_params.  FX_EINVAL for invalid sizes, FX_ENOMEM if ws_bytes is
 * too small. */
fx_status unet_init(int nx, int ny, int nzd, int train, void *d_ws, size_t ws_bytes, void *stream,
                    fx_unet **out);

/* Copy the FP32 parameter vector from / to host memory (unet_num_params()
 * floats).  Setting also resets the optimiser state (Adam moments, step). */
fx_status unet_set_params(fx_unet *u, const float *h_params);
fx_status unet_get_params(fx_unet *u, float *h_params);

/* The network input lives in the workspace.  unet_pack_input fills it from
 * a snapshot: d_P (device, nzd*ny*nx floats, z-major over the device
 * planes), h_doping (host, nzd values of N_d - N_a per plane) and v_top.
 * unet_set_input / unet_get_input copy the whole input tensor
 * (nzd*ny*nx*16 floats, rounded to BF16 when set) to / from the host. */
fx_status unet_pack_input(fx_unet *u, const float *d_P, const double *h_doping, double v_top);
fx_status unet_set_input(fx_unet *u, const float *h_in);
fx_status unet_get_input(fx_unet *u, float *h_in);

/* Forward pass on the current input; d_out (device, nzd*ny*nx floats) may
 * be NULL (the output then stays in the workspace).  Enqueues only. */
fx_status unet_forward(fx_unet *u, float *d_out);

/* Mean squared error of the network on the current input against d_target
 * (device, nzd*ny*nx floats) and its gradient (h_grad: host,
 * unet_num_params() floats, or NULL).  Requires train = 1; synchronises. */
fx_status unet_loss_grad(fx_unet *u, const float *d_target, double *h_loss, float *h_grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * loss against d_target; h_loss (may be NULL) receives the loss before the
 * step, which costs a synchronisation.  Requires train = 1. */
fx_status unet_train_step(fx_unet *u, const float *d_target, float lr, double *h_loss);

fx_status unet_destroy(fx_unet *u);

/* ---------------------------------------------------------- stack hooks
 * The network's slab must be the stack's device slab (same nx, ny and
 * device plane count); FX_EINVAL otherwise. */

/* Fill the network input from the stack's current P, its doping and v_top. */
fx_status stack_unet_input(fx_stack *s, fx_unet *u, double v_top);

/* d_target (device, nzd*ny*nx floats) := (phi - phi_lin(v_top)) / 1 V from
 * the stack's current phi: a training target (u supplies the per-plane
 * table; its input is not touched). */
fx_status stack_unet_target(fx_stack *s, fx_unet *u, double v_top, float *d_target);

/* Learned solve: the network predicts phi from the stack's current P and
 * v_top, phi := phi_lin(v_top) + prediction on the device planes (the
 * stored time levels are dropped), then poisson_solve(s, v_top, info) runs
 * from there: multigrid to tol_rel decides the result, as from any other
 * starting iterate. */
fx_status stack_learned_solve(fx_stack *s, fx_unet *u, double v_top, fx_solve_info *info);

#ifdef __cplusplus
}
#endif

#endif /* FERROX_UNET_H */
