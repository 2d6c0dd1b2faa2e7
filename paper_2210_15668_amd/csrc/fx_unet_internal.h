// Internal interface between the network (fx_unet.hip) and the stack engine
// (fx_stack.hip): the stack hooks pack the network input from a stack, place
// a prediction into a stack's phi, and form training targets.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/ferrox_unet.h"

namespace fx {

typedef unsigned short bf16_t;       // BF16 bit pattern

// Message returned by last_error() on this thread.
void set_error(const char *msg);

void unet_geometry(const fx_unet *u, int *nx, int *ny, int *nzd, hipStream_t *st);
// per-plane tables held by the network: doping (host N_d - N_a per plane) and
// phi_lin for the stack's relative permittivities and contact potentials
fx_status unet_upload_doping(fx_unet *u, const double *h_doping);
fx_status unet_upload_lin(fx_unet *u, const double *eps_r, double v_bottom, double v_top);
// enqueued on the network's stream
void unet_pack_from_f64(fx_unet *u, const double *P_slab, double v_top);
void unet_forward_enqueue(fx_unet *u);
void unet_apply(fx_unet *u, double *phi_slab);
void unet_make_target(fx_unet *u, const double *phi_slab, float *target);

}  // namespace fx
