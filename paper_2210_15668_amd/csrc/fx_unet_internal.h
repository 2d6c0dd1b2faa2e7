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

// Forward convolutions on the z-marching kernel (fx_unet_conv.hip).  A launch
// reads CA channels from tensor A (upsampled from the next coarser level when
// upa) and CB channels from tensor B (the skip connection), in that channel
// order; CA = 4 is the packed first layer (3 input channels and a zero).
// out 0: Y = relu(conv + bias) (BF16); out 1: Pf = conv (FP32, ld cout);
// out 2: Y = relu(conv + Pf + bias); out 3: Pf (FP32, one value per voxel) = the
// network's 1x1x1 head (weights hw[0..15], bias hw[16]) on what out 0 would store;
// out 4: Y as out 0 and Yp (BF16, ld cout) = its 2x2x2 average on the coarser level.
// (ca, upa, cb, cout, out) of the network's launches (d1a in two: the upsampled 64
// channels, then the 32 skip channels; b2b in two: input channels 0..31, then 32..63):
#define FX_Z_CONFIGS(F)                                                                               \
    F(4, false, 0, 16, 0) F(16, false, 0, 16, 0) F(32, true, 16, 16, 0) F(16, false, 0, 32, 0)           \
    F(32, false, 0, 32, 0) F(64, true, 0, 32, 1) F(32, false, 0, 32, 2) F(32, false, 0, 64, 0)           \
    F(32, false, 0, 64, 1) F(32, false, 0, 64, 2) F(16, false, 0, 16, 3) F(16, false, 0, 16, 4)          \
    F(32, false, 0, 32, 4)
// weight fragments per 16 output channels
int convz_nfrags(int ca, int cb);
bool convz_supported(int ca, bool upa, int cb, int cout, int out);
// fragment-ordered BF16 weights wz ((cout/16) * nfrags * 512 values) from the
// layer's FP32 W[27][cout][cin] (cin as in the parameter vector; the launch's
// channels start at ci_off)
void convz_prep(const float *theta_w, int cin, int cout, int ca, int cb, int ci_off, bf16_t *wz, hipStream_t st);
// false for an unsupported launch
bool convz_forward(int ca, bool upa, int cb, int cout, int out, const bf16_t *XA, int lda, const bf16_t *XB, int ldb,
                   const bf16_t *wz, const float *bias, bf16_t *Y, int ldy, float *Pf, const float *hw, bf16_t *Yp,
                   int nx, int ny, int nz, hipStream_t st);

}  // namespace fx
