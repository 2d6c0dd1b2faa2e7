// Learned warm start: a 3D convolutional U-Net on the device slab of a stack,
// forward and backward on the matrix cores (gfx950, BF16 operands, FP32
// accumulation), and its Adam training step.
//
// Tensors are (z, y, x, channel), channel fastest, stored as BF16 bit
// patterns.  A 3x3x3 convolution is an implicit GEMM per output voxel block:
// M = output channels, N = voxels, K = 27 taps x input channels, fed to
// v_mfma_f32_16x16x16_bf16 in 16-channel K chunks.  Lane layout of that
// instruction (wave64): lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16]
// and D[4(l/16)+r][l%16], j, r = 0..3; with A = weights W[tap][cout][cin] and
// B = input channels of one neighbour voxel per lane, both operands are one
// 8-byte load per lane and each lane stores 4 consecutive output channels.
//
// The input gradient of a convolution is the same convolution of the output
// gradient with the weights flipped in all three directions and transposed
// (cin <-> cout): the adjoint of "read x at v + d" is "write to v + d", and
// the periodic x-y wrap and the zeros beyond the z-ends are their own adjoints
// under the flip.  The weight gradient sums dZ[v][cout] x[v + d][cin] over all
// voxels: blocks stage 64 voxels of both in LDS and accumulate on the matrix
// cores; per-block partial sums are added in a fixed order (deterministic).
#include "fx_internal.h"
#include "fx_unet_internal.h"
#include "../../include/ferrox_unet.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace fx {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr float kPScale = 0.2f;          // C/m^2
constexpr double kDopingScale = 1e24;    // m^-3
constexpr double kVScale = 2.0;          // V
constexpr double kPhiScale = 1.0;        // V
constexpr int kInC = 4;                  // device input channels: P, doping, V and a zero
constexpr int kInCApi = 16;              // input channels of the parameter layout and the host API

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((unsigned)h << 16); }

// round to nearest even (NaN stays NaN)
__device__ __forceinline__ bf16_t f2bf(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
    return (bf16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------ convolution
// OUT 0: Y (BF16) = relu(conv + bias); OUT 1: Y (FP32) = conv; OUT 2: Y (FP32) += conv.
// Block: 4 waves, each 16 x NTW consecutive voxels and all COUT channels.
template <int CIN, int COUT, int NTW, int OUT>
__global__ __launch_bounds__(256) void k_conv3(const bf16_t *__restrict__ X, int ldx, const bf16_t *__restrict__ Wt,
                                               const float *__restrict__ bias, void *Yv, int ldy, int nx, int ny,
                                               int nz) {
    // with few input channels blockIdx.y picks one 16-channel output tile (more waves in
    // flight on small levels for little extra input traffic); otherwise a wave does all
    constexpr bool MSPLIT = CIN <= 32;
    constexpr int MT = MSPLIT ? 1 : COUT / 16, KC = CIN / 16;
    const int mo = MSPLIT ? blockIdx.y * 16 : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = nx * ny * nz;
    const int v0 = (blockIdx.x * 4 + wave) * (16 * NTW);
    if (v0 >= n) return;
    const int col = lane & 15, kq = lane >> 4;
    int px[NTW], py[NTW], pz[NTW];
    bool ok[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int v = v0 + 16 * t + col;
        ok[t] = v < n;
        const int vv = ok[t] ? v : 0;
        px[t] = vv % nx;
        const int q = vv / nx;
        py[t] = q % ny;
        pz[t] = q / ny;
    }
    f4 acc[MT][NTW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTW; ++t) acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
    const s4 zero4 = {0, 0, 0, 0};
    // 16-channel chunks outer, taps inner: the accumulation order of k_conv3s,
    // so both kernels give bitwise the same result
    for (int kc = 0; kc < KC; ++kc)
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                    s4 b[NTW];
#pragma unroll
                    for (int t = 0; t < NTW; ++t) {
                        const int z2 = pz[t] + dz;
                        int y2 = py[t] + dy, x2 = px[t] + dx;
                        y2 = y2 < 0 ? y2 + ny : (y2 >= ny ? y2 - ny : y2);
                        x2 = x2 < 0 ? x2 + nx : (x2 >= nx ? x2 - nx : x2);
                        const int nb = (ok[t] && z2 >= 0 && z2 < nz) ? (z2 * ny + y2) * nx + x2 : -1;
                        b[t] = nb >= 0 ? *(const s4 *)(X + (size_t)nb * ldx + kc * 16 + 4 * kq) : zero4;
                    }
                    const bf16_t *wtap = Wt + (size_t)tap * COUT * CIN + kc * 16 + 4 * kq;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        const s4 a = *(const s4 *)(wtap + (size_t)(mo + m * 16 + col) * CIN);
#pragma unroll
                        for (int t = 0; t < NTW; ++t)
                            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[m][t], 0, 0, 0);
                    }
                }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        if (!ok[t]) continue;
        const size_t v = (size_t)(v0 + 16 * t + col);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int co = mo + m * 16 + 4 * kq;
            if (OUT == 0) {
                s4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = (short)f2bf(fmaxf(acc[m][t][r] + bias[co + r], 0.f));
                *(s4 *)((bf16_t *)Yv + v * ldy + co) = o;
            } else {
                f4 *dst = (f4 *)((float *)Yv + v * ldy + co);
                if (OUT == 2) *dst = *dst + acc[m][t];
                else *dst = acc[m][t];
            }
        }
    }
}

// The same convolution with the input staged in LDS: a block computes 64
// consecutive x by 4 rows of one plane (a wave per row, 4 column tiles of 16
// voxels); for each 16-channel chunk the 3 x 6 x 66 halo tile is loaded once
// (16-byte loads) and all 27 taps read their B fragments from LDS (each wave
// reads 512 contiguous bytes per fragment: no bank conflicts).  Needs nx a
// multiple of 64 and ny a multiple of 4.
// Move a 4 x bf16 fragment between lanes of a 16-lane row with DPP (register only).

// The same convolution for small grids with the reduction split over the four
// waves of a block: a block owns 16 NTW voxels and every output channel, each
// wave a quarter of the (16-channel chunk, tap) products in the order of
// k_conv3, and wave 0 adds the four partial sums in a fixed order
// (deterministic).  On the coarsest level (32 x 32 x 15 voxels) a wave of
// k_conv3 walks all 27 CIN/16 products one after another; here each wave walks
// a quarter of them with NTW voxel tiles per weight fragment (the fragments of
// 64 output channels, a quarter used per cache line, are the traffic that bounds
// these layers).
template <int CIN, int COUT, int NTW, int OUT>
__global__ __launch_bounds__(256) void k_conv3k(const bf16_t *__restrict__ X, int ldx, const bf16_t *__restrict__ Wt,
                                                const float *__restrict__ bias, void *Yv, int ldy, int nx, int ny,
                                                int nz) {
    constexpr int MT = COUT / 16, KC = CIN / 16, NIT = KC * 27;
    __shared__ f4 part[3][MT][NTW][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = nx * ny * nz;
    const int col = lane & 15, kq = lane >> 4;
    int px[NTW], py[NTW], pz[NTW];
    bool ok[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int v = (blockIdx.x * NTW + t) * 16 + col;
        ok[t] = v < n;
        const int vv = ok[t] ? v : 0;
        px[t] = vv % nx;
        const int q = vv / nx;
        py[t] = q % ny;
        pz[t] = q / ny;
    }
    f4 acc[MT][NTW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTW; ++t) acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
    const s4 zero4 = {0, 0, 0, 0};
    const int it0 = wave * NIT / 4, it1 = (wave + 1) * NIT / 4;
    // operands of product it: the input fragments (zero beyond the z-ends, read
    // from a valid row and discarded there, so that no load sits under a branch)
    // and the weight fragments of every output tile
    auto fetch = [&](int it, s4 *b, s4 *a) {
        const int kc = it / 27, tap = it - kc * 27;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int z2 = pz[t] + dz;
            int y2 = py[t] + dy, x2 = px[t] + dx;
            y2 = y2 < 0 ? y2 + ny : (y2 >= ny ? y2 - ny : y2);
            x2 = x2 < 0 ? x2 + nx : (x2 >= nx ? x2 - nx : x2);
            const bool in = ok[t] && z2 >= 0 && z2 < nz;
            const int nb = in ? (z2 * ny + y2) * nx + x2 : 0;
            const s4 bv = *(const s4 *)(X + (size_t)nb * ldx + kc * 16 + 4 * kq);
            b[t] = in ? bv : zero4;
        }
        const bf16_t *wtap = Wt + (size_t)tap * COUT * CIN + kc * 16 + 4 * kq;
#pragma unroll
        for (int m = 0; m < MT; ++m) a[m] = *(const s4 *)(wtap + (size_t)(m * 16 + col) * CIN);
    };
    // groups of G products: all their loads first, then their MFMAs in order
    constexpr int G = (MT + 1) * NTW <= 20 ? 3 : 1;
    int it = it0;
    for (; it + G <= it1; it += G) {
        s4 b[G][NTW], a[G][MT];
#pragma unroll
        for (int u = 0; u < G; ++u) fetch(it + u, b[u], a[u]);
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < NTW; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[u][m], b[u][t], acc[m][t], 0, 0, 0);
    }
    for (; it < it1; ++it) {
        s4 b[NTW], a[MT];
        fetch(it, b, a);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NTW; ++t)
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[m], b[t], acc[m][t], 0, 0, 0);
    }
    if (wave > 0) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NTW; ++t) part[wave - 1][m][t][lane] = acc[m][t];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        if (!ok[t]) continue;
        const size_t v = (size_t)(blockIdx.x * NTW + t) * 16 + col;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            f4 s = acc[m][t];
            s = s + part[0][m][t][lane];
            s = s + part[1][m][t][lane];
            s = s + part[2][m][t][lane];
            const int co = m * 16 + 4 * kq;
            if (OUT == 0) {
                s4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = (short)f2bf(fmaxf(s[r] + bias[co + r], 0.f));
                *(s4 *)((bf16_t *)Yv + v * ldy + co) = o;
            } else {
                f4 *dst = (f4 *)((float *)Yv + v * ldy + co);
                if (OUT == 2) *dst = *dst + s;
                else *dst = s;
            }
        }
    }
}

template <int CTRL>
__device__ __forceinline__ s4 dpp_s4(s4 v) {
    union {
        s4 s;
        int i[2];
    } u;
    u.s = v;
    u.i[0] = __builtin_amdgcn_update_dpp(0, u.i[0], CTRL, 0xF, 0xF, true);
    u.i[1] = __builtin_amdgcn_update_dpp(0, u.i[1], CTRL, 0xF, 0xF, true);
    return u.s;
}
// The fragment of voxel (col + DX) of a 16-voxel tile: lane col + DX of the same row,
// or, past the row's end, lane col + DX - 16 of the next tile's fragment.
template <int DX>
__device__ __forceinline__ s4 shift_frag(s4 cur, s4 next, int col) {
    const s4 a = dpp_s4<0x100 + DX>(cur);         // row_shl: lane i reads lane i + DX
    const s4 b = dpp_s4<0x110 + 16 - DX>(next);   // row_shr: lane i reads lane i - (16 - DX)
    return col + DX < 16 ? a : b;
}

template <int CIN, int COUT, int OUT>
__global__ __launch_bounds__(256) void k_conv3s(const bf16_t *__restrict__ X, int ldx, const bf16_t *__restrict__ Wt,
                                                const float *__restrict__ bias, void *Yv, int ldy, int nx, int ny,
                                                int nz) {
    constexpr int MT = COUT / 16, KC = CIN / 16, HX = 66, HY = 6;
    __shared__ bf16_t halo[3 * HY * HX * 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int ntx = nx >> 6, nty = ny >> 2;
    const int tx = blockIdx.x % ntx, q0 = blockIdx.x / ntx, ty = q0 % nty, z = q0 / nty;
    const int x0 = tx * 64, y0 = ty * 4;
    f4 acc[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
    typedef int i4 __attribute__((ext_vector_type(4)));
    for (int kc = 0; kc < KC; ++kc) {
        // stage: 3*6*66 voxels x 32 bytes, 16 bytes per thread and step
        for (int u = threadIdx.x; u < 3 * HY * HX * 2; u += 256) {
            const int vi = u >> 1, half = u & 1;
            const int xx = vi % HX, r = vi / HX, dyh = r % HY, dzh = r / HY;
            const int z2 = z + dzh - 1;
            i4 val = {0, 0, 0, 0};
            if (z2 >= 0 && z2 < nz) {
                int y2 = y0 + dyh - 1, x2 = x0 + xx - 1;
                y2 = y2 < 0 ? y2 + ny : (y2 >= ny ? y2 - ny : y2);
                x2 = x2 < 0 ? x2 + nx : (x2 >= nx ? x2 - nx : x2);
                val = *(const i4 *)(X + (size_t)((z2 * ny + y2) * nx + x2) * ldx + kc * 16 + half * 8);
            }
            *(i4 *)(halo + vi * 16 + half * 8) = val;
        }
        // with two output tiles the chunk's weight fragments of all taps are loaded into
        // registers before the taps (measured: helps there, not with one tile or more)
        constexpr bool WREG = MT == 2;
        s4 wr[WREG ? 27 : 1][WREG ? MT : 1];
        if (WREG)
#pragma unroll
            for (int tp = 0; tp < 27; ++tp)
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    wr[tp][m] = *(const s4 *)(Wt + (size_t)tp * COUT * CIN + kc * 16 + 4 * kq +
                                              (size_t)(m * 16 + col) * CIN);
        __syncthreads();
        for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy) {
                const bf16_t *hrow = halo + ((dz * HY + wave + dy) * HX) * 16;
                // the row's fragments at dx = 0 (and the two voxels past the 64);
                // dx = 1, 2 are the same voxels shifted along each 16-lane row
                s4 b0[5];
#pragma unroll
                for (int t = 0; t < 5; ++t) b0[t] = *(const s4 *)(hrow + min(16 * t + col, HX - 1) * 16 + 4 * kq);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int tap = dz * 9 + dy * 3 + dx;
                    s4 b[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        b[t] = dx == 0 ? b0[t] : (dx == 1 ? shift_frag<1>(b0[t], b0[t + 1], col)
                                                          : shift_frag<2>(b0[t], b0[t + 1], col));
                    const bf16_t *wtap = Wt + (size_t)tap * COUT * CIN + kc * 16 + 4 * kq;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        const s4 a = WREG ? wr[WREG ? tap : 0][WREG ? m : 0]
                                          : *(const s4 *)(wtap + (size_t)(m * 16 + col) * CIN);
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[m][t], 0, 0, 0);
                    }
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const size_t v = ((size_t)z * ny + y0 + wave) * nx + x0 + 16 * t + col;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int co = m * 16 + 4 * kq;
            if (OUT == 0) {
                s4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = (short)f2bf(fmaxf(acc[m][t][r] + bias[co + r], 0.f));
                *(s4 *)((bf16_t *)Yv + v * ldy + co) = o;
            } else {
                f4 *dst = (f4 *)((float *)Yv + v * ldy + co);
                if (OUT == 2) *dst = *dst + acc[m][t];
                else *dst = acc[m][t];
            }
        }
    }
}

// Weight gradient of one tap (blockIdx.y): part[bx][tap][cout][cin] =
// sum over the block's voxels of G[v][cout] X[v + d_tap][cin].  Each round stages
// 128 voxels of both operands in LDS, transposed ([channel][voxel]) so that every
// matrix-core fragment is one 8-byte read; staging moves 8 channels (16 bytes) of one
// voxel per load, its neighbour index worked out once per such piece.
template <int CIN, int COUT, int XL = CIN>
__global__ __launch_bounds__(256) void k_wgrad(const bf16_t *__restrict__ X, int ldx, const bf16_t *__restrict__ G,
                                               int nx, int ny, int nz, float *__restrict__ part) {
    constexpr int VB = 128;
    __shared__ bf16_t gt[COUT * VB];
    __shared__ bf16_t xt[CIN * VB];
    constexpr int MT = COUT / 16, NC = CIN / 16, T = MT * NC, TPW = (T + 3) / 4;
    typedef int i4 __attribute__((ext_vector_type(4)));
    const int tap = blockIdx.y;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int n = nx * ny * nz, nchunks = (n + VB - 1) / VB;
    f4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int v0 = ch * VB;
        for (int u = threadIdx.x; u < VB * (COUT / 8); u += 256) {
            const int vl = u / (COUT / 8), c8 = (u % (COUT / 8)) * 8;
            const int v = v0 + vl;
            union {
                i4 w;
                bf16_t h[8];
            } val;
            val.w = i4{0, 0, 0, 0};
            if (v < n) val.w = *(const i4 *)(G + (size_t)v * COUT + c8);
#pragma unroll
            for (int j2 = 0; j2 < 8; ++j2) gt[(c8 + j2) * VB + vl] = val.h[j2];
        }
        for (int u = threadIdx.x; u < VB * (CIN / 8); u += 256) {
            const int vl = u / (CIN / 8), c8 = (u % (CIN / 8)) * 8;
            const int v = v0 + vl;
            union {
                i4 w;
                bf16_t h[8];
            } val;
            val.w = i4{0, 0, 0, 0};
            if (v < n) {
                const int x = v % nx, q = v / nx, y = q % ny, z = q / ny;
                const int z2 = z + dz;
                if (z2 >= 0 && z2 < nz) {
                    int y2 = y + dy, x2 = x + dx;
                    y2 = y2 < 0 ? y2 + ny : (y2 >= ny ? y2 - ny : y2);
                    x2 = x2 < 0 ? x2 + nx : (x2 >= nx ? x2 - nx : x2);
                    if constexpr (XL >= 8) {
                        val.w = *(const i4 *)(X + (size_t)((z2 * ny + y2) * nx + x2) * ldx + c8);
                    } else if (c8 == 0) {   // XL = 4 channels present, the rest zero
                        typedef int i2 __attribute__((ext_vector_type(2)));
                        const i2 h = *(const i2 *)(X + (size_t)((z2 * ny + y2) * nx + x2) * ldx);
                        val.w[0] = h[0];
                        val.w[1] = h[1];
                    }
                }
            }
#pragma unroll
            for (int j2 = 0; j2 < 8; ++j2) xt[(c8 + j2) * VB + vl] = val.h[j2];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < VB / 16; ++kk) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const int tile = wave + 4 * q;
                if (tile >= T) break;
                const int mt = tile / NC, nt = tile % NC;
                const s4 a = *(const s4 *)(gt + (mt * 16 + col) * VB + kk * 16 + 4 * kq);
                const s4 b = *(const s4 *)(xt + (nt * 16 + col) * VB + kk * 16 + 4 * kq);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float *out = part + ((size_t)blockIdx.x * 27 + tap) * COUT * CIN;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile >= T) break;
        const int mt = tile / NC, nt = tile % NC;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(size_t)(mt * 16 + 4 * kq + r) * CIN + nt * 16 + col] = acc[q][r];
    }
}

// dst[i] (+)= sum over p of part[p][i], p in a fixed order.
__global__ void k_part_sum(const float *__restrict__ part, int nparts, int m, float *__restrict__ dst, int add) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int p = 0; p < nparts; ++p) s += part[(size_t)p * m + i];
        dst[i] = add ? dst[i] + s : s;
    }
}

// ------------------------------------------------------ elementwise parts
// One thread per (coarse voxel, group of 4 channels): the 8 children of a
// coarse voxel (low grid nx, ny, nz) are decoded once and moved as 8-byte
// (BF16) or 16-byte (FP32) vectors.
struct Kids {
    size_t v[8];
};

__device__ __forceinline__ Kids kids_of(size_t p, int nx, int ny) {
    const int x = (int)(p % nx), q = (int)(p / nx), y = q % ny, z = q / ny;
    const size_t NX = 2 * (size_t)nx, NY = 2 * (size_t)ny;
    Kids k;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d) k.v[a * 4 + b * 2 + d] = ((size_t)(2 * z + a) * NY + 2 * y + b) * NX + 2 * x + d;
    return k;
}


// D[children][c] += G[parent][c] / 8.
__global__ void k_pool_bwd(const float *__restrict__ Gr, float *__restrict__ D, int ldd, int C, int nx, int ny, int nz) {
    const int G = C / 4;
    const size_t total = (size_t)nx * ny * nz * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(e % G);
        const size_t p = e / G;
        const Kids k = kids_of(p, nx, ny);
        const f4 a = 0.125f * *(const f4 *)(Gr + p * C + 4 * g);
        for (int q = 0; q < 8; ++q) {
            f4 *d = (f4 *)(D + k.v[q] * ldd + 4 * g);
            *d = *d + a;
        }
    }
}

// Y[children][c] = X[parent][c].
__global__ void k_up(const bf16_t *__restrict__ X, bf16_t *__restrict__ Y, int ldy, int C, int nx, int ny, int nz) {
    const int G = C / 4;
    const size_t total = (size_t)nx * ny * nz * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(e % G);
        const size_t p = e / G;
        const Kids k = kids_of(p, nx, ny);
        const s4 a = *(const s4 *)(X + p * C + 4 * g);
        for (int q = 0; q < 8; ++q) *(s4 *)(Y + k.v[q] * ldy + 4 * g) = a;
    }
}

// D[parent][c] = sum of G[children][c].
__global__ void k_up_bwd(const float *__restrict__ Gr, int ldg, float *__restrict__ D, int C, int nx, int ny, int nz) {
    const int G = C / 4;
    const size_t total = (size_t)nx * ny * nz * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(e % G);
        const size_t p = e / G;
        const Kids k = kids_of(p, nx, ny);
        f4 s = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < 8; ++q) s = s + *(const f4 *)(Gr + k.v[q] * ldg + 4 * g);
        *(f4 *)(D + p * C + 4 * g) = s;
    }
}

// Z = G * [Y > 0] (gradient through a ReLU whose output is Y), as BF16.
__global__ void k_mask(const float *__restrict__ G, int ldg, const bf16_t *__restrict__ Y, int ldy,
                       bf16_t *__restrict__ Z, int C, size_t n) {
    const int Gq = C / 4;
    const size_t total = n * Gq;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(e % Gq);
        const size_t v = e / Gq;
        const f4 gv = *(const f4 *)(G + v * ldg + 4 * g);
        const s4 y = *(const s4 *)(Y + v * ldy + 4 * g);
        s4 o;
        for (int j = 0; j < 4; ++j) o[j] = bf2f((bf16_t)y[j]) > 0.f ? (short)f2bf(gv[j]) : (short)0;
        *(s4 *)(Z + v * C + 4 * g) = o;
    }
}

// Per-block column sums of a BF16 [n][C] tensor: part[block][c].
__global__ __launch_bounds__(256) void k_colsum(const bf16_t *__restrict__ Z, int C, size_t n, float *__restrict__ part) {
    __shared__ float red[256];
    const int c = threadIdx.x % C, lanes = 256 / C * C;
    float s = 0.f;
    if ((int)threadIdx.x < lanes)
        for (size_t v = blockIdx.x * (size_t)(256 / C) + threadIdx.x / C; v < n; v += (size_t)gridDim.x * (256 / C))
            s += bf2f(Z[v * C + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < C) {
        float t = 0.f;
        for (int q = threadIdx.x; q < lanes; q += C) t += red[q];
        part[(size_t)blockIdx.x * C + threadIdx.x] = t;
    }
}

// Head: out[v] = b + sum_c w[c] X[v][c] (X: [n][16]).
__global__ void k_head(const bf16_t *__restrict__ X, const float *__restrict__ wb, float *__restrict__ out, size_t n) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        float s = wb[16];
        const s4 *p = (const s4 *)(X + v * 16);
        for (int q = 0; q < 4; ++q) {
            const s4 a = p[q];
            for (int j = 0; j < 4; ++j) s += wb[4 * q + j] * bf2f((bf16_t)a[j]);
        }
        out[v] = s;
    }
}

// Loss pieces: d[v] = 2 (out - t) / n and per-block sums of (out - t)^2.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ out, const float *__restrict__ tg,
                                              float *__restrict__ d, double *__restrict__ part, size_t n) {
    __shared__ double red[256];
    double s = 0.0;
    const float sc = 2.0f / (float)n;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const float e = out[v] - tg[v];
        d[v] = sc * e;
        s += (double)e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < 256; ++q) t += red[q];
        part[blockIdx.x] = t;
    }
}

__global__ void k_sum_d(const double *__restrict__ part, int n, double scale, double *__restrict__ dst) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < n; ++q) t += part[q];
        *dst = t * scale;
    }
}

// Head backward: Z[v][c] = d[v] w[c] [Y > 0]; per-block sums of d[v] Y[v][c] (c < 16) and d[v] (c = 16).
__global__ __launch_bounds__(256) void k_head_bwd(const float *__restrict__ d, const bf16_t *__restrict__ Y,
                                                  const float *__restrict__ wb, bf16_t *__restrict__ Z,
                                                  float *__restrict__ part, size_t n) {
    __shared__ float red[17][256];
    float s[17];
    for (int c = 0; c < 17; ++c) s[c] = 0.f;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const float g = d[v];
        for (int c = 0; c < 16; ++c) {
            const float y = bf2f(Y[v * 16 + c]);
            s[c] += g * y;
            Z[v * 16 + c] = y > 0.f ? f2bf(g * wb[c]) : (bf16_t)0;
        }
        s[16] += g;
    }
    for (int c = 0; c < 17; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    if (threadIdx.x < 17) {
        float t = 0.f;
        for (int q = 0; q < 256; ++q) t += red[threadIdx.x][q];
        part[(size_t)blockIdx.x * 17 + threadIdx.x] = t;
    }
}

// Adam on the flat parameter vector.
__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       size_t n, float lr, float c1, float c2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = 0.9f * m[i] + 0.1f * gi;
        const float vi = 0.999f * v[i] + 0.001f * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    }
}

// BF16 copies of one layer's weights: wt[t][co][ci] and the flipped,
// transposed wf[26 - t][ci][co] used by the input gradient.
__global__ void k_prep(const float *__restrict__ th, int cin, int cout, bf16_t *__restrict__ wt, bf16_t *__restrict__ wf) {
    const int total = 27 * cin * cout;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int ci = e % cin, q = e / cin, co = q % cout, t = q / cout;
        const bf16_t h = f2bf(th[e]);
        wt[e] = h;
        wf[((size_t)(26 - t) * cin + ci) * cout + co] = h;
    }
}

// Network input from P over the device planes (z-major), doping per plane and V.
template <typename T>
__global__ void k_pack(const T *__restrict__ P, const float *__restrict__ dop, float vs, bf16_t *__restrict__ in,
                       bf16_t *__restrict__ in_xp, int nx, int nxy, size_t n) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        s4 q0;
        q0[0] = (short)f2bf((float)P[v] / kPScale);
        q0[1] = (short)f2bf(dop[v / nxy]);
        q0[2] = (short)f2bf(vs);
        q0[3] = 0;
        *(s4 *)(in + v * kInC) = q0;
        // the x-padded copy: x + 1 in rows of nx + 2; the row ends also land in the
        // wrapped voxels at 0 and nx + 1
        const int x = (int)(v % nx), r = (int)(v / nx);
        bf16_t *row = in_xp + (size_t)r * (nx + 2) * kInC;
        *(s4 *)(row + (x + 1) * kInC) = q0;
        if (x == 0) *(s4 *)(row + (nx + 1) * kInC) = q0;
        if (x == nx - 1) *(s4 *)(row) = q0;
    }
}

// The x-padded copy of the input (after the input was set directly).
__global__ void k_pad_x(const bf16_t *__restrict__ in, bf16_t *__restrict__ in_xp, int nx, size_t n) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const s4 q = *(const s4 *)(in + v * kInC);
        const int x = (int)(v % nx), r = (int)(v / nx);
        bf16_t *row = in_xp + (size_t)r * (nx + 2) * kInC;
        *(s4 *)(row + (x + 1) * kInC) = q;
        if (x == 0) *(s4 *)(row + (nx + 1) * kInC) = q;
        if (x == nx - 1) *(s4 *)(row) = q;
    }
}

__global__ void k_bf_to_f(const bf16_t *__restrict__ a, float *__restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = bf2f(a[i]);
}

__global__ void k_f_to_bf(const float *__restrict__ a, bf16_t *__restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) b[i] = f2bf(a[i]);
}

// phi (device planes) := phi_lin[z] + scale * out.
__global__ void k_apply(const float *__restrict__ out, const double *__restrict__ lin, double *__restrict__ phi, int nxy,
                        size_t n) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        phi[v] = lin[v / nxy] + kPhiScale * (double)out[v];
}

// target := (phi - phi_lin[z]) / scale.
__global__ void k_target(const double *__restrict__ phi, const double *__restrict__ lin, float *__restrict__ tg, int nxy,
                         size_t n) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        tg[v] = (float)((phi[v] - lin[v / nxy]) / kPhiScale);
}

dim3 grid_for(size_t work) {
    const size_t b = (work + 255) / 256;
    return dim3((unsigned)(b == 0 ? 1 : (b < 8192 ? b : 8192)));
}

// -------------------------------------------------------- host dispatch
typedef void (*ConvFn)(const bf16_t *, int, const bf16_t *, const float *, void *, int, int, int, int);

template <int CIN, int COUT, int NTW, int OUT>
void conv_launch(const bf16_t *X, int ldx, const bf16_t *W, const float *b, void *Y, int ldy, int nx, int ny, int nz,
                 bool staged, hipStream_t st) {
    if (staged && nx % 64 == 0 && ny % 4 == 0) {        // LDS-staged input
        hipLaunchKernelGGL((k_conv3s<CIN, COUT, OUT>), dim3((nx / 64) * (ny / 4) * nz), dim3(256), 0, st, X, ldx, W, b,
                           Y, ldy, nx, ny, nz);
        return;
    }
    const int n = nx * ny * nz, per = 64 * NTW;
    // small grid the staged kernel cannot take: reduction split over the waves (where
    // the staged kernel applies, the direct one keeps its accumulation order)
    if constexpr (NTW == 1 && CIN >= 32) {
        if (!(nx % 64 == 0 && ny % 4 == 0)) {
            // four voxel tiles per weight fragment where there are four output tiles
            constexpr int KT = COUT >= 64 ? 4 : 1;
            hipLaunchKernelGGL((k_conv3k<CIN, COUT, KT, OUT>), dim3((n + 16 * KT - 1) / (16 * KT)), dim3(256), 0, st, X,
                               ldx, W, b, Y, ldy, nx, ny, nz);
            return;
        }
    }
    hipLaunchKernelGGL((k_conv3<CIN, COUT, NTW, OUT>), dim3((n + per - 1) / per, CIN <= 32 ? COUT / 16 : 1), dim3(256),
                       0, st, X, ldx, W, b, Y, ldy, nx, ny, nz);
}

// (cin, cout) of the forward layers (weight gradients) and of the convolutions
// that carry the gradient back through them (input gradients)
#define FX_WG_PAIRS(F) F(16, 16) F(16, 32) F(32, 32) F(32, 64) F(64, 64) F(96, 32) F(48, 16)
#define FX_IG_PAIRS(F) F(16, 16) F(16, 48) F(32, 32) F(32, 96) F(64, 64) F(64, 32) F(32, 16)

// Input-gradient convolutions (out 1: Y = conv, out 2: Y += conv, FP32): NTW = 4 on
// large grids, 1 on small ones (more blocks).  The forward pass runs on the
// z-marching kernel (fx_unet_conv.hip).
bool conv_any(int cin, int cout, int out, const bf16_t *X, int ldx, const bf16_t *W, const float *b, void *Y, int ldy,
              int nx, int ny, int nz, bool staged, hipStream_t st) {
    const bool big = (size_t)nx * ny * nz >= (size_t)256 * 64 * 4;
#define FX_CONV_CASE(ci, co)                                                                               \
    if (cin == ci && cout == co) {                                                                         \
        if (out == 1) {                                                                                    \
            if (big) conv_launch<ci, co, 4, 1>(X, ldx, W, b, Y, ldy, nx, ny, nz, staged, st);                       \
            else conv_launch<ci, co, 1, 1>(X, ldx, W, b, Y, ldy, nx, ny, nz, staged, st);                           \
        } else {                                                                                           \
            if (big) conv_launch<ci, co, 4, 2>(X, ldx, W, b, Y, ldy, nx, ny, nz, staged, st);                       \
            else conv_launch<ci, co, 1, 2>(X, ldx, W, b, Y, ldy, nx, ny, nz, staged, st);                           \
        }                                                                                                  \
        return true;                                                                                       \
    }
    if (out == 1 || out == 2) {
        FX_IG_PAIRS(FX_CONV_CASE)
    }
#undef FX_CONV_CASE
    return false;
}

bool wgrad_any(int cin, int cout, const bf16_t *X, int ldx, const bf16_t *G, int nx, int ny, int nz, float *part,
               int nparts, hipStream_t st) {
    if (cin == 16 && cout == 16 && ldx == kInC) {       // the first layer on the 4-channel input
        hipLaunchKernelGGL((k_wgrad<16, 16, kInC>), dim3(nparts, 27), dim3(256), 0, st, X, ldx, G, nx, ny, nz, part);
        return true;
    }
#define FX_WG_CASE(ci, co)                                                                                        \
    if (cin == ci && cout == co) {                                                                                \
        hipLaunchKernelGGL((k_wgrad<ci, co>), dim3(nparts, 27), dim3(256), 0, st, X, ldx, G, nx, ny, nz, part);  \
        return true;                                                                                              \
    }
    FX_WG_PAIRS(FX_WG_CASE)
#undef FX_WG_CASE
    return false;
}

}  // namespace

// ------------------------------------------------------------- the network
struct Layer {
    const char *name;
    int cin, cout, level;
    size_t woff, boff;                  // offsets in the parameter vector
    size_t bf_off;                      // offset of this layer in the BF16 weight arrays
};

static const Layer kLayerTemplate[10] = {
    {"e0a", 16, 16, 0, 0, 0, 0}, {"e0b", 16, 16, 0, 0, 0, 0}, {"e1a", 16, 32, 1, 0, 0, 0}, {"e1b", 32, 32, 1, 0, 0, 0},
    {"b2a", 32, 64, 2, 0, 0, 0}, {"b2b", 64, 64, 2, 0, 0, 0}, {"d1a", 96, 32, 1, 0, 0, 0}, {"d1b", 32, 32, 1, 0, 0, 0},
    {"d0a", 48, 16, 0, 0, 0, 0}, {"d0b", 16, 16, 0, 0, 0, 0}};
enum { E0A, E0B, E1A, E1B, B2A, B2B, D1A, D1B, D0A, D0B, NLAYER };

// Launches of the forward pass on the z-marching kernel: input channels from
// tensor A (ca, upsampled when upa) and B (cb), output mode, first input channel
// of the layer's weights, offset of the fragment-ordered weights.
struct ZLaunch {
    int layer, ca, upa, cb, out, ci_off;
    size_t wz_off;
};
static const ZLaunch kZTemplate[] = {
    {E0A, 4, 0, 0, 0, 0, 0},  {E0B, 16, 0, 0, 0, 0, 0}, {E1A, 16, 0, 0, 0, 0, 0}, {E1B, 32, 0, 0, 0, 0, 0},
    {B2A, 32, 0, 0, 0, 0, 0},
    {B2B, 32, 0, 0, 1, 0, 0},  // input channels 0..31 into an FP32 partial sum,
    {B2B, 32, 0, 0, 2, 32, 0}, // then 32..63, the partial sum, bias and ReLU
    {D1A, 64, 1, 0, 1, 0, 0},  // upsampled 64 channels into an FP32 partial sum,
    {D1A, 32, 0, 0, 2, 64, 0}, // then the 32 skip channels, the partial sum, bias and ReLU
    {D1B, 32, 0, 0, 0, 0, 0}, {D0A, 32, 1, 16, 0, 0, 0}, {D0B, 16, 0, 0, 0, 0, 0}};
enum { ZE0A, ZE0B, ZE1A, ZE1B, ZB2A, ZB2B_LO, ZB2B_HI, ZD1A_UP, ZD1A_SKIP, ZD1B, ZD0A, ZD0B, NZ };

struct UnetLayout {
    Layer L[NLAYER];
    ZLaunch Z[NZ];
    size_t nparams = 0, head_off = 0, nbf = 0, nwz = 0;
    UnetLayout() {
        size_t o = 0, bo = 0;
        for (int i = 0; i < NLAYER; ++i) {
            L[i] = kLayerTemplate[i];
            L[i].woff = o;
            o += (size_t)27 * L[i].cin * L[i].cout;
            L[i].boff = o;
            o += L[i].cout;
            L[i].bf_off = bo;
            bo += (size_t)27 * L[i].cin * L[i].cout;
        }
        head_off = o;
        nparams = o + 17;
        nbf = bo;
        size_t zo = 0;
        for (int i = 0; i < NZ; ++i) {
            Z[i] = kZTemplate[i];
            Z[i].wz_off = zo;
            zo += (size_t)convz_nfrags(Z[i].ca, Z[i].cb) * (L[Z[i].layer].cout / 16) * 512;
        }
        nwz = zo;
    }
};

static const UnetLayout &layout() {
    static const UnetLayout lay;
    return lay;
}

}  // namespace fx

using namespace fx;

struct fx_unet {
    int nx, ny, nz, train;
    bool staged;                        // LDS-staged convolutions where the x-y extents allow
    hipStream_t st;
    size_t n0, n1, n2;                  // voxels per level
    // parameters and optimiser
    float *theta, *grad, *m, *v;
    bf16_t *wt, *wf;
    bf16_t *wz;                         // fragment-ordered weights of the forward launches
    int adam_t;
    // activations (BF16)
    bf16_t *in, *a_e0a, *cat0, *p0, *a_e1a, *cat1, *p1, *a_b2a, *a_b2b, *a_d1a, *a_d1b, *a_d0a, *a_d0b;
    bf16_t *in_xp;                      // the input with one wrapped voxel at each x-end (rows of nx + 2)
    float *out;
    float *zpart;                       // FP32 partial sums of b2b (level 2, 64 channels) and d1a (level 1, 32)
    // gradients (training)
    float *dout, *g0_16, *g0_48, *g1_32a, *g1_32b, *g1_96, *g1_16, *g2_64a, *g2_64b, *g2_32;
    bf16_t *z0, *z1, *z2;
    float *part;                        // weight-gradient partial sums
    size_t part_floats;
    double *dpart, *dscal;
    float *dop;                         // doping per plane (network units)
    double *lin;                        // phi_lin per plane
    double *h_scal;                     // pinned read-back
};

namespace {

fx_status ufail(fx_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
fx_status ufail(fx_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fx::set_error(buf);
    return s;
}

#define UHIP(call)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return ufail(FX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int kWgradParts0 = 128;       // weight-gradient partitions on the finest level

int wgrad_parts(size_t n) {
    const size_t chunks = (n + 63) / 64;
    const size_t p = chunks / 32;       // at least 32 chunks per block
    return (int)(p < 1 ? 1 : (p > kWgradParts0 ? kWgradParts0 : p));
}

struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

bool valid_dims(int nx, int ny, int nz) {
    return nx >= 4 && ny >= 4 && nz >= 4 && nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0 &&
           (double)nx * ny * nz * 48 < 2147483647.0;
}

size_t carve_unet(fx_unet *u, void *ws) {
    Carve cv(ws);
    const UnetLayout &lay = layout();
    const size_t n0 = u->n0, n1 = u->n1, n2 = u->n2;
    u->theta = cv.take<float>(lay.nparams);
    u->wt = cv.take<bf16_t>(lay.nbf);
    u->wf = cv.take<bf16_t>(lay.nbf);
    u->wz = cv.take<bf16_t>(lay.nwz);
    u->in = cv.take<bf16_t>(n0 * kInC);
    u->in_xp = cv.take<bf16_t>((size_t)(u->nx + 2) * u->ny * u->nz * kInC);
    u->a_e0a = cv.take<bf16_t>(n0 * 16);
    u->cat0 = cv.take<bf16_t>(n0 * 48);
    u->p0 = cv.take<bf16_t>(n1 * 16);
    u->a_e1a = cv.take<bf16_t>(n1 * 32);
    u->cat1 = cv.take<bf16_t>(n1 * 96);
    u->p1 = cv.take<bf16_t>(n2 * 32);
    u->a_b2a = cv.take<bf16_t>(n2 * 64);
    u->a_b2b = cv.take<bf16_t>(n2 * 64);
    u->a_d1a = cv.take<bf16_t>(n1 * 32);
    u->a_d1b = cv.take<bf16_t>(n1 * 32);
    u->a_d0a = cv.take<bf16_t>(n0 * 16);
    u->a_d0b = cv.take<bf16_t>(n0 * 16);
    u->out = cv.take<float>(n0);
    u->zpart = cv.take<float>(std::max(n1 * 32, n2 * 64));
    u->dop = cv.take<float>(u->nz);
    u->lin = cv.take<double>(u->nz);
    u->dpart = cv.take<double>(8192);
    u->dscal = cv.take<double>(4);
    if (u->train) {
        u->grad = cv.take<float>(lay.nparams);
        u->m = cv.take<float>(lay.nparams);
        u->v = cv.take<float>(lay.nparams);
        u->dout = cv.take<float>(n0);
        u->g0_16 = cv.take<float>(n0 * 16);
        u->g0_48 = cv.take<float>(n0 * 48);
        u->g1_32a = cv.take<float>(n1 * 32);
        u->g1_32b = cv.take<float>(n1 * 32);
        u->g1_96 = cv.take<float>(n1 * 96);
        u->g1_16 = cv.take<float>(n1 * 16);
        u->g2_64a = cv.take<float>(n2 * 64);
        u->g2_64b = cv.take<float>(n2 * 64);
        u->g2_32 = cv.take<float>(n2 * 32);
        u->z0 = cv.take<bf16_t>(n0 * 16);
        u->z1 = cv.take<bf16_t>(n1 * 32);
        u->z2 = cv.take<bf16_t>(n2 * 64);
        size_t pf = 0;
        for (int i = 0; i < NLAYER; ++i) {
            const Layer &L = lay.L[i];
            const size_t n = L.level == 0 ? n0 : (L.level == 1 ? n1 : n2);
            pf = std::max(pf, (size_t)wgrad_parts(n) * 27 * L.cin * L.cout);
        }
        pf = std::max(pf, (size_t)8192 * 64);           // column-sum partials
        u->part_floats = pf;
        u->part = cv.take<float>(pf);
    } else {
        u->grad = u->m = u->v = u->dout = nullptr;
        u->g0_16 = u->g0_48 = u->g1_32a = u->g1_32b = u->g1_96 = u->g1_16 = u->g2_64a = u->g2_64b = u->g2_32 = nullptr;
        u->z0 = u->z1 = u->z2 = nullptr;
        u->part = nullptr;
        u->part_floats = 0;
    }
    return cv.off + 256;
}

struct Dims {
    int nx, ny, nz;
};

Dims dims_of(const fx_unet *u, int level) {
    return Dims{u->nx >> level, u->ny >> level, u->nz >> level};
}

const bf16_t *wf_of(const fx_unet *u, int l) { return u->wf + layout().L[l].bf_off; }
const float *bias_of(const fx_unet *u, int l) { return u->theta + layout().L[l].boff; }

// Forward launch zi of the z-marching convolution on the level of its layer; out >= 3
// replaces the launch's output mode (3: the head folded in, 4: the pooling folded in,
// into Yp).
void zconv(fx_unet *u, int zi, const bf16_t *XA, int lda, const bf16_t *XB, int ldb, bf16_t *Y, int ldy, int out = -1,
           bf16_t *Yp = nullptr) {
    const UnetLayout &lay = layout();
    const ZLaunch &Z = lay.Z[zi];
    const Layer &L = lay.L[Z.layer];
    const Dims d = dims_of(u, L.level);
    const int o = out >= 0 ? out : Z.out;
    convz_forward(Z.ca, Z.upa != 0, Z.cb, L.cout, o, XA, lda, XB, ldb, u->wz + Z.wz_off, bias_of(u, Z.layer), Y, ldy,
                  o == 3 ? u->out : u->zpart, u->theta + lay.head_off, Yp, d.nx, d.ny, d.nz, u->st);
}

void prep_weights(fx_unet *u) {
    const UnetLayout &lay = layout();
    for (int i = 0; i < NLAYER; ++i) {
        const Layer &L = lay.L[i];
        hipLaunchKernelGGL(k_prep, grid_for((size_t)27 * L.cin * L.cout), dim3(256), 0, u->st, u->theta + L.woff, L.cin,
                           L.cout, u->wt + L.bf_off, u->wf + L.bf_off);
    }
    for (int i = 0; i < NZ; ++i) {
        const ZLaunch &Z = lay.Z[i];
        const Layer &L = lay.L[Z.layer];
        convz_prep(u->theta + L.woff, L.cin, L.cout, Z.ca, Z.cb, Z.ci_off, u->wz + Z.wz_off, u->st);
    }
}

void enqueue_forward(fx_unet *u) {
    const Dims d1 = dims_of(u, 1), d2 = dims_of(u, 2);
    hipStream_t st = u->st;
    // skip connections: inside the concatenated tensors when training (their weight
    // gradients read [upsampled | skip]); compact in the same buffers otherwise (the
    // decoders read the upsampled channels straight from the coarser level)
    bf16_t *s0 = u->train ? u->cat0 + 32 : u->cat0, *s1 = u->train ? u->cat1 + 64 : u->cat1;
    const int l0 = u->train ? 48 : 16, l1 = u->train ? 96 : 32;
    zconv(u, ZE0A, u->in_xp, kInC, nullptr, 0, u->a_e0a, 16);      // x-padded rows of nx + 2
    // the skip layers also write their 2x2x2 averages (the next level's input)
    zconv(u, ZE0B, u->a_e0a, 16, nullptr, 0, s0, l0, 4, u->p0);
    zconv(u, ZE1A, u->p0, 16, nullptr, 0, u->a_e1a, 32);
    zconv(u, ZE1B, u->a_e1a, 32, nullptr, 0, s1, l1, 4, u->p1);
    zconv(u, ZB2A, u->p1, 32, nullptr, 0, u->a_b2a, 64);
    zconv(u, ZB2B_LO, u->a_b2a, 64, nullptr, 0, nullptr, 0);
    zconv(u, ZB2B_HI, u->a_b2a + 32, 64, nullptr, 0, u->a_b2b, 64);
    if (u->train)
        hipLaunchKernelGGL(k_up, grid_for(u->n2 * 16), dim3(256), 0, st, u->a_b2b, u->cat1, 96, 64, d2.nx, d2.ny, d2.nz);
    zconv(u, ZD1A_UP, u->a_b2b, 64, nullptr, 0, nullptr, 0);
    zconv(u, ZD1A_SKIP, s1, l1, nullptr, 0, u->a_d1a, 32);
    zconv(u, ZD1B, u->a_d1a, 32, nullptr, 0, u->a_d1b, 32);
    if (u->train)
        hipLaunchKernelGGL(k_up, grid_for(u->n1 * 8), dim3(256), 0, st, u->a_d1b, u->cat0, 48, 32, d1.nx, d1.ny, d1.nz);
    zconv(u, ZD0A, u->a_d1b, 32, s0, l0, u->a_d0a, 16);
    if (u->train) {                     // the head's gradient reads the last layer's output
        zconv(u, ZD0B, u->a_d0a, 16, nullptr, 0, u->a_d0b, 16);
        hipLaunchKernelGGL(k_head, grid_for(u->n0), dim3(256), 0, st, u->a_d0b, u->theta + layout().head_off, u->out,
                           u->n0);
    } else {                            // the head folded into the last layer
        zconv(u, ZD0B, u->a_d0a, 16, nullptr, 0, nullptr, 0, 3);
    }
}

// Bias gradient of layer l from its BF16 output gradient Z ([n][cout]).
void bias_grad(fx_unet *u, int l, const bf16_t *Z, size_t n) {
    const Layer &L = layout().L[l];
    const int nb = (int)std::min<size_t>(128, (n + 255) / 256);
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(256), 0, u->st, Z, L.cout, n, u->part);
    hipLaunchKernelGGL(k_part_sum, dim3(1), dim3(64), 0, u->st, u->part, nb, L.cout, u->grad + L.boff, 0);
}

// Weight and bias gradient of layer l (input X, ld ldx; output gradient Z),
// and optionally its input gradient into G (FP32, ld ldg; add = accumulate).
void layer_backward(fx_unet *u, int l, const bf16_t *X, int ldx, const bf16_t *Z, float *G, int ldg, int add) {
    const Layer &L = layout().L[l];
    const Dims d = dims_of(u, L.level);
    const size_t n = (size_t)d.nx * d.ny * d.nz;
    const int np = wgrad_parts(n);
    wgrad_any(L.cin, L.cout, X, ldx, Z, d.nx, d.ny, d.nz, u->part, np, u->st);
    const int m = 27 * L.cin * L.cout;
    hipLaunchKernelGGL(k_part_sum, grid_for(m), dim3(256), 0, u->st, u->part, np, m, u->grad + L.woff, 0);
    bias_grad(u, l, Z, n);
    if (G)
        conv_any(L.cout, L.cin, add ? 2 : 1, Z, L.cout, wf_of(u, l), nullptr, G, ldg, d.nx, d.ny, d.nz, u->staged, u->st);
}

void mask(fx_unet *u, const float *G, int ldg, const bf16_t *Y, int ldy, bf16_t *Z, int C, size_t n) {
    hipLaunchKernelGGL(k_mask, grid_for(n * (C / 4)), dim3(256), 0, u->st, G, ldg, Y, ldy, Z, C, n);
}

// Loss against tg and the full gradient (into u->grad); the loss is left in dscal[0].
void enqueue_backward(fx_unet *u, const float *tg) {
    const Dims d1 = dims_of(u, 1), d2 = dims_of(u, 2);
    hipStream_t st = u->st;
    const UnetLayout &lay = layout();
    const size_t n0 = u->n0, n1 = u->n1, n2 = u->n2;
    const int nbl = 256;
    hipLaunchKernelGGL(k_loss, dim3(nbl), dim3(256), 0, st, u->out, tg, u->dout, u->dpart, n0);
    hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(64), 0, st, u->dpart, nbl, 1.0 / (double)n0, u->dscal);
    // head
    hipLaunchKernelGGL(k_head_bwd, dim3(nbl), dim3(256), 0, st, u->dout, u->a_d0b, u->theta + lay.head_off, u->z0,
                       u->part, n0);
    hipLaunchKernelGGL(k_part_sum, dim3(1), dim3(64), 0, st, u->part, nbl, 17, u->grad + lay.head_off, 0);
    // level 0, up
    layer_backward(u, D0B, u->a_d0a, 16, u->z0, u->g0_16, 16, 0);
    mask(u, u->g0_16, 16, u->a_d0a, 16, u->z0, 16, n0);
    layer_backward(u, D0A, u->cat0, 48, u->z0, u->g0_48, 48, 0);
    hipLaunchKernelGGL(k_up_bwd, grid_for(n1 * 8), dim3(256), 0, st, u->g0_48, 48, u->g1_32a, 32, d1.nx, d1.ny, d1.nz);
    // level 1, up
    mask(u, u->g1_32a, 32, u->a_d1b, 32, u->z1, 32, n1);
    layer_backward(u, D1B, u->a_d1a, 32, u->z1, u->g1_32b, 32, 0);
    mask(u, u->g1_32b, 32, u->a_d1a, 32, u->z1, 32, n1);
    layer_backward(u, D1A, u->cat1, 96, u->z1, u->g1_96, 96, 0);
    hipLaunchKernelGGL(k_up_bwd, grid_for(n2 * 16), dim3(256), 0, st, u->g1_96, 96, u->g2_64a, 64, d2.nx, d2.ny, d2.nz);
    // level 2
    mask(u, u->g2_64a, 64, u->a_b2b, 64, u->z2, 64, n2);
    layer_backward(u, B2B, u->a_b2a, 64, u->z2, u->g2_64b, 64, 0);
    mask(u, u->g2_64b, 64, u->a_b2a, 64, u->z2, 64, n2);
    layer_backward(u, B2A, u->p1, 32, u->z2, u->g2_32, 32, 0);
    hipLaunchKernelGGL(k_pool_bwd, grid_for(n2 * 8), dim3(256), 0, st, u->g2_32, u->g1_96 + 64, 96, 32, d2.nx, d2.ny,
                       d2.nz);
    // level 1, down (skip 1 gradient = channels 64..95 of g1_96)
    mask(u, u->g1_96 + 64, 96, u->cat1 + 64, 96, u->z1, 32, n1);
    layer_backward(u, E1B, u->a_e1a, 32, u->z1, u->g1_32b, 32, 0);
    mask(u, u->g1_32b, 32, u->a_e1a, 32, u->z1, 32, n1);
    layer_backward(u, E1A, u->p0, 16, u->z1, u->g1_16, 16, 0);
    hipLaunchKernelGGL(k_pool_bwd, grid_for(n1 * 4), dim3(256), 0, st, u->g1_16, u->g0_48 + 32, 48, 16, d1.nx, d1.ny,
                       d1.nz);
    // level 0, down (skip 0 gradient = channels 32..47 of g0_48)
    mask(u, u->g0_48 + 32, 48, u->cat0 + 32, 48, u->z0, 16, n0);
    layer_backward(u, E0B, u->a_e0a, 16, u->z0, u->g0_16, 16, 0);
    mask(u, u->g0_16, 16, u->a_e0a, 16, u->z0, 16, n0);
    layer_backward(u, E0A, u->in, kInC, u->z0, nullptr, 0, 0);
}

// phi_lin per device plane: the P = 0, carrier-free layered stack between the contacts.
void phi_lin_planes(const double *eps, int nz, double vb, double vt, double *out) {
    double Rtot = 0.0;
    for (int k = 0; k < nz; ++k) Rtot += 1.0 / eps[k];
    double R = 0.0;
    for (int k = 0; k < nz; ++k) {
        const double half = 0.5 / eps[k];
        out[k] = vb + (vt - vb) * (R + half) / Rtot;
        R += 2.0 * half;
    }
}

}  // namespace

namespace fx {

fx_status unet_upload_doping(fx_unet *u, const double *h_doping) {
    std::vector<float> d(u->nz);
    for (int k = 0; k < u->nz; ++k) d[k] = (float)(h_doping[k] / kDopingScale);
    UHIP(hipMemcpyAsync(u->dop, d.data(), u->nz * sizeof(float), hipMemcpyHostToDevice, u->st));
    UHIP(hipStreamSynchronize(u->st));
    return FX_OK;
}

fx_status unet_upload_lin(fx_unet *u, const double *eps, double vb, double vt) {
    std::vector<double> l(u->nz);
    phi_lin_planes(eps, u->nz, vb, vt, l.data());
    UHIP(hipMemcpyAsync(u->lin, l.data(), u->nz * sizeof(double), hipMemcpyHostToDevice, u->st));
    UHIP(hipStreamSynchronize(u->st));
    return FX_OK;
}

void unet_geometry(const fx_unet *u, int *nx, int *ny, int *nz, hipStream_t *st) {
    *nx = u->nx;
    *ny = u->ny;
    *nz = u->nz;
    *st = u->st;
}

void unet_pack_from_f64(fx_unet *u, const double *P_slab, double v_top) {
    hipLaunchKernelGGL(k_pack<double>, grid_for(u->n0), dim3(256), 0, u->st, P_slab, u->dop, (float)(v_top / kVScale),
                       u->in, u->in_xp, u->nx, u->nx * u->ny, u->n0);
}

void unet_forward_enqueue(fx_unet *u) { enqueue_forward(u); }

void unet_apply(fx_unet *u, double *phi_slab) {
    hipLaunchKernelGGL(k_apply, grid_for(u->n0), dim3(256), 0, u->st, u->out, u->lin, phi_slab, u->nx * u->ny, u->n0);
}

void unet_make_target(fx_unet *u, const double *phi_slab, float *tg) {
    hipLaunchKernelGGL(k_target, grid_for(u->n0), dim3(256), 0, u->st, phi_slab, u->lin, tg, u->nx * u->ny, u->n0);
}

}  // namespace fx

extern "C" {

size_t unet_num_params(void) { return layout().nparams; }

size_t unet_workspace_bytes(int nx, int ny, int nzd, int train) {
    fx::set_error("");
    if (!valid_dims(nx, ny, nzd)) {
        ufail(FX_EINVAL, "network slab %dx%dx%d: each size must be a multiple of 4 and >= 4", nx, ny, nzd);
        return 0;
    }
    fx_unet u{};
    u.nx = nx; u.ny = ny; u.nz = nzd; u.train = train ? 1 : 0;
    u.n0 = (size_t)nx * ny * nzd;
    u.n1 = u.n0 / 8;
    u.n2 = u.n1 / 8;
    return carve_unet(&u, nullptr);
}

fx_status unet_init(int nx, int ny, int nzd, int train, void *d_ws, size_t ws_bytes, void *stream, fx_unet **out) {
    fx::set_error("");
    if (!out) return ufail(FX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!valid_dims(nx, ny, nzd)) return ufail(FX_EINVAL, "network slab %dx%dx%d: each size must be a multiple of 4 and >= 4", nx, ny, nzd);
    if (!d_ws || ((uintptr_t)d_ws & 255) != 0) return ufail(FX_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    fx_unet *u = new (std::nothrow) fx_unet();
    if (!u) return ufail(FX_ENOMEM, "host allocation failed");
    u->nx = nx; u->ny = ny; u->nz = nzd; u->train = train ? 1 : 0;
    u->n0 = (size_t)nx * ny * nzd;
    u->n1 = u->n0 / 8;
    u->n2 = u->n1 / 8;
    u->st = (hipStream_t)stream;
    {   // FERROX_UNET_STAGED=0 keeps every convolution on the unstaged kernel (same results)
        const char *e = getenv("FERROX_UNET_STAGED");
        u->staged = !(e && *e == '0');
    }
    const size_t need = carve_unet(u, nullptr);
    if (ws_bytes < need) { delete u; return ufail(FX_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need); }
    carve_unet(u, d_ws);
    if (hipHostMalloc((void **)&u->h_scal, 4 * sizeof(double), 0) != hipSuccess) {
        delete u;
        return ufail(FX_EDEVICE, "hipHostMalloc failed");
    }
    // everything defined before first use: zero the whole workspace
    launch_zero(d_ws, (need - 256) & ~(size_t)3, u->st);
    u->adam_t = 0;
    if (hipStreamSynchronize(u->st) != hipSuccess) {
        (void)hipHostFree(u->h_scal);
        delete u;
        return ufail(FX_EDEVICE, "workspace clear failed");
    }
    *out = u;
    return FX_OK;
}

fx_status unet_set_params(fx_unet *u, const float *h_params) {
    fx::set_error("");
    if (!u || !h_params) return ufail(FX_EINVAL, "NULL argument");
    const size_t n = layout().nparams;
    UHIP(hipMemcpyAsync(u->theta, h_params, n * sizeof(float), hipMemcpyHostToDevice, u->st));
    if (u->train) {
        launch_zero(u->m, n * sizeof(float), u->st);
        launch_zero(u->v, n * sizeof(float), u->st);
    }
    u->adam_t = 0;
    prep_weights(u);
    UHIP(hipStreamSynchronize(u->st));
    return FX_OK;
}

fx_status unet_get_params(fx_unet *u, float *h_params) {
    fx::set_error("");
    if (!u || !h_params) return ufail(FX_EINVAL, "NULL argument");
    UHIP(hipMemcpyAsync(h_params, u->theta, layout().nparams * sizeof(float), hipMemcpyDeviceToHost, u->st));
    UHIP(hipStreamSynchronize(u->st));
    return FX_OK;
}

fx_status unet_pack_input(fx_unet *u, const float *d_P, const double *h_doping, double v_top) {
    fx::set_error("");
    if (!u || !d_P || !h_doping) return ufail(FX_EINVAL, "NULL argument");
    if (!std::isfinite(v_top)) return ufail(FX_EINVAL, "v_top must be finite");
    fx_status st = unet_upload_doping(u, h_doping);
    if (st) return st;
    hipLaunchKernelGGL(k_pack<float>, grid_for(u->n0), dim3(256), 0, u->st, d_P, u->dop, (float)(v_top / kVScale), u->in,
                       u->in_xp, u->nx, u->nx * u->ny, u->n0);
    return FX_OK;
}

fx_status unet_set_input(fx_unet *u, const float *h_in) {
    fx::set_error("");
    if (!u || !h_in) return ufail(FX_EINVAL, "NULL argument");
    // channels 3..15 of the API layout are zero; the device keeps 4 per voxel
    std::vector<float> c(u->n0 * kInC);
    for (size_t v = 0; v < u->n0; ++v) {
        const float *x = h_in + v * kInCApi;
        for (int k = 3; k < kInCApi; ++k)
            if (x[k] != 0.f) return ufail(FX_EINVAL, "input channel %d of voxel %zu is %g: channels 3..15 must be zero", k, v, (double)x[k]);
        for (int k = 0; k < kInC; ++k) c[v * kInC + k] = x[k];
    }
    const size_t n = u->n0 * kInC;
    float *tmp = (float *)u->cat0;      // n0*48 BF16 = n0*24 floats >= n0*4
    UHIP(hipMemcpyAsync(tmp, c.data(), n * sizeof(float), hipMemcpyHostToDevice, u->st));
    hipLaunchKernelGGL(k_f_to_bf, grid_for(n), dim3(256), 0, u->st, tmp, u->in, n);
    hipLaunchKernelGGL(k_pad_x, grid_for(u->n0), dim3(256), 0, u->st, u->in, u->in_xp, u->nx, u->n0);
    UHIP(hipStreamSynchronize(u->st));
    return FX_OK;
}

fx_status unet_get_input(fx_unet *u, float *h_in) {
    fx::set_error("");
    if (!u || !h_in) return ufail(FX_EINVAL, "NULL argument");
    const size_t n = u->n0 * kInC;
    std::vector<float> c(n);
    float *tmp = (float *)u->cat0;
    hipLaunchKernelGGL(k_bf_to_f, grid_for(n), dim3(256), 0, u->st, u->in, tmp, n);
    UHIP(hipMemcpyAsync(c.data(), tmp, n * sizeof(float), hipMemcpyDeviceToHost, u->st));
    UHIP(hipStreamSynchronize(u->st));
    for (size_t v = 0; v < u->n0; ++v)
        for (int k = 0; k < kInCApi; ++k) h_in[v * kInCApi + k] = k < kInC ? c[v * kInC + k] : 0.f;
    return FX_OK;
}

fx_status unet_forward(fx_unet *u, float *d_out) {
    fx::set_error("");
    if (!u) return ufail(FX_EINVAL, "network is NULL");
    enqueue_forward(u);
    if (d_out) UHIP(hipMemcpyAsync(d_out, u->out, u->n0 * sizeof(float), hipMemcpyDeviceToDevice, u->st));
    UHIP(hipGetLastError());
    return FX_OK;
}

fx_status unet_loss_grad(fx_unet *u, const float *d_target, double *h_loss, float *h_grad) {
    fx::set_error("");
    if (!u || !d_target) return ufail(FX_EINVAL, "NULL argument");
    if (!u->train) return ufail(FX_ESTATE, "network was created without training buffers");
    enqueue_forward(u);
    enqueue_backward(u, d_target);
    UHIP(hipMemcpyAsync(u->h_scal, u->dscal, sizeof(double), hipMemcpyDeviceToHost, u->st));
    if (h_grad) UHIP(hipMemcpyAsync(h_grad, u->grad, layout().nparams * sizeof(float), hipMemcpyDeviceToHost, u->st));
    UHIP(hipStreamSynchronize(u->st));
    if (h_loss) *h_loss = u->h_scal[0];
    return FX_OK;
}

fx_status unet_train_step(fx_unet *u, const float *d_target, float lr, double *h_loss) {
    fx::set_error("");
    if (!u || !d_target) return ufail(FX_EINVAL, "NULL argument");
    if (!u->train) return ufail(FX_ESTATE, "network was created without training buffers");
    if (!(lr > 0)) return ufail(FX_EINVAL, "lr must be > 0");
    enqueue_forward(u);
    enqueue_backward(u, d_target);
    u->adam_t += 1;
    const float c1 = 1.0f - powf(0.9f, (float)u->adam_t), c2 = 1.0f - powf(0.999f, (float)u->adam_t);
    const size_t n = layout().nparams;
    hipLaunchKernelGGL(k_adam, grid_for(n), dim3(256), 0, u->st, u->theta, u->grad, u->m, u->v, n, lr, c1, c2);
    prep_weights(u);
    if (h_loss) {
        UHIP(hipMemcpyAsync(u->h_scal, u->dscal, sizeof(double), hipMemcpyDeviceToHost, u->st));
        UHIP(hipStreamSynchronize(u->st));
        *h_loss = u->h_scal[0];
    }
    UHIP(hipGetLastError());
    return FX_OK;
}

fx_status unet_destroy(fx_unet *u) {
    if (!u) return FX_OK;
    if (u->st) (void)hipStreamSynchronize(u->st); else (void)hipDeviceSynchronize();
    if (u->h_scal) (void)hipHostFree(u->h_scal);
    delete u;
    return FX_OK;
}

}  // extern "C"
