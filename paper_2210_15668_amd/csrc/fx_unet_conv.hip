// Forward 3x3x3 convolutions of the learned warm start's network on gfx950's
// v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation), z-marching.
//
// Lane layout of that instruction (wave64, checked on the device): lane l
// holds A[l%16][8(l/16)+e], B[8(l/16)+e][l%16] and D[4(l/16)+r][l%16],
// e = 0..7, r = 0..3.  A = 16 output channels x 32 K-values of the weights,
// B = the same 32 K-values of 16 consecutive x-voxels, so each lane reads
// 16 bytes of input (8 channels of one voxel) per fragment.
//
// A wave owns 16 consecutive x-voxels of RY rows and 16 output channels and
// walks the input planes z' of its block once, bottom to top.  One input
// fragment (the 16 voxels of a row of plane z', some channels, shifted by dx)
// is a K-slice of the taps (dx, dy, dz) of 9 output tiles at once: rows
// y' - dy for dy = -1..1 and planes z' - dz for dz = -1..1; the wave issues
// those MFMAs with 9 weight fragments that stay in registers for the whole
// launch.  Output plane z' - 1 is complete after plane z' and is stored
// (bias, ReLU, BF16); three rolling accumulator sets hold the planes in
// flight.  The block (4 waves) stages each input plane once in LDS (double
// buffered, the next plane's loads in flight during the MFMAs) with a one-voxel
// halo in x and y (periodic wrap) and zeros beyond the z-ends.
//
// K-slices: a 32-channel chunk gives three fragments per row (dx = -1, 0, 1),
// every lane group (l/16) one 8-channel group.  A 16-channel chunk pairs two
// voxels in one fragment: F0 = (x-1, x) x 16 channels covers dx = -1 and 0;
// F1 = (x+1 at rows y', y'+1) covers dx = +1 with weights of rows dy and dy+1,
// used at dy = -1 (rows -1, 0) and dy = +1 (row +1; the other half's weights
// zero): 15 MFMAs per output tile instead of 13.5 at full packing.  The first
// layer's 3 input channels (plus a zero) are packed 4 to a voxel and two voxels
// (two in-plane taps) to a lane: 8 in-plane taps in one fragment, the ninth
// in a second, 6 MFMAs per output tile.
//
// Input channels come from up to two tensors: A (optionally read at
// (x/2, y/2, z/2) of the next coarser level: the nearest-neighbour upsampling
// of the decoder folded into the staging) and B (the skip connection); their
// concatenation is never written out.
#include "fx_internal.h"
#include "fx_unet_internal.h"

#include <type_traits>

namespace fx {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

// round to nearest even (NaN stays NaN)
__device__ __forceinline__ bf16_t f2bf_z(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
    return (bf16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bf8 as_bf8(i4 v) { return __builtin_bit_cast(bf8, v); }

// ---------------------------------------------------------------- K plan
// Channel chunks in channel order: source A then source B, each split into
// 32-channel chunks and at most one 16-channel chunk.
__host__ __device__ constexpr int zchunks(int ca, int cb) {
    return ca == 4 ? 1 : ca / 32 + (ca % 32) / 16 + cb / 32 + (cb % 32) / 16;
}
__host__ __device__ constexpr int zchunk_w(int ca, int cb, int c) {
    if (ca == 4) return 4;
    const int n32a = ca / 32, n16a = (ca % 32) / 16, n32b = cb / 32;
    if (c < n32a) return 32;
    c -= n32a;
    if (c < n16a) return 16;
    c -= n16a;
    if (c < n32b) return 32;
    return 16;
}
__host__ __device__ constexpr int zfrags_of(int w) { return w == 32 ? 27 : (w == 16 ? 15 : 6); }
__host__ __device__ constexpr int zchunk_c0(int ca, int cb, int c) {
    int s = 0;
    for (int i = 0; i < c; ++i) s += zchunk_w(ca, cb, i);
    return s;
}
__host__ __device__ constexpr int zchunk_f0(int ca, int cb, int c) {
    int s = 0;
    for (int i = 0; i < c; ++i) s += zfrags_of(zchunk_w(ca, cb, i));
    return s;
}
__host__ __device__ constexpr int znfrags(int ca, int cb) { return zchunk_f0(ca, cb, zchunks(ca, cb)); }

// The weight behind K-value (kq, e) of fragment f (input-channel index ci and
// tap, tap = (dz+1)*9 + (dy+1)*3 + (dx+1)); false where the slot carries no weight.
__host__ __device__ bool zfrag_entry(int ca, int cb, int f, int kq, int e, int *tap, int *ci) {
    int c = 0;
    while (c + 1 < zchunks(ca, cb) && f >= zchunk_f0(ca, cb, c + 1)) ++c;
    const int w = zchunk_w(ca, cb, c), c0 = zchunk_c0(ca, cb, c), j = f - zchunk_f0(ca, cb, c);
    int dx, dy, dz, ch;
    if (w == 32) {
        dx = j / 9 - 1;
        dy = (j / 3) % 3 - 1;
        dz = j % 3 - 1;
        ch = c0 + 8 * kq + e;
    } else if (w == 16) {
        ch = c0 + 8 * (kq & 1) + e;
        if (j < 9) {                         // F0: (x-1 | x) at row y'
            dx = kq < 2 ? -1 : 0;
            dy = j / 3 - 1;
            dz = j % 3 - 1;
        } else {                             // F1: x+1 at rows y' | y'+1
            const int jj = j - 9;
            const int dyb = jj < 3 ? -1 : 1;
            dx = 1;
            dy = dyb + (kq >> 1);
            dz = jj % 3 - 1;
            if (dy > 1) return false;
        }
    } else {                                 // packed: 4 channels, two in-plane taps per lane group
        const int fb = j >= 3;
        dz = (fb ? j - 3 : j) - 1;
        int t;
        if (!fb) t = 2 * kq + (e >> 2);
        else {
            if (kq != 0 || e >= 4) return false;
            t = 8;
        }
        ch = e & 3;
        if (ch >= 3) return false;
        dx = t % 3 - 1;
        dy = t / 3 - 1;
    }
    *tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
    *ci = ch;
    return true;
}

// wz[m][f][lane][e] = BF16 weight (zero where the slot carries none); theta holds
// W[tap][cout][cin] of the layer (cin as in the parameter vector).
__global__ void k_prepz(const float *__restrict__ th, int cin, int cout, int ca, int cb, int ci_off, int nf,
                        bf16_t *__restrict__ wz) {
    const int total = (cout / 16) * nf * 64 * 8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int e = i & 7, lane = (i >> 3) & 63, q = i >> 9, f = q % nf, m = q / nf;
        const int co = 16 * m + (lane & 15), kq = lane >> 4;
        int tap, ci;
        float v = 0.f;
        if (zfrag_entry(ca, cb, f, kq, e, &tap, &ci)) v = th[((size_t)tap * cout + co) * cin + ci_off + ci];
        wz[i] = f2bf_z(v);
    }
}

// ------------------------------------------------------------- the kernel
// A block is 5 waves.  Waves 0..3 compute: MS of them split the output channels
// (16 each), KS split the channel chunks (wave part kp takes chunks c with
// c % KS == kp; their partial sums meet in LDS), and WX x WY spatial tiles of
// 16 x RY voxels.  Wave 4 stages the input planes: it issues only global->LDS
// transfers, two planes ahead, into a ring of three plane buffers, and waits for
// exactly the plane the next step needs (the compute waves issue the output
// stores, which would otherwise make every wait for a load a wait for all).
template <int CA, bool UPA, int CB, int MS, int KS, int RY, int WX>
struct ZCfg {
    static constexpr bool PK = CA == 4;
    static constexpr int CIN = CA + CB;
    static constexpr int WY = 4 / (MS * KS * WX);
    static constexpr int BX = 16 * WX, BY = RY * WY, R = BY + 3, XC = BX + 2;
    static constexpr int G = PK ? 1 : CIN / 8;          // 16-byte groups per voxel (packed: one 8-byte voxel)
    static constexpr int GA = PK ? 1 : CA / 8;          // of them from source A
    static constexpr int PLANE = R * XC * (PK ? 8 : G * 16);   // bytes of one staged plane
    // transfers of 16 bytes per lane, one wave instruction moving 64 consecutive units:
    // [row][group][column] order, packed [row][voxel pair] (the packed input has its
    // rows padded by one wrapped voxel at each x-end, so a staged row is contiguous)
    static constexpr int DU = 16;
    static constexpr int UNITS = PLANE / DU;
    static constexpr int NI = (UNITS + 63) / 64;        // transfer instructions per plane
    static constexpr int PSTRIDE = NI * 64 * DU;        // a staged plane padded to whole instructions
    static constexpr int NCH = zchunks(CA, CB);
    static constexpr int TILES = WX * WY * MS;          // output tiles (16 channels x 16 x RY voxels) per block
    static constexpr int RED = KS > 1 ? 2 * TILES * RY * 64 * 16 : 0;   // partial sums, two buffers
    static constexpr int LDS = 3 * PSTRIDE + RED;
    static_assert(MS * KS * WX * WY == 4, "4 compute waves per block");
    static_assert(KS == 1 || !PK, "the packed layer is not split");
    static_assert(!PK || XC % 2 == 0, "packed rows are whole voxel pairs");
    static_assert(RY % 2 == 0, "pooling pairs the rows of a wave");
    static_assert(NI <= 31, "two planes of transfers in flight must fit the load counter");
    // weight fragments of wave part kp, and the local index of chunk c's first one
    static constexpr int nfk(int kp) {
        int n = 0;
        for (int c = 0; c < NCH; ++c)
            if (c % KS == kp) n += zfrags_of(zchunk_w(CA, CB, c));
        return n;
    }
    static constexpr int lf0(int c) {
        int n = 0;
        for (int i = 0; i < c; ++i)
            if (i % KS == c % KS) n += zfrags_of(zchunk_w(CA, CB, i));
        return n;
    }
    // fragments per row read by wave part kp
    static constexpr int nrow(int kp) {
        int n = 0;
        for (int c = 0; c < NCH; ++c)
            if (c % KS == kp) n += PK ? 2 : (zchunk_w(CA, CB, c) == 32 ? 3 : 2);
        return n;
    }
};

// Block barrier for the hand-over of LDS data: each wave waits for its own LDS
// accesses, not for its global loads and stores in flight (__syncthreads() would
// wait for those too).  No global data passes between the waves of a block.  The
// memory clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Cross-lane sums of the epilogues without the LDS unit.  v + v(lane ^ 1) with a DPP quad
// permutation; v + v(lane ^ 16) and v + v(lane ^ 32) with gfx950's half-row swaps: swapping
// a register with itself leaves in every lane the pair (v(lane), v(lane ^ d)) in some order,
// and their sum is the same value either way.
__device__ __forceinline__ float lane_add_xor1(float v) {
#if defined(__HIP_DEVICE_COMPILE__)
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF,
                                                                       false));
#else
    return v;
#endif
}
__device__ __forceinline__ float lane_sum16(float v) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int x = __builtin_bit_cast(int, v);
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return __builtin_bit_cast(float, (int)p[0]) + __builtin_bit_cast(float, (int)p[1]);
#else
    return v;
#endif
}
__device__ __forceinline__ float lane_sum32(float v) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int x = __builtin_bit_cast(int, v);
    const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return __builtin_bit_cast(float, (int)p[0]) + __builtin_bit_cast(float, (int)p[1]);
#else
    return v;
#endif
}

// One global->LDS transfer of BYTES per lane: lane l's bytes land at dst + l * BYTES
// (dst is the same for the whole wave).  The 16-byte form exists on gfx950 only, so
// the call is left out of the host pass, which never runs a kernel body.
template <int BYTES>
__device__ __forceinline__ void global_to_lds(const void *src, void *dst) {
#if defined(__HIP_DEVICE_COMPILE__)
    static_assert(BYTES == 16 || BYTES == 4, "transfer size");
    if constexpr (BYTES == 16)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    else
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)dst, 4, 0, 0);
#else
    (void)src;
    (void)dst;
#endif
}

// s_waitcnt vmcnt(N) (gfx9 encoding; expcnt and lgkmcnt not waited for)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int I, int N, class F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor<I + 1, N>(f);
    }
}

// Which of the three planes a step feeds: bit dzi for dz = dzi - 1.  The first
// step of a block (input plane zb0 - 1) feeds only its upper neighbour, the last
// (zb0 + nq) only its lower one; a middle step feeds all three, also where that
// plane lies outside the block (a slot that is cleared before its next use).
constexpr int kDzAll = 7, kDzLow = 1, kDzHigh = 4;

// MFMAs of input row r of the current plane with fragment b into the output
// tiles it feeds: row ro = r - 1 - dy of the weight fragments' dy, the planes of
// the step's dz, accumulator slot (P - dz) mod 3.
template <int RY, int NF, int P, int MASK, int R, int DY>
__device__ __forceinline__ void zmac(f4 (&acc)[3][RY], const i4 (&af)[NF], int fbase, bf8 b) {
    constexpr int ro = R - 1 - DY;
    if constexpr (ro >= 0 && ro < RY) {
        sfor<0, 3>([&](auto di) {
            constexpr int dzi = decltype(di)::value;
            if constexpr ((MASK >> dzi) & 1) {
                constexpr int sl = (P - (dzi - 1) + 3) % 3;
                acc[sl][ro] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(af[fbase + dzi]), b, acc[sl][ro], 0, 0, 0);
            }
        });
    }
}

// The steps p = 0 .. nsteps-1 of a block, phase P = p mod 3 and the plane mask as
// compile-time arguments of fn(phase, mask, p); both roles walk the same sequence
// (and so pass the same barriers).
template <class F>
__device__ __forceinline__ void zsteps(int nsteps, F &&fn) {
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using MAll = std::integral_constant<int, kDzAll>;
    using MLow = std::integral_constant<int, kDzLow>;
    using MHigh = std::integral_constant<int, kDzHigh>;
    fn(I0{}, MLow{}, 0);
    int p = 1;
    for (; p + 3 <= nsteps - 1; p += 3) {
        fn(I1{}, MAll{}, p);
        fn(I2{}, MAll{}, p + 1);
        fn(I0{}, MAll{}, p + 2);
    }
    if (p < nsteps - 1) fn(I1{}, MAll{}, p++);
    if (p < nsteps - 1) fn(I2{}, MAll{}, p++);
    switch (p % 3) {
    case 0: fn(I0{}, MHigh{}, p); break;
    case 1: fn(I1{}, MHigh{}, p); break;
    default: fn(I2{}, MHigh{}, p); break;
    }
}

// OUT 0: Y (BF16) = relu(conv + bias); OUT 1: Pf (FP32, ld cout) = conv;
// OUT 2: Y (BF16) = relu(conv + Pf + bias) with Pf an OUT 1 result (FP32, ld cout);
// OUT 3: the network's 1x1x1 head on Y as OUT 0 would store it: Pf[v] = hw[16] +
//        sum over c of hw[c] Y[v][c] (FP32; Y itself is not stored);
// OUT 4: Y as OUT 0, and Yp (BF16, ld cout) = its 2x2x2 average on the coarser level.
template <int CA, bool UPA, int CB, int MS, int KS, int RY, int WX, int OUT>
__global__ __launch_bounds__(320) void k_convz(const bf16_t *__restrict__ XA, int lda, const bf16_t *__restrict__ XB,
                                               int ldb, const bf16_t *__restrict__ wz, const float *__restrict__ bias,
                                               bf16_t *__restrict__ Y, int ldy, float *__restrict__ Pf,
                                               const float *__restrict__ hw, bf16_t *__restrict__ Yp, int nx, int ny,
                                               int nz, int zb, int ntx, int nty, int ntiles) {
    using C = ZCfg<CA, UPA, CB, MS, KS, RY, WX>;
    constexpr int G = C::G, XC = C::XC, NI = C::NI, NF = znfrags(CA, CB);
    __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS];

    // the wave index is the same on all lanes: keep it (and all derived from it) scalar
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // each of the 8 XCDs walks one contiguous range of tiles (x fastest, then y, then
    // z), so the halo rows that neighbouring tiles share are read into the same L2
    const int nb = gridDim.x, g = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    if (g >= ntiles) return;
    const int tx = g % ntx, t1 = g / ntx, ty = t1 % nty, tz = t1 / nty;
    const int x0 = tx * C::BX, y0 = ty * C::BY, zb0 = tz * zb;
    const int nq = min(zb, nz - zb0);                 // output planes of this block
    const int nsteps = nq + 2;                        // input planes zb0-1 .. zb0+nq

    if (wave == 4) {
        // ---------------------------------------------------------- staging wave
        // unit u = 64 k + lane of a plane: its source offset (in elements, without the
        // plane) and source; units past the plane read unit 0's voxel into the padding
        int gofs[NI];
        unsigned srcb = 0;
        const int nxc = UPA ? nx >> 1 : (C::PK ? nx + 2 : nx), nyc = UPA ? ny >> 1 : ny;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int u = 64 * k + lane, uu = u < C::UNITS ? u : 0;
            int xc, r, g, e0;                          // e0: first element of the unit in its voxel
            if constexpr (C::PK) {
                // voxel pair j of row r: padded x = x0 + 2j (staged column 2j is x0 - 1 + 2j);
                // pairs past the padded row (outputs there are not stored) read its last pair
                const int j = uu % (XC / 2);
                r = uu / (XC / 2);
                int yy = (y0 - 1 + r) % ny;
                yy += yy < 0 ? ny : 0;
                gofs[k] = (yy * (nx + 2) + min(x0 + 2 * j, nx)) * lda;
                continue;
            } else {
                xc = uu % XC;
                const int t = uu / XC;
                g = t % G;
                r = t / G;
                e0 = 8 * (g < C::GA ? g : g - C::GA);
            }
            int xx = (x0 - 1 + xc) % nx, yy = (y0 - 1 + r) % ny;
            xx += xx < 0 ? nx : 0;
            yy += yy < 0 ? ny : 0;
            if (g < C::GA) {
                gofs[k] = (UPA ? ((yy >> 1) * nxc + (xx >> 1)) : (yy * nx + xx)) * lda + e0;
            } else {
                gofs[k] = (yy * nx + xx) * ldb + e0;
                srcb |= 1u << k;
            }
        }
        const size_t planeA = (size_t)nxc * nyc * lda, planeB = (size_t)nx * ny * ldb;
        (void)planeB;
        // plane p (input plane zb0 - 1 + p) into buffer BUF: transfers, or zeros
        // beyond the z-ends; true when transfers were issued
        auto stage = [&](int p, auto bufc) -> bool {
            constexpr int BUF = decltype(bufc)::value;
            unsigned char *base = lds + BUF * C::PSTRIDE;
            const int zz = zb0 - 1 + p;
            if (zz >= 0 && zz < nz) {
                const bf16_t *pa = XA + (size_t)(UPA ? zz >> 1 : zz) * planeA;
                const bf16_t *pb = XB + (size_t)zz * planeB;
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    const bf16_t *src = (CB > 0 && ((srcb >> k) & 1u)) ? pb + gofs[k] : pa + gofs[k];
                    global_to_lds<C::DU>(src, base + k * 64 * C::DU);
                }
                return true;
            }
            const i4 z = {0, 0, 0, 0};
            for (int u = lane; u < C::PSTRIDE / 16; u += 64) *(i4 *)(base + 16 * u) = z;
            return false;
        };
        // the step needs plane p; plane p + 1 was issued before plane p + 2
        bool staged0 = stage(0, std::integral_constant<int, 0>{});
        bool staged1 = nsteps > 1 ? stage(1, std::integral_constant<int, 1>{}) : false;
        (void)staged0;
        if (staged1) wait_vmcnt<NI>();
        else wait_vmcnt<0>();
        lds_barrier();
        zsteps(nsteps, [&](auto phase, auto, int p) {
            constexpr int P = decltype(phase)::value;
            // plane p + 2 goes into the buffer of plane p - 1, which every wave left at
            // the last barrier; then wait for plane p + 1 only
            bool issued = false;
            if (p + 2 < nsteps) issued = stage(p + 2, std::integral_constant<int, (P + 2) % 3>{});
            if (issued) wait_vmcnt<NI>();
            else wait_vmcnt<0>();
            lds_barrier();
        });
        return;
    }

    // ---------------------------------------------------------- compute waves
    const int col = lane & 15, kq = lane >> 4;
    const int m = wave % MS, kp = (wave / MS) % KS, s = wave / (MS * KS), wx = s % WX, wy = s / WX;

    // this lane's byte offset in a staged plane (row 0 of the wave, its voxel col)
    const int lbase = C::PK ? ((RY * wy) * XC + 16 * wx + col) * 8 : (((RY * wy) * G) * XC + 16 * wx + col) * 16;
    // per-lane parts of the fragment addresses: packed Fa = taps 2kq, 2kq+1, Fb = tap 8
    // on lane group 0 and the centre (zero weights) elsewhere; 16-channel F0 / F1
    int pk_off[2][2] = {{0, 0}, {0, 0}};
    if constexpr (C::PK) {
        for (int h = 0; h < 2; ++h) {
            const int ta = 2 * kq + h, tb = kq == 0 ? 8 : 4;
            pk_off[0][h] = ((ta / 3) * XC + ta % 3) * 8;
            pk_off[1][h] = ((tb / 3) * XC + tb % 3) * 8;
        }
    }
    const int off32 = kq * XC * 16;
    const int off16a = ((kq & 1) * XC + (kq >> 1)) * 16;
    const int off16b = (((kq >> 1) * G + (kq & 1)) * XC + 2) * 16;

    const int out_c0 = 16 * m + 4 * kq;
    float bv[4] = {0.f, 0.f, 0.f, 0.f}, hv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (OUT != 1)
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = bias[out_c0 + i];
    if constexpr (OUT == 3) {
        static_assert(MS == 1 && KS == 1, "the head follows one 16-channel tile");
#pragma unroll
        for (int i = 0; i < 4; ++i) hv[i] = hw[out_c0 + i];
        hv[4] = hw[16];
    }
    const int gx = x0 + 16 * wx + col;
    const int gy0 = y0 + RY * wy;
    const unsigned y_off = (unsigned)(col * ldy + out_c0), pf_off = (unsigned)(col * 16 * MS + out_c0);
    // partial sums of this wave's tile: [buffer][tile][row][lane] (16 bytes)
    f4 *red = (f4 *)(lds + 3 * C::PSTRIDE) + ((s * MS + m) * RY) * 64 + lane;

    // rows of the plane: packed 1..RY (dy inside the fragment), else 0..RY+1
    constexpr int RLO = C::PK ? 1 : 0, RHI = C::PK ? RY + 1 : RY + 2;

    // The whole z-march of wave part KP (its chunks, its weight fragments).
    auto body = [&](auto kpc) {
        constexpr int KP = decltype(kpc)::value;
        constexpr int NFK = C::nfk(KP), NR = C::nrow(KP);
        // weight fragments of this wave's 16 output channels and chunks, resident for
        // the launch (the empty asm keeps the compiler from reloading them in the loop)
        i4 af[NFK];
        {
            const i4 *src = (const i4 *)(wz + (size_t)m * NF * 512) + lane;
            sfor<0, C::NCH>([&](auto ci) {
                constexpr int c = decltype(ci)::value;
                if constexpr (c % KS == KP) {
                    constexpr int f0 = zchunk_f0(CA, CB, c), l0 = C::lf0(c), n = zfrags_of(zchunk_w(CA, CB, c));
#pragma unroll
                    for (int f = 0; f < n; ++f) af[l0 + f] = src[(f0 + f) * 64];
                }
            });
#pragma unroll
            for (int f = 0; f < NFK; ++f) asm volatile("" : "+v"(af[f]));
#pragma unroll
            for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(bv[i]));
            if constexpr (OUT == 3)
#pragma unroll
                for (int i = 0; i < 5; ++i) asm volatile("" : "+v"(hv[i]));
        }
        f4 acc[3][RY];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int r = 0; r < RY; ++r) acc[a][r] = f4{0.f, 0.f, 0.f, 0.f};
        // pooling (OUT 4): the row pair in progress and the pooled rows of an even plane
        f4 prow = {0.f, 0.f, 0.f, 0.f}, pacc[(RY + 1) / 2];
#pragma unroll
        for (int r = 0; r < (RY + 1) / 2; ++r) pacc[r] = f4{0.f, 0.f, 0.f, 0.f};
        (void)prow;
        (void)pacc;

        // the NR fragments of row r of a staged plane
        auto read_row = [&](const unsigned char *cur, auto rr, bf8 (&fr)[NR]) {
            constexpr int r = decltype(rr)::value;
            if constexpr (C::PK) {
                const unsigned char *q0 = cur + (r - 1) * XC * 8;
                sfor<0, 2>([&](auto fbi) {
                    constexpr int fb = decltype(fbi)::value;
                    const i2 lo = *(const i2 *)(q0 + pk_off[fb][0]);
                    const i2 hi = *(const i2 *)(q0 + pk_off[fb][1]);
                    fr[fb] = as_bf8(i4{lo[0], lo[1], hi[0], hi[1]});
                });
            } else {
                const unsigned char *rowp = cur + r * G * XC * 16;
                int k = 0;
                sfor<0, C::NCH>([&](auto ci) {
                    constexpr int c = decltype(ci)::value;
                    constexpr int w = zchunk_w(CA, CB, c), g0 = zchunk_c0(CA, CB, c) / 8;
                    if constexpr (c % KS == KP) {
                        if constexpr (w == 32) {
                            sfor<0, 3>([&](auto dd) {
                                constexpr int dxi = decltype(dd)::value;
                                fr[k++] = as_bf8(*(const i4 *)(rowp + off32 + (g0 * XC + dxi) * 16));
                            });
                        } else {
                            fr[k++] = as_bf8(*(const i4 *)(rowp + off16a + g0 * XC * 16));
                            fr[k++] = as_bf8(*(const i4 *)(rowp + off16b + g0 * XC * 16));
                        }
                    }
                });
            }
        };
        // the MFMAs of row r
        auto mac_row = [&](auto phase, auto mask, auto rr, const bf8 (&fr)[NR]) {
            constexpr int P = decltype(phase)::value, MASK = decltype(mask)::value, r = decltype(rr)::value;
            if constexpr (C::PK) {
                zmac<RY, NFK, P, MASK, r, 0>(acc, af, 0, fr[0]);
                zmac<RY, NFK, P, MASK, r, 0>(acc, af, 3, fr[1]);
            } else {
                int k = 0;
                sfor<0, C::NCH>([&](auto ci) {
                    constexpr int c = decltype(ci)::value;
                    constexpr int w = zchunk_w(CA, CB, c), f0 = C::lf0(c);
                    if constexpr (c % KS == KP) {
                        if constexpr (w == 32) {
                            sfor<0, 3>([&](auto dd) {
                                constexpr int dxi = decltype(dd)::value;
                                zmac<RY, NFK, P, MASK, r, -1>(acc, af, f0 + dxi * 9 + 0, fr[k]);
                                zmac<RY, NFK, P, MASK, r, 0>(acc, af, f0 + dxi * 9 + 3, fr[k]);
                                zmac<RY, NFK, P, MASK, r, 1>(acc, af, f0 + dxi * 9 + 6, fr[k]);
                                ++k;
                            });
                        } else {
                            zmac<RY, NFK, P, MASK, r, -1>(acc, af, f0 + 0, fr[k]);
                            zmac<RY, NFK, P, MASK, r, 0>(acc, af, f0 + 3, fr[k]);
                            zmac<RY, NFK, P, MASK, r, 1>(acc, af, f0 + 6, fr[k]);
                            zmac<RY, NFK, P, MASK, r, -1>(acc, af, f0 + 9, fr[k + 1]);
                            zmac<RY, NFK, P, MASK, r, 1>(acc, af, f0 + 12, fr[k + 1]);
                            k += 2;
                        }
                    }
                });
            }
        };
        // output plane q (0-based gz = zb0 + q - 1) from accumulator slot SO (plus the
        // other wave part's partial sums in buffer rb when the chunks are split)
        auto finish = [&](auto slot, int q, int rb) {
            constexpr int SO = decltype(slot)::value;
            if (q >= 1 && q <= nq) {
                const int gz = zb0 + q - 1;
                f4 pin[RY];                            // the partial sums of an earlier launch, all
                if constexpr (OUT == 2) {              // read before the first store
#pragma unroll
                    for (int ro = 0; ro < RY; ++ro) {
                        const int gy = min(gy0 + ro, ny - 1);
                        const size_t v0 = (size_t)(gz * ny + gy) * nx + x0 + 16 * wx;
                        pin[ro] = gx < nx ? *(const f4 *)(Pf + v0 * (16 * MS) + pf_off) : f4{0.f, 0.f, 0.f, 0.f};
                    }
                }
#pragma unroll
                for (int ro = 0; ro < RY; ++ro) {
                    f4 a = acc[SO][ro];
                    if constexpr (KS > 1) a = a + red[(rb * C::TILES * RY + ro) * 64];
                    if constexpr (OUT == 2) a = a + pin[ro];
                    const int gy = gy0 + ro;
                    if (gy < ny) {
                        // the row's first voxel of this wave (uniform) plus a per-lane
                        // offset that stays in one register for every row
                        const size_t v0 = (size_t)(gz * ny + gy) * nx + x0 + 16 * wx;
                        if constexpr (OUT == 1) {
                            if (gx < nx) *(f4 *)(Pf + v0 * (16 * MS) + pf_off) = a;
                        } else {
                            const f2 lo = {fmaxf(a[0] + bv[0], 0.f), fmaxf(a[1] + bv[1], 0.f)};
                            const f2 hi = {fmaxf(a[2] + bv[2], 0.f), fmaxf(a[3] + bv[3], 0.f)};
                            const bf2 blo = __builtin_convertvector(lo, bf2), bhi = __builtin_convertvector(hi, bf2);
                            const i2 o = {__builtin_bit_cast(int, blo), __builtin_bit_cast(int, bhi)};
                            if constexpr (OUT != 3) {
                                if (gx < nx) *(i2 *)(Y + v0 * ldy + y_off) = o;
                            }
                            if constexpr (OUT == 3 || OUT == 4) {
                                // the stored (rounded) values, widened from the rounded pairs
                                // themselves (taken back out of the packed vector o, the high
                                // pair was compiled as a copy of the low one)
                                const f2 rl = __builtin_convertvector(blo, f2);
                                const f2 rh = __builtin_convertvector(bhi, f2);
                                if constexpr (OUT == 3) {
                                    // head: this lane's 4 channels, then the 4 lane groups of the voxel
                                    float h = hv[0] * rl[0];
                                    h = fmaf(hv[1], rl[1], h);
                                    h = fmaf(hv[2], rh[0], h);
                                    h = fmaf(hv[3], rh[1], h);
                                    h = lane_sum16(h);
                                    h = lane_sum32(h);
                                    if (kq == 0 && gx < nx) Pf[v0 + col] = h + hv[4];
                                } else {
                                    // average pooling: x pairs (lanes col, col ^ 1), then the
                                    // row pair (ro, ro + 1), then the plane pair (gz, gz + 1)
                                    f4 t = {rl[0], rl[1], rh[0], rh[1]};
#pragma unroll
                                    for (int i = 0; i < 4; ++i) t[i] = lane_add_xor1(t[i]);
                                    if ((ro & 1) == 0) {
                                        prow = t;
                                    } else {
                                        t = prow + t;
                                        if ((gz & 1) == 0) {
                                            pacc[ro >> 1] = t;
                                        } else {
                                            t = (pacc[ro >> 1] + t) * 0.125f;
                                            if ((col & 1) == 0 && gx < nx) {
                                                const f2 a0 = {t[0], t[1]}, a1 = {t[2], t[3]};
                                                const i2 po = {__builtin_bit_cast(int, __builtin_convertvector(a0, bf2)),
                                                               __builtin_bit_cast(int, __builtin_convertvector(a1, bf2))};
                                                const size_t pv = ((size_t)(gz >> 1) * (ny >> 1) + (gy >> 1)) * (nx >> 1) +
                                                                  (gx >> 1);
                                                *(i2 *)(Yp + pv * (16 * MS) + out_c0) = po;
                                            }
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int ro = 0; ro < RY; ++ro) acc[SO][ro] = f4{0.f, 0.f, 0.f, 0.f};
        };

        lds_barrier();                                 // plane 0 staged
        // one input plane (buffer p mod 3): its fragments and MFMAs, then the completed
        // output plane q = p - 1.  With split chunks part 1 leaves its partial sums of q
        // in LDS and part 0 finishes q at the start of the next step, after the barrier.
        zsteps(nsteps, [&](auto phase, auto mask, int p) {
            constexpr int P = decltype(phase)::value;
            using SDone = std::integral_constant<int, (P + 2) % 3>;     // slot of q = p - 1
            using SPrev = std::integral_constant<int, (P + 1) % 3>;     // slot of q = p - 2
            if constexpr (KS > 1 && KP == 0) finish(SPrev{}, p - 2, (p - 1) & 1);
            const unsigned char *cur = lds + P * C::PSTRIDE + lbase;
            if constexpr (NR * (RHI - RLO) <= 12) {     // every fragment of the plane at once
                bf8 fr[RHI - RLO][NR];
                sfor<RLO, RHI>([&](auto rr) { read_row(cur, rr, fr[decltype(rr)::value - RLO]); });
                sfor<RLO, RHI>([&](auto rr) { mac_row(phase, mask, rr, fr[decltype(rr)::value - RLO]); });
            } else {                                     // row by row, one row read ahead
                bf8 fa[NR], fb[NR];
                read_row(cur, std::integral_constant<int, RLO>{}, fa);
                sfor<RLO, RHI>([&](auto rr) {
                    constexpr int r = decltype(rr)::value;
                    constexpr bool even = ((r - RLO) & 1) == 0;
                    if constexpr (r + 1 < RHI) read_row(cur, std::integral_constant<int, r + 1>{}, even ? fb : fa);
                    mac_row(phase, mask, rr, even ? fa : fb);
                });
            }
            if constexpr (KS == 1) {
                finish(SDone{}, p - 1, 0);
            } else if constexpr (KP == 1) {
                const int q = p - 1;
                if (q >= 1 && q <= nq)
#pragma unroll
                    for (int ro = 0; ro < RY; ++ro) red[((p & 1) * C::TILES * RY + ro) * 64] = acc[SDone::value][ro];
#pragma unroll
                for (int ro = 0; ro < RY; ++ro) acc[SDone::value][ro] = f4{0.f, 0.f, 0.f, 0.f};
            }
            lds_barrier();
        });
        // the last output plane of a split: its partial sums are in buffer (nsteps-1) & 1
        if constexpr (KS > 1 && KP == 0) {
            const int p = nsteps - 1;
            switch (p % 3) {
            case 0: finish(std::integral_constant<int, 2>{}, p - 1, p & 1); break;
            case 1: finish(std::integral_constant<int, 0>{}, p - 1, p & 1); break;
            default: finish(std::integral_constant<int, 1>{}, p - 1, p & 1); break;
            }
        }
    };

    if constexpr (KS == 1) {
        body(std::integral_constant<int, 0>{});
    } else {
        if (kp == 0) body(std::integral_constant<int, 0>{});
        else body(std::integral_constant<int, 1>{});
    }
}

// ---------------------------------------------------------------- host side
struct ZShape {
    int ntx, nty, zb, nzc;
};

// Planes per block: the fewest rounds of blocks over the chip, then the least
// staging overhead ((zb + 2) / zb input planes per output plane).
ZShape zshape(int nx, int ny, int nz, int bx, int by, int blocks_per_cu, bool even) {
    ZShape s;
    s.ntx = (nx + bx - 1) / bx;
    s.nty = (ny + by - 1) / by;
    const long xy = (long)s.ntx * s.nty;
    const long slots = 256L * blocks_per_cu;
    double best = 1e30;
    s.zb = nz;
    for (int zb = even ? 2 : 1; zb <= nz; zb += even ? 2 : 1) {
        const long nzc = (nz + zb - 1) / zb;
        if (!even && zb > 1 && (long)((nz + zb - 2) / (zb - 1)) == nzc) continue;   // same chunk count, smaller chunks
        const long rounds = (xy * nzc + slots - 1) / slots;
        const double cost = (double)rounds * (zb + 2);
        if (cost < best - 1e-9) {
            best = cost;
            s.zb = zb;
        }
    }
    s.nzc = (nz + s.zb - 1) / s.zb;
    return s;
}

template <int CA, bool UPA, int CB, int MS, int KS, int RY, int WX, int OUT>
void launch_z(const bf16_t *XA, int lda, const bf16_t *XB, int ldb, const bf16_t *wz, const float *bias, bf16_t *Y,
              int ldy, float *Pf, const float *hw, bf16_t *Yp, int nx, int ny, int nz, hipStream_t st) {
    using C = ZCfg<CA, UPA, CB, MS, KS, RY, WX>;
    // resident blocks per compute unit (registers and LDS), asked once per instantiation
    static int bpc = 0;
    if (bpc == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_convz<CA, UPA, CB, MS, KS, RY, WX, OUT>, 320, 0) !=
                hipSuccess || n < 1)
            n = 1;
        bpc = n;
    }
    // pooling pairs planes: blocks start on even planes (nz is even there)
    const ZShape s = zshape(nx, ny, nz, C::BX, C::BY, bpc, OUT == 4);
    const int ntiles = s.ntx * s.nty * s.nzc;
    hipLaunchKernelGGL((k_convz<CA, UPA, CB, MS, KS, RY, WX, OUT>), dim3((ntiles + 7) / 8 * 8), dim3(320), 0, st, XA,
                       lda, XB, ldb, wz, bias, Y, ldy, Pf, hw, Yp, nx, ny, nz, s.zb, s.ntx, s.nty, ntiles);
}

// Rows per wave: 6 (fewer halo rows per staged row) for the 16-channel layers, whose
// accumulators fit beside 15 weight fragments without spilling (measured faster there;
// the packed first layer and the split layers keep two blocks per compute unit with 4),
// where two planes of transfers fit the load counter; else 4.
constexpr int zrows(int ca, int cb, int ms, int ks, int wx) {
    const bool fits = ms * ks < 4 && ca == 16 && cb == 0;
    const int wy = 4 / (ms * ks * wx), ry = fits ? 6 : 4;
    const int plane = (ry * wy + 3) * (16 * wx + 2) * (ca == 4 ? 8 : (ca + cb) * 2);
    const int ni = (plane / (ca == 4 ? 4 : 16) + 63) / 64;
    return ni <= 31 ? ry : 4;
}

// The chunks are split over two waves where one wave would hold more than 36 weight
// fragments for 16 output channels (and two waves per output tile fit); the spatial
// tile is the widest x-extent that fits nx.
template <int CA, bool UPA, int CB, int MS, int OUT>
void launch_zw(const bf16_t *XA, int lda, const bf16_t *XB, int ldb, const bf16_t *wz, const float *bias, bf16_t *Y,
               int ldy, float *Pf, const float *hw, bf16_t *Yp, int nx, int ny, int nz, hipStream_t st) {
    constexpr int KS = MS <= 2 && znfrags(CA, CB) > 36 ? 2 : 1;
    static_assert(znfrags(CA, CB) / KS <= 36, "weight fragments per wave");
    constexpr int WXMAX = 4 / (MS * KS);
    if (WXMAX > 1 && nx > 16 * (WXMAX / 2))
        launch_z<CA, UPA, CB, MS, KS, zrows(CA, CB, MS, KS, WXMAX), WXMAX, OUT>(XA, lda, XB, ldb, wz, bias, Y, ldy,
                                                                                 Pf, hw, Yp, nx, ny, nz, st);
    else
        launch_z<CA, UPA, CB, MS, KS, zrows(CA, CB, MS, KS, 1), 1, OUT>(XA, lda, XB, ldb, wz, bias, Y, ldy, Pf, hw,
                                                                          Yp, nx, ny, nz, st);
}

}  // namespace

int convz_nfrags(int ca, int cb) { return znfrags(ca, cb); }

bool convz_supported(int ca, bool upa, int cb, int cout, int out) {
#define FX_Z_CASE(a, u, b, co, o) if (ca == a && upa == u && cb == b && cout == co && out == o) return true;
    FX_Z_CONFIGS(FX_Z_CASE)
#undef FX_Z_CASE
    return false;
}

void convz_prep(const float *theta_w, int cin, int cout, int ca, int cb, int ci_off, bf16_t *wz, hipStream_t st) {
    const int nf = znfrags(ca, cb);
    const int total = (cout / 16) * nf * 512;
    hipLaunchKernelGGL(k_prepz, dim3((total + 255) / 256), dim3(256), 0, st, theta_w, cin, cout, ca, cb, ci_off, nf,
                       wz);
}

bool convz_forward(int ca, bool upa, int cb, int cout, int out, const bf16_t *XA, int lda, const bf16_t *XB, int ldb,
                   const bf16_t *wz, const float *bias, bf16_t *Y, int ldy, float *Pf, const float *hw, bf16_t *Yp,
                   int nx, int ny, int nz, hipStream_t st) {
    if ((upa || out == 4) && ((nx | ny | nz) & 1)) return false;     // the coarser level is exactly half
#define FX_Z_CASE(a, u, b, co, o)                                                                               \
    if (ca == a && upa == u && cb == b && cout == co && out == o) {                                             \
        launch_zw<a, u, b, co / 16, o>(XA, lda, XB, ldb, wz, bias, Y, ldy, Pf, hw, Yp, nx, ny, nz, st);         \
        return true;                                                                                            \
    }
    FX_Z_CONFIGS(FX_Z_CASE)
#undef FX_Z_CASE
    return false;
}

}  // namespace fx
