// HIP kernels of the TDGL + Poisson time step (gfx950, wave64).
//
// Layout: fields are z-major with x fastest.  Multigrid levels with even x
// and y extents store their cells split by red/black colour (LevelArgs), so a
// Gauss-Seidel half-sweep streams contiguous arrays.  Workgroups are 64x4
// threads (one wave per row).  Every launch covers all instances of a batch:
// a block's global tile index is first remapped so that each of the 8 XCDs
// walks one contiguous range of tiles (consecutive planes and rows, keeping
// stencil neighbours in that XCD's L2), then split into (instance, tile) by a
// binary search in the launch's prefix table.
#include "fx_internal.h"

#include <hip/hip_ext.h>

namespace fx {

namespace {

__device__ __forceinline__ int wrap_p(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// Explicit address spaces.  Pointers read from the instance table are
// generic; used as such they become flat instructions, which need 64-bit
// per-lane addresses and make every wait for a scalar load also wait for the
// vector loads in flight.  The kernels therefore view the arrays through
// global (1) pointers, and the coarse kernel its LDS copies through LDS (3)
// pointers.
#define FX_AS(n) __attribute__((address_space(n)))
template <int AS, typename T>
__device__ __forceinline__ T FX_AS(AS) *asp(T *p) { return (T FX_AS(AS) *)p; }

typedef InstState FX_AS(1) GState;
typedef double dpair __attribute__((ext_vector_type(2)));   // a 16-byte phi pair

template <typename T, int AS>
struct Lv {
    using value_type = T;
    int nx, ny, nz, rb;
    const T FX_AS(AS) *cxy, *czm, *czp, *dg;
    T FX_AS(AS) *e, *r, *sig;
    int sig_lo, sig_hi;
};

template <typename T, int AS = 1>
struct Xv {
    const int FX_AS(AS) *cks, *ccnt, *fthick, *cthick, *pka, *pkb;
    const T FX_AS(AS) *pwa, *pwb;
    int xy;
};

template <typename T>
__device__ __forceinline__ Lv<T, 1> gview(const LevelArgs<T> &L) {
    Lv<T, 1> v;
    v.nx = L.nx; v.ny = L.ny; v.nz = L.nz; v.rb = L.rb;
    v.cxy = asp<1>(L.cxy); v.czm = asp<1>(L.czm); v.czp = asp<1>(L.czp); v.dg = asp<1>(L.dg);
    v.e = asp<1>(L.e); v.r = asp<1>(L.r); v.sig = asp<1>(L.sig);
    v.sig_lo = L.sig_lo; v.sig_hi = L.sig_hi;
    return v;
}

template <typename T>
__device__ __forceinline__ Xv<T> xview(const XferArgs<T> &X) {
    Xv<T> v;
    v.cks = asp<1>(X.cks); v.ccnt = asp<1>(X.ccnt); v.fthick = asp<1>(X.fthick); v.cthick = asp<1>(X.cthick);
    v.pka = asp<1>(X.pka); v.pkb = asp<1>(X.pkb); v.pwa = asp<1>(X.pwa); v.pwb = asp<1>(X.pwb);
    v.xy = X.xy;
    return v;
}

// State of instance inst of a work-table launch, addressed from the kernel argument
// (one load, not a load of the pointer held in the instance and then of the state).
__device__ __forceinline__ GState *wstate(const Work &w, int inst) { return asp<1>(w.st + inst); }

struct Blk {
    int inst, t;
    bool ok;
};

__device__ __forceinline__ Blk find_block(const Work &w) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int g = (b & 7) * (nb >> 3) + (b >> 3);
    Blk r;
    r.ok = g < w.total;
    r.inst = 0;
    r.t = 0;
    if (!r.ok) return r;
    if (w.ninst == 1) {                       // prefix[0] = 0: no table lookup
        r.t = g;
        return r;
    }
    const int FX_AS(1) *pre = asp<1>(w.prefix);
    int lo = 0, hi = w.ninst;                 // largest lo with prefix[lo] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= g) lo = mid;
        else hi = mid;
    }
    r.inst = __builtin_amdgcn_readfirstlane(lo);
    r.t = g - pre[r.inst];
    return r;
}

struct T3 {
    int tx, ty, tz;
};
__device__ __forceinline__ T3 split3(int t, int nxw, int ny) {
    const int ntx = (nxw + BX - 1) / BX, nty = (ny + BY - 1) / BY;
    T3 r;
    r.tx = t % ntx;
    const int q = t / ntx;
    r.ty = q % nty;
    r.tz = q / nty;
    return r;
}

// The same tiles in z-fastest order (nzt tiles per column): consecutive tiles of one
// column share their halo planes, which the next tile then finds in L2.
__device__ __forceinline__ T3 split3z(int t, int nxw, int nzt) {
    const int ntx = (nxw + BX - 1) / BX;
    T3 r;
    r.tz = t % nzt;
    const int q = t / nzt;
    r.tx = q % ntx;
    r.ty = q / ntx;
    return r;
}

// Tile of 2^lbx x 2^(8-lbx) threads (a 256-thread block, x fastest); the
// smoother's tile shape is chosen per level at run time.
__device__ __forceinline__ T3 split3r(int t, int nxw, int ny, int lbx) {
    const int ntx = (nxw + (1 << lbx) - 1) >> lbx, nty = (ny + (256 >> lbx) - 1) >> (8 - lbx);
    T3 r;
    r.tx = t % ntx;
    const int q = t / ntx;
    r.ty = q % nty;
    r.tz = q / nty;
    return r;
}

dim3 grid_of(int total) { return dim3((total + 7) / 8 * 8); }

template <typename V>
__device__ __forceinline__ int cidx(const V &L, int i, int j, int k) {
    const int lin = (k * L.ny + j) * L.nx + i;
    if (!L.rb) return lin;
    return (((i + j + k) & 1) ? ((L.nx * L.ny * L.nz) >> 1) : 0) + (lin >> 1);
}

template <typename V>
__device__ __forceinline__ bool has_sig(const V &L, int k) { return k >= L.sig_lo && k < L.sig_hi; }

template <typename V>
__device__ __forceinline__ int sidx(const V &L, int i, int j, int k) {
    const int lin = ((k - L.sig_lo) * L.ny + j) * L.nx + i;
    if (!L.rb) return lin;
    return (((i + j + k) & 1) ? ((L.nx * L.ny * (L.sig_hi - L.sig_lo)) >> 1) : 0) + (lin >> 1);
}

// sum over the 6 neighbours of coefficient * e(neighbour); Dirichlet neighbours are zero
template <typename V, typename P>
__device__ __forceinline__ typename V::value_type nb_sum(const V &L, P e, int i, int j, int k) {
    using T = typename V::value_type;
    T s = 0;
    const T cx = L.cxy[k];
    if (L.nx > 1) s += cx * (e[cidx(L, wrap_p(i, L.nx), j, k)] + e[cidx(L, wrap_m(i, L.nx), j, k)]);
    if (L.ny > 1) s += cx * (e[cidx(L, i, wrap_p(j, L.ny), k)] + e[cidx(L, i, wrap_m(j, L.ny), k)]);
    if (k > 0) s += L.czm[k] * e[cidx(L, i, j, k - 1)];
    if (k < L.nz - 1) s += L.czp[k] * e[cidx(L, i, j, k + 1)];
    return s;
}

template <typename V>
__device__ __forceinline__ typename V::value_type diag_of(const V &L, int i, int j, int k) {
    typename V::value_type d = L.dg[k];
    if (has_sig(L, k)) d += L.sig[sidx(L, i, j, k)];
    return d;
}

// Gauss-Seidel update of one cell of (L + diag sigma) e = r.
template <typename V>
__device__ __forceinline__ void gs_cell(const V &L, int i, int j, int k, int zero_init) {
    const int c = cidx(L, i, j, k);
    const auto d = diag_of(L, i, j, k);
    L.e[c] = zero_init ? L.r[c] / d : (L.r[c] + nb_sum(L, L.e, i, j, k)) / d;
}

// Colour of a cell on a plainly stored level (odd x or y extent).  With an
// odd periodic extent the parity colouring makes the wrap neighbours equal
// coloured, so the last column / row (for odd nx / ny) get colours 2 and 3:
// no two cells of one colour are then neighbours, and a sweep is the four
// colours in turn.
template <typename V>
__device__ __forceinline__ int nat_color(const V &L, int i, int j, int k) {
    const int par = (i + j + k) & 1;
    const bool edge = ((L.nx & 1) && i == L.nx - 1) || ((L.ny & 1) && j == L.ny - 1);
    return edge ? 2 + par : par;
}

// Residual of the finer level restricted to one coarse cell: volume-weighted
// mean over the children, likewise sigma.  On a red/black level the black
// children are skipped: right after a black half-sweep their residual is
// zero (each black equation has just been solved exactly).
// The child loops are unrolled (XY fixes their extent, a coarse plane has one
// or two children) so that a thread issues all its loads together.  XY is the
// lateral transfer mode: 0 none, 1 x and y halved, 2 x halved on a single row.
template <int XY, typename V, typename X>
__device__ __forceinline__ void restrict_cell_t(const V &F, const V &C, const X &Xf, int I, int J, int K) {
    using T = typename V::value_type;
    constexpr int nsx = XY ? 2 : 1, nsy = XY == 1 ? 2 : 1;
    double sr = 0.0, ss = 0.0;
    const int ks = Xf.cks[K], cnt = Xf.ccnt[K];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        if (dz >= cnt) break;
        const int k = ks + dz;
        const double wz = (double)Xf.fthick[k] / (double)Xf.cthick[K];
        const bool hs = has_sig(F, k);
#pragma unroll
        for (int dy = 0; dy < nsy; ++dy) {
            const int j = XY == 1 ? 2 * J + dy : J;
#pragma unroll
            for (int dx = 0; dx < nsx; ++dx) {
                const int i = XY ? 2 * I + dx : I;
                const T sg = hs ? F.sig[sidx(F, i, j, k)] : T(0);
                ss += wz * (double)sg;
                if (F.rb && ((i + j + k) & 1)) continue;
                const int c = cidx(F, i, j, k);
                const T res = F.r[c] - ((F.dg[k] + sg) * F.e[c] - nb_sum(F, F.e, i, j, k));
                sr += wz * (double)res;
            }
        }
    }
    const double wxy = XY == 1 ? 0.25 : (XY == 2 ? 0.5 : 1.0);
    C.r[cidx(C, I, J, K)] = (T)(sr * wxy);
    if (has_sig(C, K)) C.sig[sidx(C, I, J, K)] = (T)(ss * wxy);
}
template <typename V, typename X>
__device__ __forceinline__ void restrict_cell(const V &F, const V &C, const X &Xf, int I, int J, int K) {
    if (Xf.xy == 1) restrict_cell_t<1>(F, C, Xf, I, J, K);
    else if (Xf.xy == 2) restrict_cell_t<2>(F, C, Xf, I, J, K);
    else restrict_cell_t<0>(F, C, Xf, I, J, K);
}

// The same restriction for a red/black level halved in x and y, in global
// memory, with every load issued before any arithmetic: in each child row the
// red child is the one with dx = (dy + k) & 1, a coarse plane with a single
// child reads that plane twice (the copy is skipped below), and sigma outside
// the semiconductor planes is read from the cell's own residual and ignored.
// Without conditional loads the compiler keeps all of them (48) in flight at
// once instead of waiting on each child's stencil in turn.
template <typename V, typename X>
__device__ __forceinline__ void restrict_cell_rbxy(const V &F, const V &C, const X &Xf, int I, int J, int K) {
    using T = typename V::value_type;
    const int ks = Xf.cks[K], cnt = Xf.ccnt[K];
    T sg[2][2][2], rv[2][2], ev[2][2], nb[2][2][6], cx[2], czm[2], czp[2], dg[2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        const int k = ks + (dz < cnt ? dz : 0);
        const bool hs = has_sig(F, k);
        const int km = k > 0 ? k - 1 : k, kp = k < F.nz - 1 ? k + 1 : k;
        cx[dz] = F.cxy[k];
        czm[dz] = F.czm[k];
        czp[dz] = F.czp[k];
        dg[dz] = F.dg[k];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int j = 2 * J + dy;
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int i = 2 * I + dx;
                const auto sp = hs ? F.sig + sidx(F, i, j, k) : F.r + cidx(F, i, j, k);
                sg[dz][dy][dx] = *sp;
            }
            const int i = 2 * I + ((dy + k) & 1);
            const int c = cidx(F, i, j, k);
            rv[dz][dy] = F.r[c];
            ev[dz][dy] = F.e[c];
            nb[dz][dy][0] = F.e[cidx(F, wrap_p(i, F.nx), j, k)];
            nb[dz][dy][1] = F.e[cidx(F, wrap_m(i, F.nx), j, k)];
            nb[dz][dy][2] = F.e[cidx(F, i, wrap_p(j, F.ny), k)];
            nb[dz][dy][3] = F.e[cidx(F, i, wrap_m(j, F.ny), k)];
            nb[dz][dy][4] = F.e[cidx(F, i, j, km)];
            nb[dz][dy][5] = F.e[cidx(F, i, j, kp)];
        }
    }
    double sr = 0.0, ss = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        if (dz >= cnt) break;
        const int k = ks + dz;
        const double wz = (double)Xf.fthick[k] / (double)Xf.cthick[K];
        const bool hs = has_sig(F, k);
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const T sgc = hs ? sg[dz][dy][dx] : T(0);
                ss += wz * (double)sgc;
                if (dx != ((dy + k) & 1)) continue;
                T nbs = 0;
                nbs += cx[dz] * (nb[dz][dy][0] + nb[dz][dy][1]);
                nbs += cx[dz] * (nb[dz][dy][2] + nb[dz][dy][3]);
                if (k > 0) nbs += czm[dz] * nb[dz][dy][4];
                if (k < F.nz - 1) nbs += czp[dz] * nb[dz][dy][5];
                const T res = rv[dz][dy] - ((dg[dz] + sgc) * ev[dz][dy] - nbs);
                sr += wz * (double)res;
            }
        }
    }
    C.r[cidx(C, I, J, K)] = (T)(sr * 0.25);
    if (has_sig(C, K)) C.sig[sidx(C, I, J, K)] = (T)(ss * 0.25);
}

// Fused multiply-add of the working precision, written out so that every kernel that
// interpolates rounds alike whatever the compiler would contract.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The lateral interpolant of one coarse plane: sum of w[yy][xx] v[yy][xx] in row order,
// the first term a product and the others fused multiply-adds.  With lint_z, the value
// of a fine plane from its parent plane s0 and the neighbour plane s1.  Every
// prolongation (per fine cell, fused into the red half-sweep, by coarse columns, and
// inside the coarse kernel) goes through these two, so their corrections agree bit for
// bit.
template <int NY, int NX, typename T>
__device__ __forceinline__ T lint_xy(const T (&w)[2][2], const T (&v)[2][2]) {
    T s = w[0][0] * v[0][0];
#pragma unroll
    for (int yy = 0; yy < NY; ++yy)
#pragma unroll
        for (int xx = 0; xx < NX; ++xx)
            if (yy + xx > 0) s = fmad(w[yy][xx], v[yy][xx], s);
    return s;
}
template <typename T>
__device__ __forceinline__ T lint_z(T wa, T s0, T wb, T s1) {
    return fmad(wb, s1, wa * s0);
}

// e_f += I e_c: bilinear in x,y (cell-centred 3/4, 1/4), in z linear in the
// series resistance between coarse plane centres (zero on contact faces).  On
// a red/black level only black cells are corrected: the red values are
// overwritten by the next red half-sweep without being read.
// Unrolled like the restriction: all coarse values are loaded together; a
// missing second plane (contact side) reads the first with weight zero.
// prolong_value returns the interpolated correction of fine cell (i, j, k);
// XY is the lateral transfer mode as in the restriction (2: linear in x only).
template <int XY, typename V, typename X>
__device__ __forceinline__ typename V::value_type prolong_value(const V &C, const X &Xf, int i, int j, int k) {
    using T = typename V::value_type;
    constexpr int nsx = XY ? 2 : 1, nsy = XY == 1 ? 2 : 1;
    int ix[2], jy[2];
    T wx[2], wy[2];
    if (XY == 1) {
        const int I = i >> 1, J = j >> 1;
        ix[0] = I; ix[1] = (i & 1) ? wrap_p(I, C.nx) : wrap_m(I, C.nx);
        jy[0] = J; jy[1] = (j & 1) ? wrap_p(J, C.ny) : wrap_m(J, C.ny);
        wx[0] = wy[0] = T(0.75);
        wx[1] = wy[1] = T(0.25);
    } else if (XY == 2) {
        const int I = i >> 1;
        ix[0] = I; ix[1] = (i & 1) ? wrap_p(I, C.nx) : wrap_m(I, C.nx);
        jy[0] = jy[1] = j;
        wx[0] = T(0.75);
        wx[1] = T(0.25);
        wy[0] = T(1);
        wy[1] = T(0);
    } else {
        ix[0] = ix[1] = i; jy[0] = jy[1] = j; wx[0] = wy[0] = T(1);
        wx[1] = wy[1] = T(0);
    }
    const int ka = Xf.pka[k], kb = Xf.pkb[k];
    const int kz[2] = {ka, kb >= 0 ? kb : ka};
    T w[2][2], s[2];
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int xx = 0; xx < 2; ++xx) w[yy][xx] = wx[xx] * wy[yy];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        T v[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
        for (int yy = 0; yy < nsy; ++yy)
#pragma unroll
            for (int xx = 0; xx < nsx; ++xx) v[yy][xx] = C.e[cidx(C, ix[xx], jy[yy], kz[q])];
        s[q] = lint_xy<nsy, nsx>(w, v);
    }
    return lint_z(T(Xf.pwa[k]), s[0], kb >= 0 ? T(Xf.pwb[k]) : T(0), s[1]);
}
template <typename V, typename X>
__device__ __forceinline__ void prolong_cell(const V &F, const V &C, const X &Xf, int i, int j, int k) {
    if (F.rb && !((i + j + k) & 1)) return;
    F.e[cidx(F, i, j, k)] += Xf.xy == 1   ? prolong_value<1>(C, Xf, i, j, k)
                             : Xf.xy == 2 ? prolong_value<2>(C, Xf, i, j, k)
                                          : prolong_value<0>(C, Xf, i, j, k);
}

// Sum over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if ((tid & 63) == 0) lds[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int q = 0; q < (int)((blockDim.x * blockDim.y) >> 6); ++q) s += lds[q];
    return s;
}

// phi buffer holding the input / output of the cycle in progress (cycle c = cycles)
__device__ __forceinline__ int cyc_src(const GState *s) {
    return s->cycles == 0 ? s->start : ((s->cycles - 1) % 2 == 0 ? s->oth0 : s->oth1);
}
__device__ __forceinline__ int cyc_dst(const GState *s) { return s->cycles % 2 == 0 ? s->oth0 : s->oth1; }

// ------------------------------------------------------------------- TDGL
// eq. (TDGL2) with forward Euler (Step 1a); surface stencils of eqs. (Pbc),
// (PbcFree), (PbcDir) on the two ferroelectric boundary planes.
__device__ __forceinline__ double surface_value(int pbc, double lambda, double h, double p0, double p1) {
    if (pbc == 0) return (9.0 * p0 - p1) * 0.125;
    if (pbc == 1) return 0.0;
    return lambda * (9.0 * p0 - p1) / (8.0 * lambda + 3.0 * h);
}

// The variational force dF/dP of eq. (TDGL2) at cell (i, j, k), c its index;
// the time derivative is -Gamma times it.
template <typename T>
__device__ __forceinline__ double tdgl_force(const Inst<T> &a, const double FX_AS(1) *P,
                                             const double FX_AS(1) *phi, int i, int j, int k, size_t c) {
    const size_t nxy = (size_t)a.nx * a.ny;
    const double h = a.h, ih2 = 1.0 / (h * h), i2h = 0.5 / h;
    const double p = P[c];
    const size_t row = c - i;
    const double dxx = (P[row + wrap_p(i, a.nx)] - 2.0 * p + P[row + wrap_m(i, a.nx)]) * ih2;
    const size_t pl = (size_t)k * nxy + i;
    const double dyy = (P[pl + (size_t)wrap_p(j, a.ny) * a.nx] - 2.0 * p + P[pl + (size_t)wrap_m(j, a.ny) * a.nx]) * ih2;
    double dzz, dphi;
    if (k == a.f0) {
        const double p1 = P[c + nxy];
        dzz = 4.0 * (2.0 * surface_value(a.pbc, a.lambda, h, p, p1) - 3.0 * p + p1) * ih2 * (1.0 / 3.0);
        dphi = (-3.0 * phi[c] + 4.0 * phi[c + nxy] - phi[c + 2 * nxy]) * i2h;
    } else if (k == a.f1 - 1) {
        const double p1 = P[c - nxy];
        dzz = 4.0 * (2.0 * surface_value(a.pbc, a.lambda, h, p, p1) - 3.0 * p + p1) * ih2 * (1.0 / 3.0);
        dphi = (3.0 * phi[c] - 4.0 * phi[c - nxy] + phi[c - 2 * nxy]) * i2h;
    } else {
        dzz = (P[c + nxy] - 2.0 * p + P[c - nxy]) * ih2;
        dphi = (phi[c + nxy] - phi[c - nxy]) * i2h;
    }
    const double p2 = p * p;
    const double landau = p * (a.alpha + p2 * (a.beta + a.gamma * p2));
    return landau - a.g44 * (dxx + dyy) - a.g11 * dzz + dphi;
}

template <typename T>
__global__ __launch_bounds__(256) void k_tdgl(const Inst<T> *I, Work w, int sel) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *s = wstate(w, b.inst);
    const int adv = s->adv;
    if (!b.ok | ((sel != 0) & (adv == 0))) return;  // one exit test: see smooth_kernel
    const int pcur = s->pcur;
    const T3 t = split3(b.t, a.nx, a.ny);
    const int i = t.tx * BX + threadIdx.x;
    const int j = t.ty * BY + threadIdx.y;
    const int k = a.f0 + t.tz;
    if (i >= a.nx || j >= a.ny) return;
    const size_t c = ((size_t)k * a.ny + j) * a.nx + i;
    const double FX_AS(1) *P = asp<1>(a.P[pcur]);
    const double dF = tdgl_force(a, P, asp<1>(a.phi[s->cur]), i, j, k, c);
    asp<1>(a.P[1 - pcur])[c] = P[c] - s->dt * a.Gamma * dF;
}

// Corrector (Step 2a): P^{n+1} = P^n + dt/2 f(P^n, phi^n) + dt/2 f(P*, phi*); with
// P* = P^n + dt f(P^n, phi^n) this is (P^n + P*)/2 + dt/2 f(P*, phi*).  P^n is
// the other P buffer and is overwritten in place (each cell reads only its own).
template <typename T>
__global__ __launch_bounds__(256) void k_tdgl_corr(const Inst<T> *I, Work w) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *s = wstate(w, b.inst);
    const int corr = s->corr;
    if (!b.ok | (corr == 0)) return;  // one exit test: see smooth_kernel
    const int pcur = s->pcur;
    const T3 t = split3(b.t, a.nx, a.ny);
    const int i = t.tx * BX + threadIdx.x;
    const int j = t.ty * BY + threadIdx.y;
    const int k = a.f0 + t.tz;
    if (i >= a.nx || j >= a.ny) return;
    const size_t c = ((size_t)k * a.ny + j) * a.nx + i;
    const double FX_AS(1) *Ps = asp<1>(a.P[pcur]);
    double FX_AS(1) *Pn = asp<1>(a.P[1 - pcur]);
    const double dF = tdgl_force(a, Ps, asp<1>(a.phi[s->cur]), i, j, k, c);
    Pn[c] = 0.5 * (Pn[c] + Ps[c]) - 0.5 * s->dt * a.Gamma * dF;
}

// ------------------------------------------------------- solve bookkeeping
// After a stand-alone TDGL update: the new P is in the other buffer, and the
// stored time levels no longer belong to one time series.
template <typename T>
__global__ void k_flip(const Inst<T> *I, int ninst) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ninst) return;
    GState *s = asp<1>(I[n].st);
    s->pcur ^= 1;
    s->hist = 0;
}

// One thread per instance: start a solve.  sel = 1 (time step, instances
// flagged by the advance slot): the TDGL update just written becomes the
// current P, the gate potential comes from the run's schedule, and the
// starting iterate may be extrapolated in time.  sel = 0: a plain solve of
// every instance from its current phi.
template <typename T>
__global__ void k_begin(const Inst<T> *I, InstState *S, int ninst, int sel) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ninst) return;
    const Inst<T> &a = I[n];
    GState *gs = asp<1>(S + n);                   // the state array itself (not through the
                                                  // instance): one dependent load fewer
    // read whole, updated in registers and written back once; an instance that
    // starts no solve here is computed alike and not written back, so that no
    // branch stands between the kernel's loads
    InstState st = *(const InstState *)gs, *s = &st;
    const bool run = !(sel && !s->adv && !s->corr);
    if (sel) {
        s->pcur ^= 1;
        const int q = s->step - s->sched_base;
        if (s->adv && q >= 0 && q < s->sched_len) s->v_top = asp<1>(a.vsched)[q];
    } else {
        s->phase = 0;
        s->pstar = -1;
    }
    // A corrector's solve starts from the predictor's phi*, O(dt^2) away from phi^{n+1},
    // unless the history through phi^n supports an extrapolation of order >= 2, which is
    // O(dt^3) away or closer.  A predictor's target phi* differs from phi^{n+1} by a
    // smooth O(dt^2) offset: with the last step's phi* kept, it starts from the
    // extrapolation plus that step's offset phi*_n - phi^n, O(dt^3) away.
    int order = 0;
    if (sel && s->adv) order = min(s->hist, a.warm);
    else if (sel) order = min(s->hist - 1, a.warm) >= 2 ? min(s->hist - 1, a.warm) : 0;
    const int usestar = sel && s->adv && a.order2 && s->pstar >= 0;
    if (!usestar) s->pstar = -1;
    int oth[2] = {0, 0}, no = 0;
    for (int q = 0; q < a.nbuf && no < 2; ++q) {
        bool used = q == s->cur || q == s->pstar;
#pragma unroll
        for (int m = 0; m < kMaxHist; ++m) used |= m < s->hist && s->prev[m] == q;
        if (!used) oth[no++] = q;
    }
    s->oth0 = oth[0];
    s->oth1 = oth[1];
    s->order = order;
    s->usestar = usestar;
    s->start = order > 0 || usestar ? oth[1] : s->cur;
    s->ts = sel;
    s->done = 0;
    s->cycles = 0;
    s->zpend = 0;
    s->fresh = 1;
    s->insolve = 1;
    s->light = 0;
    if (run) *(InstState *)gs = st;
}

// Lagrange extrapolation to t^{n+1} through t^n, t^{n-1}, ... (equal steps).
__constant__ double kExtrapC[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};

template <typename T>
__global__ __launch_bounds__(256) void k_extrap(const Inst<T> *I, Work w) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *s = wstate(w, b.inst);
    const int order = s->order, fresh = s->fresh, usestar = s->usestar;
    if (!b.ok | (fresh == 0) | ((order == 0) & (usestar == 0))) return;  // one exit test: see smooth_kernel
    const size_t nxy = (size_t)a.nx * a.ny, off = (size_t)a.kb * nxy, n = (size_t)a.nzd * nxy;
    const double FX_AS(1) *in[4];
    // newest level phi^n: the current iterate, or for a corrector the last stored level
    const int sh = s->phase == 1 ? 1 : 0;
    in[0] = asp<1>(a.phi[sh ? s->prev[0] : s->cur]) + off;
    for (int q = 1; q <= order; ++q) in[q] = asp<1>(a.phi[s->prev[q - 1 + sh]]) + off;
    double FX_AS(1) *out = asp<1>(a.phi[s->start]) + off;
    const double FX_AS(1) *star = asp<1>(a.phi[s->usestar ? s->pstar : s->cur]) + off;
    const size_t base = (size_t)b.t * kExtrapChunk;
    const int tid = threadIdx.y * BX + threadIdx.x;
    for (int q = 0; q < kExtrapChunk / 256; ++q) {
        const size_t c = base + (size_t)q * 256 + tid;
        if (c >= n) break;
        double v = kExtrapC[order][0] * in[0][c];
        for (int m = 1; m <= order; ++m) v += kExtrapC[order][m] * in[m][c];
        if (s->usestar) v += star[c] - in[0][c];
        out[c] = v;
    }
}

// One thread per instance, first kernel of an advance slot (advance = 1) or
// after a plain solve (advance = 0).  A solve that has stopped is finalized:
// its last iterate becomes phi^{n+1} and, after a successful time step, phi^n
// the newest stored level; the statistics and the status are recorded.
// With advance set, an instance that is idle and below its run target (and
// whose last solve succeeded) is flagged to start the next time step in this
// slot; one that has reached the target or failed is parked.
template <typename T>
__global__ void k_head(const Inst<T> *I, InstState *S, int ninst, int advance) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ninst) return;
    // the state is read whole, updated in registers and written back once (one
    // round trip instead of one per dependent field); the copies go through a generic
    // view (the implicit copy operations take no address-space-qualified operand),
    // which the compiler maps back to global loads and stores
    GState *gs = asp<1>(S + n);
    InstState st = *(const InstState *)gs, *s = &st;
    const int order2 = I[n].order2;
    int zf = 0, corr = 0, stepped = 0;
    if (s->insolve && s->done != 0) {
        const int c = s->cycles;
        s->solves += 1;
        s->total_cycles += c;
        s->max_cycles_step = max(s->max_cycles_step, c);
        s->insolve = 0;
        if (s->done == 2) {                   // non-finite: keep phi^n, drop the history
            s->status = 5;
            s->failed += 1;
            s->hist = 0;
        } else {
            const int fin = c == 0 ? s->start : ((c - 1) % 2 == 0 ? s->oth0 : s->oth1);
            s->status = s->done == 1 ? 0 : 4;
            if (s->status != 0) s->failed += 1;
            const bool ok_step = s->ts && s->status == 0;
            if (ok_step && s->phase == 1) {
                // corrector done: phi^{n+1}; the predictor's phi* is kept for the next
                // predictor's start, phi^n stays the newest stored level
                s->step += 1;
                s->phase = 0;
                stepped = 1;
                s->pstar = s->cur;
            } else if (ok_step) {
                // Euler step, or the predictor of a second-order step: phi^n
                // becomes the newest stored level
                if (fin != s->cur) {
                    // Euler keeps 3 levels; a predictor-corrector instance 4, so that
                    // its corrector, whose newest level is phi^n, extrapolates cubically
                    const int hmax = order2 ? kMaxHist : kMaxHist - 1;
#pragma unroll
                    for (int m = kMaxHist - 1; m > 0; --m)
                        if (m < hmax) s->prev[m] = s->prev[m - 1];
                    s->prev[0] = s->cur;
                    s->hist = min(s->hist + 1, hmax);
                } else {
                    s->hist = 0;
                }
                if (order2) { s->phase = 1; corr = 1; }
                else { s->step += 1; stepped = 1; }
                s->pstar = -1;
            } else {
                s->hist = 0;
                s->phase = 0;
                s->pstar = -1;
            }
            s->cur = fin;
            zf = s->done == 1 && s->zpend;
        }
    }
    s->zero_fix = zf;
    int adv = 0;
    if (advance && !s->parked && !s->insolve && !corr) {
        if (s->status != 0 || s->step >= s->target) s->parked = 1;
        else adv = 1;
    }
    s->adv = adv;
    s->corr = corr;
    s->stepped = stepped;
    *(InstState *)gs = st;
}

// Q-V diagnostics (Results, MFIM).  Across the ferroelectric/dielectric face, with L
// the lower and R the upper plane, the Poisson operator's flux is
// D = -eps_f (phi_R - phi_L)/h + P_f (harmonic-mean eps_f, P_f = (eps_R P_L + eps_L P_R)
// / (eps_L + eps_R)), equal to eps0 eps_DE E_z in the dielectric half cell.  The face
// potential follows from the lower half cell, D = -eps_L (phi_int - phi_L)/(h/2) + P_L.
// Each block sums D and phi_int over a strided share of the face (fixed order), then
// a tree in LDS; the finishing kernel adds the blocks' sums in block order.
template <typename T>
__global__ __launch_bounds__(256) void k_qv_part(const Inst<T> *I, int record) {
    const int inst = blockIdx.x / kQvBlocks, blk = blockIdx.x % kQvBlocks;
    const Inst<T> &a = I[inst];
    const GState *s = asp<1>(a.st);
    if (a.qv_kl < 0 || (record && !s->stepped)) return;
    const size_t nxy = (size_t)a.nx * a.ny;
    const double FX_AS(1) *phL = asp<1>(a.phi[s->cur]) + (size_t)a.qv_kl * nxy;
    const double FX_AS(1) *phR = phL + nxy;
    const double FX_AS(1) *Pfe = asp<1>(a.P[s->pcur]) + (size_t)(a.qv_kl + a.qv_fe_up) * nxy;
    const double eL = a.qv_el, eR = a.qv_er, ih = 1.0 / a.h;
    const double ef = 2.0 * eL * eR / (eL + eR), wL = eR / (eL + eR), wR = eL / (eL + eR);
    const double hh_eL = 0.5 * a.h / eL;
    double sd = 0.0, sp = 0.0;
    for (size_t c = (size_t)blk * 256 + threadIdx.x; c < nxy; c += (size_t)kQvBlocks * 256) {
        const double p = Pfe[c];
        const double pL = a.qv_fe_up ? 0.0 : p, pR = a.qv_fe_up ? p : 0.0;
        const double D = -ef * (phR[c] - phL[c]) * ih + wL * pL + wR * pR;
        sd += D;
        sp += phL[c] - (D - pL) * hh_eL;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = sd;
    red[1][threadIdx.x] = sp;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) {
            red[0][threadIdx.x] += red[0][threadIdx.x + m];
            red[1][threadIdx.x] += red[1][threadIdx.x + m];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double FX_AS(1) *o = asp<1>(a.qv_part) + 2 * blk;
        o[0] = red[0][0];
        o[1] = red[1][0];
    }
}

template <typename T>
__global__ void k_qv_fin(const Inst<T> *I, int ninst, int record, double *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ninst) return;
    const Inst<T> &a = I[n];
    const GState *s = asp<1>(a.st);
    if (record && (a.qv_kl < 0 || !s->stepped)) return;
    double Q = __builtin_nan(""), V = __builtin_nan("");
    if (a.qv_kl >= 0) {
        double sd = 0.0, sp = 0.0;
        const double FX_AS(1) *p = asp<1>(a.qv_part);
        for (int b = 0; b < kQvBlocks; ++b) { sd += p[2 * b]; sp += p[2 * b + 1]; }
        const double area = (double)a.nx * a.ny;
        Q = -sd / area;
        V = s->v_top - sp / area;
    }
    if (record) {
        const int q = s->step - 1 - s->sched_base;
        if (q >= 0 && q < kRecSteps) {
            double FX_AS(1) *r = asp<1>(a.qv_rec) + 2 * q;
            r[0] = Q;
            r[1] = V;
        }
    } else {
        asp<1>(out)[2 * n] = Q;
        asp<1>(out)[2 * n + 1] = V;
    }
}

// ------------------------------------------------------ fine-level residual
// Per-plane tables of the finest level the residual reads (scaled by h^2/eps0).
struct ResTab {
    const double FX_AS(1) *cxy, *czm, *czp, *wl, *wr, *p0e, *n0e;
};
template <typename T>
__device__ __forceinline__ ResTab res_tab(const Inst<T> &a) {
    return ResTab{asp<1>(a.cxy0), asp<1>(a.czm0), asp<1>(a.czp0), asp<1>(a.wl), asp<1>(a.wr), asp<1>(a.p0e),
                  asp<1>(a.n0e)};
}

// One device cell of plane k (eq. (Poisson) with eq. (rho), scaled by h^2/eps0): the
// right-hand side f (contact terms and the bound charge -(P_f(k+1/2) - P_f(k-1/2))/h),
// the residual r = f - N(phi) and the Newton sigma = -d rho_c/d phi (semiconductor
// planes).  v0 is the cell's phi, vx0/vx1 and vy0/vy1 its x+1/x-1 and y+1/y-1
// neighbours, vzm/vzp its z neighbours (not used on the contact planes), pm/pc/pp P on
// planes k-1, k, k+1 (read only where a polarised face touches the plane).  Fused
// multiply-adds are written out, so that every residual kernel rounds alike.  FD = 0
// leaves the Fermi-Dirac branch out (launches whose instances all take Boltzmann carriers:
// fewer registers, no scalar registers parked in vector lanes).
template <typename T, int FD>
__device__ __forceinline__ void res_cell(const Inst<T> &a, const ResTab &tb, int k, int nzd, int fl, double v_t,
                                        double v0, double vx0, double vx1, double vy0, double vy1, double vzm,
                                        double vzp, double pm, double pc, double pp, double &f_o, double &r_o,
                                        double &sg_o) {
    const double nb = fmad(-2.0, v0, vx0 + vx1) + fmad(-2.0, v0, vy0 + vy1);
    const double dn = k > 0 ? vzm : 0.0;
    const double up = k < nzd - 1 ? vzp : 0.0;
    const double Lphi = fmad(tb.czp[k], v0 - up, fmad(tb.czm[k], v0 - dn, -tb.cxy[k] * nb));
    double f = 0.0;
    if (fl & PF_P) {
        const double pup = k == nzd - 1 ? pc : fmad(tb.wr[k], pp, tb.wl[k] * pc);
        const double pdn = k == 0 ? pc : fmad(tb.wr[k - 1], pc, tb.wl[k - 1] * pm);
        f = -(pup - pdn) * a.p_scale;
    }
    if (k == 0) f = fmad(tb.czm[k], a.v_b, f);
    if (k == nzd - 1) f = fmad(tb.czp[k], v_t, f);
    double r = f - Lphi, sg = 0.0;
    if (fl & PF_SC) {
        const double u = v0 * a.vt_inv;
        const double p0e = tb.p0e[k], n0e = tb.n0e[k];
        if (FD && a.fd) {
            // differences from the neutral state: rho_c(0) = 0 exactly
            const double FX_AS(1) *ft = asp<1>(a.fdt) + 4 * k;
            double Fp, dFp, Fn, dFn;
            fd_half(ft[0] - u, Fp, dFp);
            fd_half(ft[1] + u, Fn, dFn);
            r = fmad(fmad(p0e, Fp - ft[2], -(n0e * (Fn - ft[3]))), a.rho_scale, r);
            sg = fmad(p0e, dFp, n0e * dFn) * a.sig_scale;
        } else {
            // e^u - 1 and e^-u - 1 from one expm1: with t = e^|u| - 1 the other
            // is -t / (1 + t), free of cancellation for either sign of u
            const double t1 = expm1(fabs(u));
            const double t2 = -t1 / (1.0 + t1);
            const double ep = u >= 0.0 ? t1 : t2, em = u >= 0.0 ? t2 : t1;
            r = fmad(fmad(p0e, em, -(n0e * ep)), a.rho_scale, r);           // + rho_c
            sg = fmad(p0e, 1.0 + em, n0e * (1.0 + ep)) * a.sig_scale;
        }
    }
    f_o = f;
    r_o = r;
    sg_o = sg;
}

// Each thread owns a column of kResZ planes.  All loads are issued before any
// arithmetic (clamped indices instead of boundary branches; the column's
// z-neighbours are loaded once) and all stores follow it, so a wave makes one
// memory round trip for kResZ cells.  Mode 0 evaluates the current iterate; mode 2 (update not
// folded into the smoother) first forms phi_out = phi_in + clip(e).
template <typename T, int MODE, int FD>
__device__ __forceinline__ void residual_body(const Inst<T> &a, const GState *s, const T3 &t, int after_cycle,
                                              double &rr, double &ff) {
    const int ZT = kResZ;
    const int nx = a.nx, ny = a.ny, nzd = a.nzd;
    const int ii = t.tx * BX + threadIdx.x;
    const int jj = t.ty * BY + threadIdx.y;
    const bool live = ii < nx && jj < ny;
    const int i = live ? ii : 0, j = live ? jj : 0;
    const int k0 = t.tz * ZT;
    const int nxy = nx * ny;
    const size_t off = (size_t)a.kb * nxy;
    const int bin = MODE == 2 ? cyc_src(s) : (after_cycle ? cyc_dst(s) : s->start);
    const double FX_AS(1) *phi = asp<1>(a.phi[bin]) + off;
    double FX_AS(1) *phi_out = asp<1>(a.phi[cyc_dst(s)]) + off;
    const double FX_AS(1) *P = asp<1>(a.P[s->pcur]) + off;
    const Lv<T, 1> L = gview(a.lv[0]);
    const int FX_AS(1) *pflags = asp<1>(a.pflags);
    const int col = j * nx + i;
    const int ox0 = wrap_p(i, nx) - i, ox1 = wrap_m(i, nx) - i;
    const int oy0 = (wrap_p(j, ny) - j) * nx, oy1 = (wrap_m(j, ny) - j) * nx;
    const int rb = L.rb;
    const int half = (nxy * nzd) >> 1;
    const double big = 1e300;
    auto kcl = [&](int k) { return k < 0 ? 0 : (k >= nzd ? nzd - 1 : k); };
    int fl[ZT];
#pragma unroll
    for (int z = 0; z < ZT; ++z) fl[z] = pflags[kcl(k0 + z)];
    bool anyP = false;
#pragma unroll
    for (int z = 0; z < ZT; ++z) anyP |= (k0 + z < nzd) && (fl[z] & PF_P);
    // P is read only by columns that hold a polarised plane; the others load
    // the phi cells they read anyway (cache hits, values unused), so that no
    // branch joins ahead of the phi loads and every load is in flight at once.
    const double FX_AS(1) *Psrc = anyP ? P : phi;
    double pz[ZT + 2];
#pragma unroll
    for (int z = 0; z < ZT + 2; ++z) pz[z] = Psrc[kcl(k0 - 1 + z) * nxy + col];
    double vc[ZT + 2], vx0[ZT], vx1[ZT], vy0[ZT], vy1[ZT];
    auto at = [&](int k, int o, int par, double *dst) {
        const int c = k * nxy + col + o;
        double v = phi[c];
        if (MODE == 2) {
            const double d = (double)L.e[rb ? (par ? half : 0) + (c >> 1) : c];
            const double lim = (pflags[k] & PF_SC) ? a.dmax : big;
            v += fmin(fmax(d, -lim), lim);
        }
        *dst = v;
    };
    const int par0 = (i + j) & 1;
#pragma unroll
    for (int z = 0; z < ZT + 2; ++z) {
        const int k = kcl(k0 - 1 + z);
        at(k, 0, par0 ^ (k & 1), &vc[z]);
    }
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = kcl(k0 + z);
        const int pn = par0 ^ (k & 1) ^ 1;
        // one row (ny = 1): the y neighbours are the cell itself, of its own colour, so
        // that their terms cancel as in the operator
        const int py = ny > 1 ? pn : pn ^ 1;
        at(k, ox0, pn, &vx0[z]);
        at(k, ox1, pn, &vx1[z]);
        at(k, oy0, py, &vy0[z]);
        at(k, oy1, py, &vy1[z]);
    }
    const double v_t = s->v_top;
    const ResTab tb = res_tab(a);
    double res[ZT], sg[ZT];
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = k0 + z;
        res[z] = 0.0;
        sg[z] = 0.0;
        if (k >= nzd) break;
        double f;
        res_cell<T, FD>(a, tb, k, nzd, fl[z], v_t, vc[z + 1], vx0[z], vx1[z], vy0[z], vy1[z], vc[z], vc[z + 2], pz[z],
                 pz[z + 1], pz[z + 2], f, res[z], sg[z]);
        if (live) {
            rr = fmad(res[z], res[z], rr);
            ff = fmad(f, f, ff);
        }
    }
    if (!live) return;
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = k0 + z;
        if (k >= nzd) break;
        if (MODE == 2) phi_out[k * nxy + col] = vc[z + 1];
        if (fl[z] & PF_SC) L.sig[sidx(L, i, j, k)] = (T)sg[z];
        L.r[cidx(L, i, j, k)] = (T)res[z];
    }
}

// MODE 0 covers every instance except, after a cycle, those whose update is
// not folded into the smoother; MODE 2 covers exactly those (two kernels
// rather than one branch: each keeps its own, smaller register budget).
template <typename T, int MODE, int FD>
__global__ __launch_bounds__(256) void k_residual(const Inst<T> *I, Work w, int after_cycle) {
    __shared__ double lds_r[4];
    __shared__ double lds_f[4];
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *s = wstate(w, b.inst);
    // one exit test: see smooth_kernel
    const int done = s->done, fresh = s->fresh, fold = a.fold;
    if (!b.ok | (after_cycle ? done != 0 : fresh == 0) | ((MODE == 2) != ((after_cycle != 0) & (fold == 0)))) return;
    // tiles walk each column up in z (halo planes shared through L2); the partial sums
    // keep the x-fastest tile index, so the reduction's order does not depend on it
    const int nzt = (a.nzd + kResZ - 1) / kResZ;
    const T3 t = split3z(b.t, a.nx, nzt);
    const int tl = t.tx + ((a.nx + BX - 1) / BX) * (t.ty + ((a.ny + BY - 1) / BY) * t.tz);
    double rr = 0.0, ff = 0.0;
    residual_body<T, MODE, FD>(a, s, t, after_cycle, rr, ff);
    const double sr = block_sum(rr, lds_r);
    const double sf = block_sum(ff, lds_f);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double FX_AS(1) *part = asp<1>(a.part);
        part[2 * tl] = sr;
        part[2 * tl + 1] = sf;
    }
}

// Deterministic final sum of one instance's residual partials (a block per
// instance) and its stop decision.  f = 0 exactly with a nonzero residual: N(0) = 0,
// so phi = 0 is the root; the block sets the solve's last iterate to it at once
// (the slot that finalizes the solve reads that buffer as phi^{n+1}).
template <typename T, int CC>
__global__ __launch_bounds__(1024) void k_reduce(const Inst<T> *I, InstState *S) {
    __shared__ double lr[16];
    __shared__ double lf[16];
    __shared__ int lz;
    const Inst<T> &a = I[blockIdx.x];
    GState *s = asp<1>(S + blockIdx.x);
    // the state and the partials are read together, the partials two per thread at a
    // time, so that the block waits on memory once for them (an instance that is not
    // reduced here ignores what it read); each thread still adds its partials in
    // index order
    const double FX_AS(1) *part = asp<1>(a.part);
    const bool skip = CC ? s->done != 0 : !s->fresh;
    // what the stop decision reads, fetched with the rest
    const double x_prev = s->rn2, tol2 = a.tol2, light_r2 = a.light_r2, light_c2 = a.light_c2;
    const int cycles = s->cycles + (CC ? 1 : 0), max_cycles = a.max_cycles, light_ok = a.light_ok;
    // the solve's last iterate: the start before any cycle, else the latest cycle's output
    const int fin = cycles == 0 ? s->start : ((cycles - 1) % 2 == 0 ? s->oth0 : s->oth1);
    const int n = tiles3(a.nx, a.ny, (a.nzd + kResZ - 1) / kResZ);
    const int B = blockDim.x;
    double r = 0.0, f = 0.0;
    int q = threadIdx.x;
    for (; q + B < n; q += 2 * B) {
        const double r0 = part[2 * q], f0 = part[2 * q + 1];
        const double r1 = part[2 * (q + B)], f1 = part[2 * (q + B) + 1];
        r += r0;
        f += f0;
        r += r1;
        f += f1;
    }
    if (q < n) { r += part[2 * q]; f += part[2 * q + 1]; }
    if (skip) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) { r += __shfl_down(r, off, 64); f += __shfl_down(f, off, 64); }
    if ((threadIdx.x & 63) == 0) { lr[threadIdx.x >> 6] = r; lf[threadIdx.x >> 6] = f; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { x += lr[q]; y += lf[q]; }
        s->rn2 = x;
        s->fn2 = y;
        s->fresh = 0;
        if (CC) s->cycles = cycles;
        int zb = -1;
        if (!isfinite(x) || !isfinite(y)) s->done = 2;
        else if (y == 0.0) {
            s->done = 1;
            s->zpend = x != 0.0;
            if (x != 0.0) zb = fin;
        }
        else if (x <= tol2 * y || x == 0.0) s->done = 1;
        else if (cycles >= max_cycles) s->done = 3;
        // within kLightRatio of the tolerance, after a cycle that contracted the
        // residual at least kLightContraction-fold (the linear regime, as in a
        // time step's first cycle), one V(1,1)-like cycle (contraction about 0.2)
        // finishes the solve at a little over half the cost
        s->light = light_ok && CC && x <= light_r2 * tol2 * y && x * light_c2 <= x_prev;
        lz = zb;
    }
    __syncthreads();
    const int zb = lz;
    if (zb >= 0) {
        const size_t nxy = (size_t)a.nx * a.ny, nn = (size_t)a.nzd * nxy;
        double FX_AS(1) *out = asp<1>(a.phi[zb]) + (size_t)a.kb * nxy;
        for (size_t c = threadIdx.x; c < nn; c += blockDim.x) out[c] = 0.0;
    }
}

// ----------------------------------------------------------------- smoother
// Neighbour sum of a red/black cell from the other colour's six values (the
// z terms vanish on the contact planes); one expression shared by every kernel
// that updates a cell, so that they round alike.
template <typename T, int AS>
__device__ __forceinline__ T rb_nb_sum(const Lv<T, AS> &L, int k, T ex0, T ex1, T ey0, T ey1, T ez0, T ez1) {
    const T cx = L.cxy[k];
    const T cy = L.ny > 1 ? cx : T(0);
    return cx * (ex0 + ex1) + cy * (ey0 + ey1) + (k > 0 ? L.czm[k] : T(0)) * ez0 +
           (k < L.nz - 1 ? L.czp[k] : T(0)) * ez1;
}

// One colour of red-black Gauss-Seidel on (L + diag sigma) e = r.  Split
// storage: a thread per cell of that colour, ZT planes per thread with all
// loads issued first; plainly stored levels: a thread per cell and ZT planes
// of a tile.  UPD (finest level, last black half-sweep, instances whose
// update is folded in) also writes phi_out = phi_in + clip(e) for each black
// cell and its red partner (the pair 2m, 2m+1 of a row).
template <typename T, int ZI, int ZT, int UPD>
__device__ __forceinline__ void smooth_rb_body(const Inst<T> &a, const GState *st, const Lv<T, 1> &L, int t, int color, int lbx) {
    const int hx = L.nx >> 1;
    const T3 tt = split3r(t, hx, L.ny, lbx);
    const int mm = (tt.tx << lbx) + (threadIdx.x & ((1 << lbx) - 1));
    const int jj = (tt.ty << (8 - lbx)) + (threadIdx.x >> lbx);
    const bool live = mm < hx && jj < L.ny;
    const int m = live ? mm : 0, j = live ? jj : 0;           // (0, 0): see the stores
    const int half = (L.nx * L.ny * L.nz) >> 1;
    const int plane = L.ny * hx;
    const T FX_AS(1) *eo = L.e + (color ? 0 : half);
    T FX_AS(1) *es = L.e + (color ? half : 0);
    const T FX_AS(1) *rs = L.r + (color ? half : 0);
    const int hsz = (L.nx * L.ny * (L.sig_hi - L.sig_lo)) >> 1;
    const int oy0 = L.ny > 1 ? (wrap_p(j, L.ny) - j) * hx : 0;
    const int oy1 = L.ny > 1 ? (wrap_m(j, L.ny) - j) * hx : 0;
    const bool upd = UPD && a.fold;
    const double FX_AS(1) *phi_in = nullptr;
    double FX_AS(1) *phi_out = nullptr;
    const int FX_AS(1) *pflags = asp<1>(a.pflags);
    if (upd) {
        const GState *s = st;
        const size_t off = (size_t)a.kb * a.nx * a.ny;
        phi_in = asp<1>(a.phi[cyc_src(s)]) + off;
        phi_out = asp<1>(a.phi[cyc_dst(s)]) + off;
    }
    T out[ZT];
    T rr[ZT], sg[ZT], ex0[ZT], ex1[ZT], ey0[ZT], ey1[ZT], ez0[ZT], ez1[ZT];
    dpair ph[ZT];
    double lim[ZT];
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = min(tt.tz * ZT + z, L.nz - 1);
        const int row = k * plane + j * hx;
        const int q = row + m;
        const bool hs = k >= L.sig_lo && k < L.sig_hi;
        rr[z] = rs[q];
        sg[z] = L.sig[hs ? (color ? hsz : 0) + (k - L.sig_lo) * plane + j * hx + m : 0];
        if (!ZI) {
            const int i = 2 * m + ((color + j + k) & 1);
            const int ip = i + 1 == L.nx ? 0 : i + 1, im = i == 0 ? L.nx - 1 : i - 1;
            ex0[z] = eo[row + (ip >> 1)];
            ex1[z] = eo[row + (im >> 1)];
            ey0[z] = eo[q + oy0];
            ey1[z] = eo[q + oy1];
            ez0[z] = eo[k > 0 ? q - plane : q];
            ez1[z] = eo[k < L.nz - 1 ? q + plane : q];
        }
        if (upd) {
            ph[z] = *(const dpair FX_AS(1) *)(phi_in + (size_t)k * L.nx * L.ny + (size_t)j * L.nx + 2 * m);
            lim[z] = (pflags[k] & PF_SC) ? a.dmax : 1e300;
        }
    }
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = min(tt.tz * ZT + z, L.nz - 1);
        const bool hs = k >= L.sig_lo && k < L.sig_hi;
        T acc = 0;
        if (!ZI) acc = rb_nb_sum(L, k, ex0[z], ex1[z], ey0[z], ey1[z], ez0[z], ez1[z]);
        out[z] = (rr[z] + acc) / (L.dg[k] + (hs ? sg[z] : T(0)));
    }
    // Stores outside branches: a lane past the row end works on cell (0, 0) and a slot past
    // the top on plane nz - 1, from the same inputs as the lane owning that cell, so its store
    // repeats the owner's bits.  (A store under a branch made the next plane's arithmetic
    // wait for it to complete.)
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = min(tt.tz * ZT + z, L.nz - 1);
        es[k * plane + j * hx + m] = out[z];
        if (upd) {
            // the pair's red cell is this black cell's x - 1 (black at 2m + 1) or x + 1
            // neighbour (black at 2m), already read as ex1 / ex0
            const bool odd = ((color + j + k) & 1) != 0;
            const double db = fmin(fmax((double)out[z], -lim[z]), lim[z]);
            const double dr = fmin(fmax((double)(odd ? ex1[z] : ex0[z]), -lim[z]), lim[z]);
            dpair o;
            o.x = ph[z].x + (odd ? dr : db);
            o.y = ph[z].y + (odd ? db : dr);
            *(dpair FX_AS(1) *)(phi_out + (size_t)k * L.nx * L.ny + (size_t)j * L.nx + 2 * m) = o;
        }
    }
}

template <typename T, int ZT>
__device__ __forceinline__ void smooth_nat_body(const Lv<T, 1> &L, int t, int color, int zero_init, int lbx) {
    const T3 tt = split3r(t, L.nx, L.ny, lbx);
    const int i = (tt.tx << lbx) + (threadIdx.x & ((1 << lbx) - 1));
    const int j = (tt.ty << (8 - lbx)) + (threadIdx.x >> lbx);
    if (i >= L.nx || j >= L.ny) return;
    for (int z = 0; z < ZT; ++z) {
        const int k = tt.tz * ZT + z;
        if (k >= L.nz) break;
        if (nat_color(L, i, j, k) != color) {
            if (zero_init) L.e[cidx(L, i, j, k)] = T(0);
            continue;
        }
        gs_cell(L, i, j, k, zero_init);
    }
}

// Zero-start pair on a red/black level: the first red half-sweep of a cycle
// (the correction starts at zero, so a red value is r / diag) and the black
// half-sweep after it, in one launch.  A thread per black cell forms the six red
// neighbour values itself, exactly as the red sweep computes them, and also
// stores the red cell of its own (2m, 2m+1) pair, which is one of its two x
// neighbours: the pairs tile each row, so every red cell is written once, with
// the value the red launch would have written.
template <typename T, int ZT>
__device__ __forceinline__ void smooth_zpair_body(const Lv<T, 1> &L, int t, int lbx) {
    const int hx = L.nx >> 1;
    const T3 tt = split3r(t, hx, L.ny, lbx);
    const int m = (tt.tx << lbx) + (threadIdx.x & ((1 << lbx) - 1));
    const int j = (tt.ty << (8 - lbx)) + (threadIdx.x >> lbx);
    if (m >= hx || j >= L.ny) return;
    const int half = (L.nx * L.ny * L.nz) >> 1;
    const int plane = L.ny * hx;
    const int hsz = (L.nx * L.ny * (L.sig_hi - L.sig_lo)) >> 1;
    T FX_AS(1) *e_red = L.e;
    T FX_AS(1) *e_blk = L.e + half;
    const T FX_AS(1) *r_red = L.r, *r_blk = L.r + half;
    const int oy0 = L.ny > 1 ? (wrap_p(j, L.ny) - j) * hx : 0;
    const int oy1 = L.ny > 1 ? (wrap_m(j, L.ny) - j) * hx : 0;
    // red value at red index c of plane kk after a zero-start red half-sweep
    auto red = [&](int c, int kk) {
        const bool hs = kk >= L.sig_lo && kk < L.sig_hi;
        const T sg = L.sig[hs ? (kk - L.sig_lo) * plane + (c - kk * plane) : 0];
        return (r_red[c] + T(0)) / (L.dg[kk] + (hs ? sg : T(0)));
    };
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = tt.tz * ZT + z;
        if (k >= L.nz) break;
        const int row = k * plane + j * hx;
        const int q = row + m;
        const int i = 2 * m + ((1 + j + k) & 1);
        const int ip = i + 1 == L.nx ? 0 : i + 1, im = i == 0 ? L.nx - 1 : i - 1;
        const bool hs = k >= L.sig_lo && k < L.sig_hi;
        const T rb = r_blk[q];
        const T sb = L.sig[hs ? hsz + (k - L.sig_lo) * plane + j * hx + m : 0];
        const T ex0 = red(row + (ip >> 1), k), ex1 = red(row + (im >> 1), k);
        const T ey0 = red(q + oy0, k), ey1 = red(q + oy1, k);
        const T ez0 = k > 0 ? red(q - plane, k - 1) : red(q, k);
        const T ez1 = k < L.nz - 1 ? red(q + plane, k + 1) : red(q, k);
        const T acc = rb_nb_sum(L, k, ex0, ex1, ey0, ey1, ez0, ez1);
        e_blk[q] = (rb + acc) / (L.dg[k] + (hs ? sb : T(0)));
        e_red[q] = (i & 1) ? ex1 : ex0;                  // the pair's red cell: x - 1 or x + 1
    }
}

template <typename T, int ZT>
__global__ __launch_bounds__(256) void k_smooth_zpair(const Inst<T> *I, Work w, int level, int lbx) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const int done = wstate(w, b.inst)->done;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    const Lv<T, 1> L = gview(a.lv[level]);
    if (!L.rb) return;                               // the host fuses only all-red/black levels
    smooth_zpair_body<T, ZT>(L, b.t, lbx);
}

// probe (instrumentation): the first tile of each instance that works adds
// the launch's algorithmic bytes for that instance -- one touch each of this
// colour's r, sigma and e, the other colour's e (not read when zero_init),
// and the phi pair read and written where the update is folded in.
template <typename T, int ZI, int ZT, int UPD>
__device__ __forceinline__ void smooth_kernel(const Inst<T> *I, const Work &w, int level, int color, int lbx,
                                              double *probe, int skip_light) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *st = wstate(w, b.inst);
    // one exit test with no short-circuit, so that the state's fields and the
    // launch's arguments are read in one round trip (a block past the table's end
    // reads instance 0's; level < 0 never holds)
    const int done = st->done, light = st->light;
    if (!b.ok | (done != 0) | ((skip_light != 0) & (light != 0)) | (level < 0)) return;
    const Lv<T, 1> L = gview(a.lv[level]);
    if (L.rb) {
        if (color > 1) return;
        smooth_rb_body<T, ZI, ZT, UPD>(a, st, L, b.t, color, lbx);
    } else {
        smooth_nat_body<T, ZT>(L, b.t, color, ZI, lbx);
    }
    // after the sweep: an atomic ahead of it would stop the per-plane tables
    // from being read through the scalar cache
    if (probe && b.t == 0 && threadIdx.x == 0 && (L.rb ? color < 2 : true)) {
        const double n = (double)L.nx * L.ny * L.nz, ns = (double)L.nx * L.ny * (L.sig_hi - L.sig_lo);
        double by = sizeof(T) * (0.5 * n + 0.5 * ns + 0.5 * n);
        if (!ZI) by += sizeof(T) * 0.5 * n;
        if (UPD && a.fold && L.rb) by += 16.0 * n;
        atomicAdd(probe, by);
    }
}

// Two register budgets: the compiler's own, and one that keeps at least 8
// waves per SIMD resident (64 VGPRs); the autotuner picks per level.
template <typename T, int ZI, int ZT, int UPD>
__global__ __launch_bounds__(256) void k_smooth(const Inst<T> *I, Work w, int level, int color, int lbx,
                                                double *probe, int skip_light) {
    smooth_kernel<T, ZI, ZT, UPD>(I, w, level, color, lbx, probe, skip_light);
}

template <typename T, int ZI, int ZT, int UPD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_smooth_w8(
    const Inst<T> *I, Work w, int level, int color, int lbx, double *probe, int skip_light) {
    smooth_kernel<T, ZI, ZT, UPD>(I, w, level, color, lbx, probe, skip_light);
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const Inst<T> *I, Work w, int level) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const int done = wstate(w, b.inst)->done;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    const Lv<T, 1> C = gview(a.lv[level + 1]);
    const T3 t = split3(b.t, C.nx, C.ny);
    const int I0 = t.tx * BX + threadIdx.x;
    const int J0 = t.ty * BY + threadIdx.y;
    if (I0 >= C.nx || J0 >= C.ny) return;
    const Lv<T, 1> F = gview(a.lv[level]);
    const Xv<T> X = xview(a.xf[level]);
    if (F.rb && X.xy == 1) restrict_cell_rbxy(F, C, X, I0, J0, t.tz);
    else restrict_cell(F, C, X, I0, J0, t.tz);
}

// A thread per column of kProZ planes (black cells only on a red/black
// level): every correction is formed, and every corrected cell read, before
// any cell is updated, so the column's loads are all in flight together.
template <int XY, typename T>
__device__ __forceinline__ void prolong_column(const Lv<T, 1> &F, const Lv<T, 1> &C, const Xv<T> &X, int m, int j,
                                               int k0) {
    T v[kProZ], e[kProZ];
    int c[kProZ];
#pragma unroll
    for (int z = 0; z < kProZ; ++z) {
        const int k = min(k0 + z, F.nz - 1);
        const int i = F.rb ? 2 * m + ((1 + j + k) & 1) : m;
        v[z] = prolong_value<XY>(C, X, i, j, k);
        c[z] = cidx(F, i, j, k);
        e[z] = F.e[c[z]];          // read before any store: a store could alias it
    }
#pragma unroll
    for (int z = 0; z < kProZ; ++z)
        if (k0 + z < F.nz) F.e[c[z]] = e[z] + v[z];
}

// Prolongation fused with the red half-sweep after it, on a red/black level:
// the correction touches only black cells, and the black half-sweep that
// follows recomputes every black cell without reading it, so the corrected
// black values are needed by this red half-sweep alone.  A thread per red cell
// corrects its six black neighbours in registers (same operands, same order as
// prolong_column) and updates itself from them (same expression as the red
// half-sweep); nothing but the red cells is stored.
template <int XY, typename T, int ZT>
__device__ __forceinline__ void prolong_red_body(const Lv<T, 1> &F, const Lv<T, 1> &C, const Xv<T> &X, int t,
                                                 int lbx) {
    const int hx = F.nx >> 1;
    const T3 tt = split3r(t, hx, F.ny, lbx);
    const int m = (tt.tx << lbx) + (threadIdx.x & ((1 << lbx) - 1));
    const int j = (tt.ty << (8 - lbx)) + (threadIdx.x >> lbx);
    if (m >= hx || j >= F.ny) return;
    const int half = (F.nx * F.ny * F.nz) >> 1;
    const int plane = F.ny * hx;
    const T FX_AS(1) *eb = F.e + half;                 // black values before the correction
    T FX_AS(1) *er = F.e;
    const int jp = wrap_p(j, F.ny), jm = wrap_m(j, F.ny);
    const int oy0 = (jp - j) * hx, oy1 = (jm - j) * hx;
    // corrected black value at black index c, fine cell (i, jj, kk)
    auto blk = [&](int c, int i, int jj, int kk) { return eb[c] + prolong_value<XY>(C, X, i, jj, kk); };
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = tt.tz * ZT + z;
        if (k >= F.nz) break;
        const int row = k * plane + j * hx;
        const int q = row + m;
        const int i = 2 * m + ((j + k) & 1);
        const int ip = i + 1 == F.nx ? 0 : i + 1, im = i == 0 ? F.nx - 1 : i - 1;
        const bool hs = k >= F.sig_lo && k < F.sig_hi;
        const T rr = F.r[q];
        const T sg = F.sig[hs ? (k - F.sig_lo) * plane + j * hx + m : 0];
        const T ex0 = blk(row + (ip >> 1), ip, j, k), ex1 = blk(row + (im >> 1), im, j, k);
        // one row (ny = 1): the y terms carry a zero coefficient and read the
        // pair's black cell, as the red half-sweep does
        const T ey0 = F.ny > 1 ? blk(q + oy0, i, jp, k) : blk(q, i ^ 1, j, k);
        const T ey1 = F.ny > 1 ? blk(q + oy1, i, jm, k) : blk(q, i ^ 1, j, k);
        const T ez0 = k > 0 ? blk(q - plane, i, j, k - 1) : blk(q, i ^ 1, j, k);
        const T ez1 = k < F.nz - 1 ? blk(q + plane, i, j, k + 1) : blk(q, i ^ 1, j, k);
        const T acc = rb_nb_sum(F, k, ex0, ex1, ey0, ey1, ez0, ez1);
        er[q] = (rr + acc) / (F.dg[k] + (hs ? sg : T(0)));
    }
}

template <typename T, int ZT>
__global__ __launch_bounds__(256) void k_prolong_red(const Inst<T> *I, Work w, int level, int lbx) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const int done = wstate(w, b.inst)->done;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    const Lv<T, 1> F = gview(a.lv[level]);
    if (!F.rb) return;                               // the host fuses only all-red/black levels
    const Lv<T, 1> C = gview(a.lv[level + 1]);
    const Xv<T> X = xview(a.xf[level]);
    if (X.xy == 1) prolong_red_body<1, T, ZT>(F, C, X, b.t, lbx);
    else if (X.xy == 2) prolong_red_body<2, T, ZT>(F, C, X, b.t, lbx);
    else prolong_red_body<0, T, ZT>(F, C, X, b.t, lbx);
}

// Prolongation into a red/black level halved in x and y and paired in z, a thread
// per coarse column of cz planes.  For each coarse plane the thread loads the
// 3 x 3 neighbourhood of its column once and forms the bilinear values at its four
// child columns; every fine plane of its children then combines the values of its
// parent plane and of the neighbour plane named by the z tables, kept in registers
// as the thread marches up.  Each value goes through lint_xy and lint_z with the
// operands of prolong_value, so the corrections are those of prolong_column bit for
// bit; only black children are corrected (the red ones are overwritten by the next
// red half-sweep without being read).
template <typename T>
__device__ __forceinline__ void prolong_cc_interp(const Lv<T, 1> &C, int K, int Im, int I, int Ip, int Jm, int J,
                                                  int Jp, T (&s)[2][2]) {
    const int ii[3] = {Im, I, Ip}, jj[3] = {Jm, J, Jp};
    T v[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) v[b][a] = C.e[cidx(C, ii[a], jj[b], K)];
    const T wx[2] = {T(0.75), T(0.25)}, wy[2] = {T(0.75), T(0.25)};
    T w[2][2];
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int xx = 0; xx < 2; ++xx) w[yy][xx] = wx[xx] * wy[yy];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int ix[2] = {1, dx ? 2 : 0}, jy[2] = {1, dy ? 2 : 0};
            T u[2][2];
#pragma unroll
            for (int yy = 0; yy < 2; ++yy)
#pragma unroll
                for (int xx = 0; xx < 2; ++xx) u[yy][xx] = v[jy[yy]][ix[xx]];
            s[dy][dx] = lint_xy<2, 2>(w, u);
        }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_cc(const Inst<T> *Ia, Work w, int level, int cz) {
    const Blk b = find_block(w);
    const Inst<T> &a = Ia[b.inst];
    const int done = wstate(w, b.inst)->done;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    const Lv<T, 1> C = gview(a.lv[level + 1]);
    const T3 t = split3(b.t, C.nx, C.ny);
    const int I = t.tx * BX + threadIdx.x;
    const int J = t.ty * BY + threadIdx.y;
    if (I >= C.nx || J >= C.ny) return;
    const Lv<T, 1> F = gview(a.lv[level]);
    const Xv<T> X = xview(a.xf[level]);
    const int Im = wrap_m(I, C.nx), Ip = wrap_p(I, C.nx), Jm = wrap_m(J, C.ny), Jp = wrap_p(J, C.ny);
    const int K0 = t.tz * cz, K1 = min(K0 + cz, C.nz);
    T sp[2][2], sc[2][2], sn[2][2];
    prolong_cc_interp(C, K0 > 0 ? K0 - 1 : K0, Im, I, Ip, Jm, J, Jp, sp);
    prolong_cc_interp(C, K0, Im, I, Ip, Jm, J, Jp, sc);
    for (int K = K0; K < K1; ++K) {
        prolong_cc_interp(C, K + 1 < C.nz ? K + 1 : K, Im, I, Ip, Jm, J, Jp, sn);
        int c[4];
        T e[4], v[4];
        int nf = 0;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz) {
            const int k = 2 * K + dz;
            if (k >= F.nz) break;
            const int kb = X.pkb[k];
            const T wa = X.pwa[k], wb = kb >= 0 ? X.pwb[k] : T(0);
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                // the black child of this row on plane k: (dx + dy + k) odd
                const int dx = (1 + dy + k) & 1;
                const T s0 = sc[dy][dx];
                const T s1 = kb < 0 ? s0 : (kb < K ? sp[dy][dx] : sn[dy][dx]);
                const T val = lint_z(wa, s0, wb, s1);
                const int q = 2 * dz + dy;
                c[q] = cidx(F, 2 * I + dx, 2 * J + dy, k);
                e[q] = F.e[c[q]];
                v[q] = val;
            }
            nf = 2 * dz + 2;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < nf) F.e[c[q]] = e[q] + v[q];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                sp[dy][dx] = sc[dy][dx];
                sc[dy][dx] = sn[dy][dx];
            }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong(const Inst<T> *I, Work w, int level) {
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const int done = wstate(w, b.inst)->done;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    const Lv<T, 1> F = gview(a.lv[level]);
    const int nxe = F.rb ? F.nx >> 1 : F.nx;      // black cells per row on a red/black level
    const T3 t = split3(b.t, nxe, F.ny);
    const int m = t.tx * BX + threadIdx.x;
    const int j = t.ty * BY + threadIdx.y;
    if (m >= nxe || j >= F.ny) return;
    const Lv<T, 1> C = gview(a.lv[level + 1]);
    const Xv<T> X = xview(a.xf[level]);
    if (X.xy == 1) prolong_column<1>(F, C, X, m, j, t.tz * kProZ);
    else if (X.xy == 2) prolong_column<2>(F, C, X, m, j, t.tz * kProZ);
    else prolong_column<0>(F, C, X, m, j, t.tz * kProZ);
}

// --------------------------------------- temporal blocking below the finest level
// On a red/black level small enough for its launches to be latency-bound, the
// pre-smoothing sweeps and the restriction are one launch, and so are the
// prolongation and the post-smoothing sweeps.  A block owns a tile of kTbT x kTbT
// columns of every plane and keeps a box of the tile plus a kTbH-cell ring of
// e in LDS, kTbQ threads per box column (each a share of its planes).  Each
// half-sweep over the box leaves one ring fewer valid, so nu sweeps need a ring of
// 2 nu cells (nu <= 2 here), recomputed by every block that needs it.  Every value
// goes through the expressions of the separate launches (the zero-start value,
// rb_nb_sum and the division by the same divisor; the lateral and z interpolants of
// prolong_value; the restriction's residual and sums in the same order) with the same
// operands, so the results are theirs bit for bit.
//   pre:  nu zero-start sweeps on e (red then black), the restriction of the
//         red children's residuals and of sigma into the coarse level, and the
//         tile's black values stored in ealt (the only ones the post launch reads);
//   post: black values of ealt plus the interpolated correction, nu sweeps (the
//         first red half-sweep reads the corrected black values, as the fused
//         prolongation does), and both colours of the tile stored in e.
// The post launch reads ealt around its tile while other blocks store e, so the
// two arrays keep the launches free of races.  Every global value a thread needs
// (its cells' r and sigma, the coarse values it interpolates, its black values) is
// loaded at the start in one round trip; the per-plane tables go to LDS, and the
// sweeps then touch LDS alone.
static_assert(kTbW * kTbW == 256, "a 256-column box");
constexpr int kTbCW = kTbW / 2 + 2;           // coarse columns under a box, with the interpolation's neighbours
// Q threads per box column (256 Q per block), each with ZQ cells of one colour.
template <int Q>
struct TbShape {
    static constexpr int threads = Q * kTbW * kTbW;
    static constexpr int zq = (kTbMaxNz / 2 + Q - 1) / Q;
};
// Threads per column: four where the registers allow (FP32); in FP64 three for the
// pre-smoothing and two for the post-smoothing, whose half-sweeps form two cells at a
// time, so that neither spills registers.
template <typename T> struct TbCfg {
    static constexpr int pre_q = sizeof(T) == 8 ? 3 : 4, post_q = sizeof(T) == 8 ? 2 : 4;
    static constexpr int post_g = sizeof(T) == 8 ? 2 : TbShape<post_q>::zq;
};

struct TbCol {
    int gi, gj, ring, q0;                  // global column, its ring (0 inside the tile), pair index in a plane
    int bx, by, tx, ty;                    // box column, tile
    int z0;                                // first colour-cell index of this thread's share of the column
};

template <int ZQ, typename V>
__device__ __forceinline__ TbCol tb_col(const V &L, int t) {
    const int ntx = L.nx / kTbT;
    TbCol c;
    c.ty = t / ntx;
    c.tx = t - c.ty * ntx;
    c.bx = threadIdx.x & (kTbW - 1);
    c.by = (threadIdx.x >> 4) & (kTbW - 1);
    c.z0 = (threadIdx.x >> 8) * ZQ;       // threads 256 q .. 256 q + 255 take share q
    int gi = c.tx * kTbT - kTbH + c.bx, gj = c.ty * kTbT - kTbH + c.by;
    gi += gi < 0 ? L.nx : (gi >= L.nx ? -L.nx : 0);
    gj += gj < 0 ? L.ny : (gj >= L.ny ? -L.ny : 0);
    c.gi = gi;
    c.gj = gj;
    const int rx = c.bx < kTbH ? kTbH - c.bx : (c.bx >= kTbH + kTbT ? c.bx - (kTbH + kTbT - 1) : 0);
    const int ry = c.by < kTbH ? kTbH - c.by : (c.by >= kTbH + kTbT ? c.by - (kTbH + kTbT - 1) : 0);
    c.ring = rx > ry ? rx : ry;
    c.q0 = gj * (L.nx >> 1) + (gi >> 1);
    return c;
}

// Plane of this thread's z-th cell of colour col (planes past the top are clamped: their
// values are formed but never stored).
__device__ __forceinline__ int tb_k(const TbCol &c, int col, int z, int nz) {
    return min(2 * (c.z0 + z) + ((col + c.bx + c.by) & 1), nz - 1);
}
__device__ __forceinline__ bool tb_in(const TbCol &c, int col, int z, int nz) {
    return 2 * (c.z0 + z) + ((col + c.bx + c.by) & 1) < nz;
}
__device__ __forceinline__ int tb_l(const TbCol &c, int k) { return (k * kTbW + c.by) * kTbW + c.bx; }

// LDS after the box: the level's per-plane tables (cxy, czm, czp, dg), the z weights
// and parent planes of its prolongation (pwa, pwb, pka, pkb).
template <typename T>
struct TbTab {
    Lv<T, 3> L;                            // the level with its tables in LDS (no arrays)
    const T FX_AS(3) *pwa, *pwb;
    const int FX_AS(3) *pka, *pkb;
};

template <typename T>
__device__ __forceinline__ TbTab<T> tb_tables(const Lv<T, 1> &L, const Xv<T> &X, T FX_AS(3) *box, int with_z) {
    T FX_AS(3) *tab = box + L.nz * kTbW * kTbW;
    int FX_AS(3) *itab = (int FX_AS(3) *)(tab + 6 * L.nz);
    for (int c = threadIdx.x; c < L.nz; c += blockDim.x) {
        tab[c] = L.cxy[c];
        tab[L.nz + c] = L.czm[c];
        tab[2 * L.nz + c] = L.czp[c];
        tab[3 * L.nz + c] = L.dg[c];
        if (with_z) {
            tab[4 * L.nz + c] = X.pwa[c];
            tab[5 * L.nz + c] = X.pwb[c];
            itab[c] = X.pka[c];
            itab[L.nz + c] = X.pkb[c];
        }
    }
    TbTab<T> t;
    t.L.nx = L.nx; t.L.ny = L.ny; t.L.nz = L.nz; t.L.rb = L.rb;
    t.L.cxy = tab; t.L.czm = tab + L.nz; t.L.czp = tab + 2 * L.nz; t.L.dg = tab + 3 * L.nz;
    t.L.e = nullptr; t.L.r = nullptr; t.L.sig = nullptr;
    t.L.sig_lo = L.sig_lo; t.L.sig_hi = L.sig_hi;
    t.pwa = tab + 4 * L.nz; t.pwb = tab + 5 * L.nz;
    t.pka = itab; t.pkb = itab + L.nz;
    return t;
}

// This thread's cells of colour col: right-hand sides and sigma (0 off the
// semiconductor planes), loaded without conditions.
template <typename T, int ZQ>
__device__ __forceinline__ void tb_col_rs(const Lv<T, 1> &L, const TbCol &c, int col, T (&rr)[ZQ], T (&sg)[ZQ]) {
    const int plane = L.ny * (L.nx >> 1);
    const int half = plane * L.nz;
    const int hsz = plane * (L.sig_hi - L.sig_lo);
    const T FX_AS(1) *rs = L.r + (col ? half : 0);
    const T FX_AS(1) *ss = L.sig + (col ? hsz : 0);
#pragma unroll
    for (int z = 0; z < ZQ; ++z) {
        const int k = tb_k(c, col, z, L.nz);
        const bool hs = k >= L.sig_lo && k < L.sig_hi;
        rr[z] = rs[k * plane + c.q0];
        const T v = ss[hs ? (k - L.sig_lo) * plane + c.q0 : 0];
        sg[z] = hs ? v : T(0);
    }
}
// The divisors, as the separate half-sweeps form them (tables in LDS hold the same values).
template <typename T, int ZQ>
__device__ __forceinline__ void tb_col_den(const Lv<T, 3> &Lt, const TbCol &c, int col, T (&sg)[ZQ]) {
#pragma unroll
    for (int z = 0; z < ZQ; ++z) {
        const int k = tb_k(c, col, z, Lt.nz);
        const bool hs = k >= Lt.sig_lo && k < Lt.sig_hi;
        sg[z] = Lt.dg[k] + (hs ? sg[z] : T(0));
    }
}

// One half-sweep of colour col over the box columns within ring R (ZI: from a zero
// start).  The box origin is even in x and y, so a box cell's colour is the parity of
// its box coordinates and plane, and its red/black partner (the other cell of its
// storage pair, the stand-in operand of the zero-coefficient z terms) is box x ^ 1.
// Cells of one colour are not neighbours, so the new values of a group of G cells are
// formed before any of them is stored (G bounds the registers held by the operands).
template <typename T, int ZI, int ZQ, int G = ZQ>
__device__ __forceinline__ void tb_half(const Lv<T, 3> &Lt, const TbCol &c, T FX_AS(3) *box, int col, int R,
                                        const T (&rr)[ZQ], const T (&den)[ZQ]) {
    if (c.ring <= R) {
#pragma unroll
        for (int z0 = 0; z0 < ZQ; z0 += G) {
            T v[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int z = z0 + g < ZQ ? z0 + g : ZQ - 1;
                const int k = tb_k(c, col, z, Lt.nz);
                const int l = tb_l(c, k);
                T acc = 0;
                if (!ZI) {
                    const T ez0 = k > 0 ? box[l - kTbW * kTbW] : box[l ^ 1];
                    const T ez1 = k < Lt.nz - 1 ? box[l + kTbW * kTbW] : box[l ^ 1];
                    acc = rb_nb_sum(Lt, k, box[l + 1], box[l - 1], box[l + kTbW], box[l - kTbW], ez0, ez1);
                }
                v[g] = (rr[z] + acc) / den[z];
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (z0 + g < ZQ && tb_in(c, col, z0 + g, Lt.nz)) box[tb_l(c, tb_k(c, col, z0 + g, Lt.nz))] = v[g];
        }
    }
    __syncthreads();
}

// Restriction of coarse cell (I, J, K) from the box (restrict_cell_rbxy's loads and
// arithmetic; the box holds e, the tile's red cells and their black neighbours valid).
template <typename T, typename X>
__device__ __forceinline__ void tb_restrict_cell(const Lv<T, 1> &F, const Lv<T, 1> &C, const X &Xf, const T FX_AS(3) *box,
                                                 int I, int J, int K, int bx0, int by0) {
    const int ks = Xf.cks[K], cnt = Xf.ccnt[K];
    T sg[2][2][2], rv[2][2], ev[2][2], nb[2][2][6], cx[2], czm[2], czp[2], dg[2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        const int k = ks + (dz < cnt ? dz : 0);
        const bool hs = has_sig(F, k);
        const int km = k > 0 ? k - 1 : k, kp = k < F.nz - 1 ? k + 1 : k;
        cx[dz] = F.cxy[k];
        czm[dz] = F.czm[k];
        czp[dz] = F.czp[k];
        dg[dz] = F.dg[k];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int j = 2 * J + dy;
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int i = 2 * I + dx;
                const T FX_AS(1) *sp = hs ? F.sig + sidx(F, i, j, k) : F.r + cidx(F, i, j, k);
                sg[dz][dy][dx] = *sp;
            }
            const int dxr = (dy + k) & 1;
            const int i = 2 * I + dxr;
            rv[dz][dy] = F.r[cidx(F, i, j, k)];
            const int l = (k * kTbW + by0 + dy) * kTbW + bx0 + dxr;
            ev[dz][dy] = box[l];
            nb[dz][dy][0] = box[l + 1];
            nb[dz][dy][1] = box[l - 1];
            nb[dz][dy][2] = box[l + kTbW];
            nb[dz][dy][3] = box[l - kTbW];
            nb[dz][dy][4] = box[l + (km - k) * kTbW * kTbW];
            nb[dz][dy][5] = box[l + (kp - k) * kTbW * kTbW];
        }
    }
    double sr = 0.0, ss = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        if (dz >= cnt) break;
        const int k = ks + dz;
        const double wz = (double)Xf.fthick[k] / (double)Xf.cthick[K];
        const bool hs = has_sig(F, k);
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const T sgc = hs ? sg[dz][dy][dx] : T(0);
                ss += wz * (double)sgc;
                if (dx != ((dy + k) & 1)) continue;
                T nbs = 0;
                nbs += cx[dz] * (nb[dz][dy][0] + nb[dz][dy][1]);
                nbs += cx[dz] * (nb[dz][dy][2] + nb[dz][dy][3]);
                if (k > 0) nbs += czm[dz] * nb[dz][dy][4];
                if (k < F.nz - 1) nbs += czp[dz] * nb[dz][dy][5];
                const T res = rv[dz][dy] - ((dg[dz] + sgc) * ev[dz][dy] - nbs);
                sr += wz * (double)res;
            }
        }
    }
    C.r[cidx(C, I, J, K)] = (T)(sr * 0.25);
    if (has_sig(C, K)) C.sig[sidx(C, I, J, K)] = (T)(ss * 0.25);
}

template <typename T>
__global__ __launch_bounds__(TbShape<TbCfg<T>::pre_q>::threads) void k_pre_tb(const Inst<T> *I, Work w, int level,
                                                                                int nu) {
    constexpr int ZQ = TbShape<TbCfg<T>::pre_q>::zq;
    extern __shared__ double tb_raw[];
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *st = wstate(w, b.inst);
    const int done = st->done, light = st->light;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    if (light) nu = 1;                         // the sweeps after the first are left out
    const Lv<T, 1> L = gview(a.lv[level]);
    const Xv<T> X = xview(a.xf[level]);
    T FX_AS(3) *box = asp<3>((T *)tb_raw);
    const TbCol c = tb_col<ZQ>(L, b.t);
    T rr0[ZQ], den0[ZQ], rr1[ZQ], den1[ZQ];
    tb_col_rs(L, c, 0, rr0, den0);
    tb_col_rs(L, c, 1, rr1, den1);
    const TbTab<T> tt = tb_tables(L, X, box, 0);
    __syncthreads();                               // tables
    tb_col_den(tt.L, c, 0, den0);
    tb_col_den(tt.L, c, 1, den1);
    tb_half<T, 1>(tt.L, c, box, 0, 2 * nu, rr0, den0);
    tb_half<T, 0>(tt.L, c, box, 1, 2 * nu - 1, rr1, den1);
    if (nu > 1) {
        tb_half<T, 0>(tt.L, c, box, 0, 2, rr0, den0);
        tb_half<T, 0>(tt.L, c, box, 1, 1, rr1, den1);
    }
    // the tile's black values for the post launch
    if (c.ring == 0) {
        const int plane = L.ny * (L.nx >> 1), half = plane * L.nz;
        T FX_AS(1) *ealt = asp<1>(a.lv[level].ealt);
#pragma unroll
        for (int z = 0; z < ZQ; ++z) {
            const int k = tb_k(c, 1, z, L.nz);
            if (tb_in(c, 1, z, L.nz)) ealt[half + k * plane + c.q0] = box[tb_l(c, k)];
        }
    }
    // restriction: kTbT/2 x kTbT/2 coarse columns of the tile, every coarse plane
    const Lv<T, 1> C = gview(a.lv[level + 1]);
    constexpr int kC = kTbT / 2;
    for (int u = threadIdx.x; u < kC * kC * C.nz; u += blockDim.x) {
        const int K = u / (kC * kC), cc = u - K * kC * kC;
        const int cj = cc / kC, ci = cc - cj * kC;
        tb_restrict_cell(L, C, X, box, c.tx * kC + ci, c.ty * kC + cj, K, kTbH + 2 * ci, kTbH + 2 * cj);
    }
}

template <typename T>
__global__ __launch_bounds__(TbShape<TbCfg<T>::post_q>::threads) void k_post_tb(const Inst<T> *I, Work w, int level,
                                                                                  int nu) {
    constexpr int ZQ = TbShape<TbCfg<T>::post_q>::zq;
    constexpr int G = TbCfg<T>::post_g;
    extern __shared__ double tb_raw[];
    const Blk b = find_block(w);
    const Inst<T> &a = I[b.inst];
    const GState *st = wstate(w, b.inst);
    const int done = st->done, light = st->light;
    if (!b.ok | (done != 0) | (level < 0)) return;  // one exit test: see smooth_kernel
    if (light) nu = 1;                         // one sweep: the fused prolongation's and the black after it
    const Lv<T, 1> F = gview(a.lv[level]);
    const Lv<T, 1> C = gview(a.lv[level + 1]);
    const Xv<T> X = xview(a.xf[level]);
    T FX_AS(3) *box = asp<3>((T *)tb_raw);
    const TbCol c = tb_col<ZQ>(F, b.t);
    const int plane = F.ny * (F.nx >> 1), half = plane * F.nz;
    const bool corr = c.ring <= 2 * nu;
    // The coarse values under the box (kTbCW x kTbCW coarse columns, every coarse plane),
    // one load each, into the box's planes above those the interpolants take; then this
    // thread's black values.  Box column bx lies over coarse box column
    // (tile x - kTbH + bx) / 2 - (tile x kTbT/2 - kTbH/2 - 1), its x neighbour one further
    // on the side of its parity, as prolong_value takes them (wrapping included).
    T FX_AS(3) *cb = box + C.nz * kTbW * kTbW;
    const int cx0 = c.tx * (kTbT / 2) - kTbH / 2 - 1, cy0 = c.ty * (kTbT / 2) - kTbH / 2 - 1;
    for (int u = threadIdx.x; u < kTbCW * kTbCW * C.nz; u += blockDim.x) {
        const int K = u / (kTbCW * kTbCW), rem = u - K * kTbCW * kTbCW;
        const int cj = rem / kTbCW, ci = rem - cj * kTbCW;
        int I = cx0 + ci, J = cy0 + cj;
        I += I < 0 ? C.nx : (I >= C.nx ? -C.nx : 0);
        J += J < 0 ? C.ny : (J >= C.ny ? -C.ny : 0);
        cb[u] = C.e[cidx(C, I, J, K)];
    }
    T ebv[ZQ];
    const T FX_AS(1) *eb = asp<1>(a.lv[level].ealt) + half;
#pragma unroll
    for (int z = 0; z < ZQ; ++z) ebv[z] = eb[tb_k(c, 1, z, F.nz) * plane + c.q0];
    const TbTab<T> tt = tb_tables(F, X, box, 1);
    __syncthreads();                               // coarse values, tables
    // the lateral interpolants (prolong_value's weights and operands), parked in the box
    // for the z interpolation
    if (corr) {
        const T wx[2] = {T(0.75), T(0.25)}, wy[2] = {T(0.75), T(0.25)};
        T wgt[2][2];
#pragma unroll
        for (int yy = 0; yy < 2; ++yy)
#pragma unroll
            for (int xx = 0; xx < 2; ++xx) wgt[yy][xx] = wx[xx] * wy[yy];
        const int gu = c.tx * kTbT - kTbH + c.bx, gv = c.ty * kTbT - kTbH + c.by;   // unwrapped
        const int ci[2] = {(gu >> 1) - cx0, (gu >> 1) - cx0 + ((gu & 1) ? 1 : -1)};
        const int cj[2] = {(gv >> 1) - cy0, (gv >> 1) - cy0 + ((gv & 1) ? 1 : -1)};
        T sv[ZQ];
#pragma unroll
        for (int q = 0; q < ZQ; ++q) {
            const int K = min(c.z0 + q, C.nz - 1);
            T v[2][2];
#pragma unroll
            for (int yy = 0; yy < 2; ++yy)
#pragma unroll
                for (int xx = 0; xx < 2; ++xx) v[yy][xx] = cb[(K * kTbCW + cj[yy]) * kTbCW + ci[xx]];
            sv[q] = lint_xy<2, 2>(wgt, v);
        }
#pragma unroll
        for (int q = 0; q < ZQ; ++q)
            if (c.z0 + q < C.nz) box[tb_l(c, c.z0 + q)] = sv[q];
    }
    __syncthreads();                               // interpolants
    // black values with the correction: eb + lint_z of the parent and neighbour planes
    T vb[ZQ];
    if (corr) {
#pragma unroll
        for (int z = 0; z < ZQ; ++z) {
            const int k = tb_k(c, 1, z, F.nz);
            const int ka = tt.pka[k], kb = tt.pkb[k];
            const T s0 = box[tb_l(c, ka)];
            const T s1 = box[tb_l(c, kb >= 0 ? kb : ka)];
            vb[z] = ebv[z] + lint_z(tt.pwa[k], s0, kb >= 0 ? tt.pwb[k] : T(0), s1);
        }
    }
    __syncthreads();                               // interpolants read
    if (corr) {
#pragma unroll
        for (int z = 0; z < ZQ; ++z)
            if (tb_in(c, 1, z, F.nz)) box[tb_l(c, tb_k(c, 1, z, F.nz))] = vb[z];
    }
    // this thread's cells' r and sigma (loaded after the correction, which needs the registers)
    T rr0[ZQ], den0[ZQ], rr1[ZQ], den1[ZQ];
    tb_col_rs(F, c, 0, rr0, den0);
    tb_col_rs(F, c, 1, rr1, den1);
    tb_col_den(tt.L, c, 0, den0);
    tb_col_den(tt.L, c, 1, den1);
    __syncthreads();
    tb_half<T, 0, ZQ, G>(tt.L, c, box, 0, 2 * nu - 1, rr0, den0);
    tb_half<T, 0, ZQ, G>(tt.L, c, box, 1, 2 * nu - 2, rr1, den1);
    if (nu > 1) {
        tb_half<T, 0, ZQ, G>(tt.L, c, box, 0, 1, rr0, den0);
        tb_half<T, 0, ZQ, G>(tt.L, c, box, 1, 0, rr1, den1);
    }
    if (c.ring == 0) {
#pragma unroll
        for (int col = 0; col < 2; ++col)
#pragma unroll
            for (int z = 0; z < ZQ; ++z) {
                const int k = tb_k(c, col, z, F.nz);
                if (tb_in(c, col, z, F.nz)) F.e[(col ? half : 0) + k * plane + c.q0] = box[tb_l(c, k)];
            }
    }
}

// --------------------------------------------- coarse levels in one workgroup
// Quotient q / d for 0 <= q < 2^31 and 1 <= d < 2^16 without an integer division:
// (q + 1/2) / d lies at least 1/(2d) >= 2^-17 from the next integer, while the
// product with the rounded reciprocal is off by at most 2^-52 q/d < 2^-21.
struct FDiv {
    int d;
    double inv;
};
__device__ __forceinline__ FDiv fdiv_of(int d) { return {d, 1.0 / (double)d}; }
__device__ __forceinline__ int fquo(int q, const FDiv &f) { return (int)(((double)q + 0.5) * f.inv); }

// (i, j, k) of natural index c on an nx x ny x nz level
struct Split3 {
    FDiv fx, fy;
};
__device__ __forceinline__ void split_c(int c, const Split3 &s, int &i, int &j, int &k) {
    const int row = fquo(c, s.fx);
    i = c - row * s.fx.d;
    k = fquo(row, s.fy);
    j = row - k * s.fy.d;
}

// A coarse-kernel phase: the whole workgroup strides over the level's cells,
// and a workgroup barrier separates it from the next phase.
template <typename V>
__device__ void smooth_color(const V &L, int color, int zero_init) {
    using T = typename V::value_type;
    const int st = (int)blockDim.x;
    if (L.rb) {
        // gs_cell on split storage with the indices written out: the cell's pair q, its
        // x neighbours at the pairs of i +- 1 in its row, the others at pair q of the
        // neighbouring row or plane (the other colour's array throughout); the sum in
        // nb_sum's order, the divisor as diag_of forms it
        const int hx = L.nx >> 1;
        const int plane = hx * L.ny;
        const int n = plane * L.nz;
        const int hsz = plane * (L.sig_hi - L.sig_lo);
        T FX_AS(3) *es = L.e + (color ? n : 0);
        const T FX_AS(3) *eo = L.e + (color ? 0 : n);
        const T FX_AS(3) *rs = L.r + (color ? n : 0);
        const T FX_AS(3) *ss = L.sig + (color ? hsz : 0);
        const Split3 sp{fdiv_of(hx), fdiv_of(L.ny)};
        for (int q = threadIdx.x; q < n; q += st) {
            int m, j, k;
            split_c(q, sp, m, j, k);
            T d = L.dg[k];
            if (k >= L.sig_lo && k < L.sig_hi) d += ss[q - L.sig_lo * plane];
            if (zero_init) {
                es[q] = rs[q] / d;
                continue;
            }
            const int i = 2 * m + ((color + j + k) & 1);
            const int row = q - m;
            const int ip = i + 1 == L.nx ? 0 : i + 1, im = i == 0 ? L.nx - 1 : i - 1;
            T s = 0;
            const T cx = L.cxy[k];
            s += cx * (eo[row + (ip >> 1)] + eo[row + (im >> 1)]);
            if (L.ny > 1) s += cx * (eo[q + (wrap_p(j, L.ny) - j) * hx] + eo[q + (wrap_m(j, L.ny) - j) * hx]);
            if (k > 0) s += L.czm[k] * eo[q - plane];
            if (k < L.nz - 1) s += L.czp[k] * eo[q + plane];
            es[q] = (rs[q] + s) / d;
        }
    } else {
        const int n = L.nx * L.ny * L.nz;
        const Split3 sp{fdiv_of(L.nx), fdiv_of(L.ny)};
        for (int c = threadIdx.x; c < n; c += st) {
            int i, j, k;
            split_c(c, sp, i, j, k);
            if (nat_color(L, i, j, k) == color) gs_cell(L, i, j, k, zero_init);
            else if (zero_init) L.e[cidx(L, i, j, k)] = T(0);
        }
    }
}

// One full Gauss-Seidel sweep (2 colours on split levels, 4 otherwise).
template <typename V>
__device__ void smooth_sweep(const V &L, int zero_init) {
    const int ncol = L.rb ? 2 : 4;
    for (int c = 0; c < ncol; ++c) {
        smooth_color(L, c, zero_init && c == 0);
        __syncthreads();
    }
}

// Restriction into level C and prolongation from it, as one phase each.
// On a red/black level halved in x and y both take the global kernels' forms (every load
// of a coarse cell's children before its arithmetic; black cells alone corrected), which
// compute what restrict_cell and prolong_cell compute, in the same order.
template <typename T, typename X_>
__device__ void restrict_phase(const Lv<T, 3> &L, const Lv<T, 3> &C, const X_ &X) {
    const int n = C.nx * C.ny * C.nz;
    const Split3 sp{fdiv_of(C.nx), fdiv_of(C.ny)};
    const bool rbxy = L.rb && X.xy == 1;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        int I0, J0, K0;
        split_c(c, sp, I0, J0, K0);
        if (rbxy) restrict_cell_rbxy(L, C, X, I0, J0, K0);
        else restrict_cell(L, C, X, I0, J0, K0);
    }
    __syncthreads();
}
template <typename T, typename X_>
__device__ void prolong_phase(const Lv<T, 3> &L, const Lv<T, 3> &C, const X_ &X) {
    if (L.rb) {
        const int hx = L.nx >> 1;
        const int n = hx * L.ny * L.nz;
        T FX_AS(3) *eb = L.e + n;
        const Split3 sp{fdiv_of(hx), fdiv_of(L.ny)};
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            int m, j, k;
            split_c(q, sp, m, j, k);
            const int i = 2 * m + ((1 + j + k) & 1);
            const T v = X.xy == 1 ? prolong_value<1>(C, X, i, j, k)
                        : X.xy == 2 ? prolong_value<2>(C, X, i, j, k) : prolong_value<0>(C, X, i, j, k);
            eb[q] += v;
        }
    } else {
        const int n = L.nx * L.ny * L.nz;
        const Split3 sp{fdiv_of(L.nx), fdiv_of(L.ny)};
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            int i, j, k;
            split_c(c, sp, i, j, k);
            prolong_cell(L, C, X, i, j, k);
        }
    }
    __syncthreads();
}

// Dot product over a whole workgroup, accumulated in double in a fixed order
// (deterministic); every thread returns the total.
template <typename P>
__device__ double block_dot(P x, P y, int n, double FX_AS(3) *red) {
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int c = tid; c < n; c += blockDim.x) s += (double)x[c] * (double)y[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
    __syncthreads();
    return t;
}

// Bottom solve on the coarsest level: conjugate gradients on the symmetric
// positive definite (L + diag sigma) e = r from e = 0, until the residual has
// dropped by sqrt(tol2) or after iters steps.  r is overwritten by the
// residual.  Unlike a fixed number of Gauss-Seidel sweeps this also solves
// coarsest levels that keep many cells in x and y (odd lateral sizes stop the
// x-y coarsening early).
// Sum over the 64 lanes of a wave, formed in lane 0 in a fixed order and
// broadcast (every lane gets the same bits).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return __shfl(v, 0, 64);
}

// The same conjugate gradients for a bottom level of at most 64 cells, run by
// the first wave alone with one cell per lane: the operator's neighbours are
// read from other lanes' registers, the dot products are wave sums, and no
// workgroup barrier is needed inside the iteration.
template <typename T>
__device__ void bottom_cg_wave(const Lv<T, 3> &B, int iters, double tol2) {
    const int n = B.nx * B.ny * B.nz;
    const int c = threadIdx.x;
    const bool on = c < n;
    int i = 0, j = 0, k = 0;
    if (on) {
        const Split3 sp{fdiv_of(B.nx), fdiv_of(B.ny)};
        split_c(c, sp, i, j, k);
    }
    // neighbour lanes (natural order) and coefficients; absent neighbours weigh 0
    int nl[6];
    double w[6];
    const double cx = on ? (double)B.cxy[k] : 0.0;
    nl[0] = (k * B.ny + j) * B.nx + wrap_p(i, B.nx);
    nl[1] = (k * B.ny + j) * B.nx + wrap_m(i, B.nx);
    w[0] = w[1] = B.nx > 1 ? cx : 0.0;
    nl[2] = (k * B.ny + wrap_p(j, B.ny)) * B.nx + i;
    nl[3] = (k * B.ny + wrap_m(j, B.ny)) * B.nx + i;
    w[2] = w[3] = B.ny > 1 ? cx : 0.0;
    nl[4] = k > 0 ? c - B.nx * B.ny : c;
    w[4] = on && k > 0 ? (double)B.czm[k] : 0.0;
    nl[5] = k < B.nz - 1 ? c + B.nx * B.ny : c;
    w[5] = on && k < B.nz - 1 ? (double)B.czp[k] : 0.0;
    const int ci = on ? cidx(B, i, j, k) : 0;
    const double d = on ? (double)diag_of(B, i, j, k) : 1.0;
    double r = on ? (double)B.r[ci] : 0.0;
    double x = 0.0, p = r;
    double rr = wave_sum(r * r);
    const double stop = tol2 * rr;
    for (int it = 0; it < iters && rr > stop; ++it) {
        double q = d * p;
#pragma unroll
        for (int m = 0; m < 6; ++m) q -= w[m] * __shfl(p, nl[m], 64);
        if (!on) q = 0.0;
        const double pq = wave_sum(p * q);
        if (!(pq > 0.0)) break;
        const double alpha = rr / pq;
        x += alpha * p;
        r -= alpha * q;
        const double rn = wave_sum(r * r);
        const double beta = rn / rr;
        rr = rn;
        p = r + beta * p;
    }
    if (on) {
        B.e[ci] = (T)x;
        B.r[ci] = (T)r;
    }
}

template <typename T>
__device__ void bottom_cg(const Lv<T, 3> &B, T FX_AS(3) *p, T FX_AS(3) *q, double FX_AS(3) *red, int iters,
                          double tol2) {
    const int n = B.nx * B.ny * B.nz;
    if (n <= 64) {
        if (threadIdx.x < 64) bottom_cg_wave(B, iters, tol2);
        __syncthreads();
        return;
    }
    T FX_AS(3) *e = B.e;
    T FX_AS(3) *r = B.r;
    const Split3 sp{fdiv_of(B.nx), fdiv_of(B.ny)};
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        e[c] = T(0);
        p[c] = r[c];
    }
    __syncthreads();
    double rr = block_dot(r, r, n, red);
    const double stop = tol2 * rr;
    for (int it = 0; it < iters && rr > stop; ++it) {
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            int i, j, k;
            split_c(c, sp, i, j, k);
            const int ci = cidx(B, i, j, k);
            q[ci] = diag_of(B, i, j, k) * p[ci] - nb_sum(B, p, i, j, k);
        }
        __syncthreads();
        const double pq = block_dot(p, q, n, red);
        if (!(pq > 0.0)) break;
        const double alpha = rr / pq;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            e[c] += (T)(alpha * (double)p[c]);
            r[c] -= (T)(alpha * (double)q[c]);
        }
        __syncthreads();
        const double rn = block_dot(r, r, n, red);
        const double beta = rn / rr;
        rr = rn;
        for (int c = threadIdx.x; c < n; c += blockDim.x) p[c] = r[c] + (T)(beta * (double)p[c]);
        __syncthreads();
    }
}

constexpr int kCoarseThreads = 1024;

// A block per instance: the V-cycle from level lc down to the coarsest with
// every level's e, r, sigma and coefficient tables resident in LDS.
template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse(const Inst<T> *I, InstState *S) {
    extern __shared__ double lds_raw[];
    const Inst<T> &A = I[blockIdx.x];
    const GState *sta = asp<1>(S + blockIdx.x);
    if (sta->done) return;
    unsigned char FX_AS(3) *lds = asp<3>((unsigned char *)lds_raw);
    const int l0 = A.lc, nl = A.nlev - A.lc;
    auto lvl = [&](int q) {
        const LevelArgs<T> &G = A.lv[l0 + q];
        Lv<T, 3> L;
        L.nx = G.nx; L.ny = G.ny; L.nz = G.nz; L.rb = G.rb;
        L.sig_lo = G.sig_lo; L.sig_hi = G.sig_hi;
        L.e = (T FX_AS(3) *)(lds + A.off_e[q]);
        L.r = (T FX_AS(3) *)(lds + A.off_r[q]);
        L.sig = (T FX_AS(3) *)(lds + A.off_s[q]);
        T FX_AS(3) *tab = (T FX_AS(3) *)(lds + A.off_t[q]);
        L.cxy = tab;
        L.czm = tab + L.nz;
        L.czp = tab + 2 * L.nz;
        L.dg = tab + 3 * L.nz;
        return L;
    };
    // transfer tables between levels q and q + 1 in LDS
    auto xlds = [&](int q) {
        const int nf = A.lv[l0 + q].nz, nc = A.lv[l0 + q + 1].nz;
        int FX_AS(3) *ib = (int FX_AS(3) *)(lds + A.off_x[q]);
        Xv<T, 3> X;
        X.cks = ib;
        X.ccnt = ib + nc;
        X.cthick = ib + 2 * nc;
        X.fthick = ib + 3 * nc;
        X.pka = ib + 3 * nc + nf;
        X.pkb = ib + 3 * nc + 2 * nf;
        const T FX_AS(3) *wb =
            (const T FX_AS(3) *)(lds + ((A.off_x[q] + (3 * nc + 3 * nf) * (int)sizeof(int) + 15) & ~15));
        X.pwa = wb;
        X.pwb = wb + nf;
        X.xy = A.xf[l0 + q].xy;
        return X;
    };
    // Copy into LDS: the top level's r and sigma (all threads), one level's per-plane
    // coefficient tables and one level pair's transfer tables per wave.  Every load of the
    // first pass is issued before the first LDS store, so the copy costs one round trip to
    // memory; the later passes (levels with more than 64 planes, more than 8 levels, more
    // than 8 values per thread) follow.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    constexpr int kU = 8;
    const Lv<T, 1> G0 = gview(A.lv[l0]);
    const Lv<T, 3> L0 = lvl(0);
    const int n0 = G0.nx * G0.ny * G0.nz;
    const int ns0 = G0.nx * G0.ny * (G0.sig_hi - G0.sig_lo);
    T v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int c = threadIdx.x + u * blockDim.x;
        v[u] = c < n0 ? G0.r[c] : (c < n0 + ns0 ? G0.sig[c - n0] : T(0));
    }
    const bool tq = wave < nl, xq = wave + 1 < nl;
    T tv[4] = {T(0), T(0), T(0), T(0)};
    int tnz = 0;
    if (tq) {
        const Lv<T, 1> G = gview(A.lv[l0 + wave]);
        tnz = G.nz;
        if (lane < tnz) { tv[0] = G.cxy[lane]; tv[1] = G.czm[lane]; tv[2] = G.czp[lane]; tv[3] = G.dg[lane]; }
    }
    int xc[3] = {0, 0, 0}, xf[3] = {0, 0, 0};
    T xw[2] = {T(0), T(0)};
    int xnf = 0, xnc = 0;
    if (xq) {
        const Xv<T> G = xview(A.xf[l0 + wave]);
        xnf = A.lv[l0 + wave].nz;
        xnc = A.lv[l0 + wave + 1].nz;
        if (lane < xnc) { xc[0] = G.cks[lane]; xc[1] = G.ccnt[lane]; xc[2] = G.cthick[lane]; }
        if (lane < xnf) {
            xf[0] = G.fthick[lane]; xf[1] = G.pka[lane]; xf[2] = G.pkb[lane];
            xw[0] = G.pwa[lane]; xw[1] = G.pwb[lane];
        }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int c = threadIdx.x + u * blockDim.x;
        if (c < n0) L0.r[c] = v[u];
        else if (c < n0 + ns0) L0.sig[c - n0] = v[u];
    }
    if (tq && lane < tnz) {
        T FX_AS(3) *tab = (T FX_AS(3) *)(lds + A.off_t[wave]);
        tab[lane] = tv[0]; tab[tnz + lane] = tv[1]; tab[2 * tnz + lane] = tv[2]; tab[3 * tnz + lane] = tv[3];
    }
    if (xq) {
        const Xv<T, 3> X = xlds(wave);
        int FX_AS(3) *ib = (int FX_AS(3) *)X.cks;
        T FX_AS(3) *wb = (T FX_AS(3) *)X.pwa;
        if (lane < xnc) { ib[lane] = xc[0]; ib[xnc + lane] = xc[1]; ib[2 * xnc + lane] = xc[2]; }
        if (lane < xnf) {
            ib[3 * xnc + lane] = xf[0]; ib[3 * xnc + xnf + lane] = xf[1]; ib[3 * xnc + 2 * xnf + lane] = xf[2];
            wb[lane] = xw[0]; wb[xnf + lane] = xw[1];
        }
    }
    for (int c = threadIdx.x + kU * blockDim.x; c < n0 + ns0; c += blockDim.x) {
        if (c < n0) L0.r[c] = G0.r[c];
        else L0.sig[c - n0] = G0.sig[c - n0];
    }
    for (int q = wave; q < nl; q += nwave) {
        const Lv<T, 1> G = gview(A.lv[l0 + q]);
        T FX_AS(3) *tab = (T FX_AS(3) *)(lds + A.off_t[q]);
        for (int c = (q == wave ? 64 : 0) + lane; c < G.nz; c += 64) {
            tab[c] = G.cxy[c];
            tab[G.nz + c] = G.czm[c];
            tab[2 * G.nz + c] = G.czp[c];
            tab[3 * G.nz + c] = G.dg[c];
        }
    }
    for (int q = wave; q + 1 < nl; q += nwave) {
        const Xv<T> G = xview(A.xf[l0 + q]);
        const int nf = A.lv[l0 + q].nz, nc = A.lv[l0 + q + 1].nz;
        const Xv<T, 3> X = xlds(q);
        int FX_AS(3) *ib = (int FX_AS(3) *)X.cks;
        T FX_AS(3) *wb = (T FX_AS(3) *)X.pwa;
        const int c0 = q == wave ? 64 : 0;
        for (int c = c0 + lane; c < nc; c += 64) {
            ib[c] = G.cks[c];
            ib[nc + c] = G.ccnt[c];
            ib[2 * nc + c] = G.cthick[c];
        }
        for (int c = c0 + lane; c < nf; c += 64) {
            ib[3 * nc + c] = G.fthick[c];
            ib[3 * nc + nf + c] = G.pka[c];
            ib[3 * nc + 2 * nf + c] = G.pkb[c];
            wb[c] = G.pwa[c];
            wb[nf + c] = G.pwb[c];
        }
    }
    __syncthreads();
    const int light = sta->light;
    const int nu1 = light ? 1 : A.nu1, nu2 = light ? 1 : A.nu2;
    for (int q = 0; q < nl - 1; ++q) {
        const Lv<T, 3> L = lvl(q);
        for (int s = 0; s < nu1; ++s) smooth_sweep(L, s == 0);
        restrict_phase(L, lvl(q + 1), xlds(q));
    }
    bottom_cg<T>(lvl(nl - 1), (T FX_AS(3) *)(lds + A.off_p), (T FX_AS(3) *)(lds + A.off_q),
                 (double FX_AS(3) *)(lds + A.off_red), A.bottom_iters, A.bottom_tol2);
    for (int q = nl - 2; q >= 0; --q) {
        const Lv<T, 3> L = lvl(q);
        prolong_phase(L, lvl(q + 1), xlds(q));
        for (int s = 0; s < nu2; ++s) smooth_sweep(L, 0);
    }
    {
        const Lv<T, 1> G = gview(A.lv[l0]);
        const Lv<T, 3> L0 = lvl(0);
        const int n = G.nx * G.ny * G.nz;
        for (int c = threadIdx.x; c < n; c += blockDim.x) G.e[c] = L0.e[c];
    }
}

// Start of a run (or of one chunk of its schedule): nsteps more time steps.
// first = 0 keeps instances whose solve failed in an earlier chunk parked.
template <typename T>
__global__ void k_run_setup(const Inst<T> *I, int ninst, int nsteps, int has_sched, double dt, int first) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ninst) return;
    GState *s = asp<1>(I[n].st);
    const bool failed = !first && s->status != 0;
    if (first) { s->status = 0; s->max_cycles_step = 0; }
    s->target = s->step + nsteps;
    s->sched_base = s->step;
    s->sched_len = has_sched ? nsteps : 0;
    s->dt = dt;
    s->parked = nsteps == 0 || failed;
    s->adv = 0;
}

template <typename T>
__global__ void k_set_vtop(const Inst<T> *I, int ninst, double v) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < ninst) asp<1>(I[n].st)->v_top = v;
}

__global__ void k_put_state(InstState *dst, InstState v) {
    if (threadIdx.x == 0) *dst = v;
}

__global__ void k_zero32(unsigned *x, size_t n) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) x[c] = 0u;
}

__global__ void k_fill(double *x, size_t n, double v) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) x[c] = v;
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define FX_LAUNCH(kern, w, ...)                                                                            \
    do {                                                                                                   \
        if ((w).total > 0) hipLaunchKernelGGL(kern, grid_of((w).total), dim3(BX, BY), 0, st, __VA_ARGS__); \
    } while (0)

template <typename T>
void launch_tdgl(const Inst<T> *I, const Work &w, int sel, hipStream_t st) {
    FX_LAUNCH(k_tdgl<T>, w, I, w, sel);
}
template <typename T>
void launch_tdgl_corr(const Inst<T> *I, const Work &w, hipStream_t st) {
    FX_LAUNCH(k_tdgl_corr<T>, w, I, w);
}

inline dim3 per_inst(int ninst) { return dim3((ninst + 63) / 64); }

template <typename T>
void launch_qv(const Inst<T> *I, int ninst, int record, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_qv_part<T>, dim3(ninst * kQvBlocks), dim3(256), 0, st, I, record);
    hipLaunchKernelGGL(k_qv_fin<T>, per_inst(ninst), dim3(64), 0, st, I, ninst, record, out);
}

template <typename T>
void launch_flip(const Inst<T> *I, int ninst, hipStream_t st) {
    hipLaunchKernelGGL(k_flip<T>, per_inst(ninst), dim3(64), 0, st, I, ninst);
}

template <typename T>
void launch_begin(const Inst<T> *I, InstState *S, int ninst, int sel, hipStream_t st) {
    hipLaunchKernelGGL(k_begin<T>, per_inst(ninst), dim3(64), 0, st, I, S, ninst, sel);
}

template <typename T>
void launch_extrap(const Inst<T> *I, const Work &w, hipStream_t st) {
    FX_LAUNCH(k_extrap<T>, w, I, w);
}

template <typename T>
void launch_residual(const Inst<T> *I, const ResWork &w, int after_cycle, int any_fd, hipStream_t st) {
    auto *k0 = any_fd ? &k_residual<T, 0, 1> : &k_residual<T, 0, 0>;
    auto *k2 = any_fd ? &k_residual<T, 2, 1> : &k_residual<T, 2, 0>;
    FX_LAUNCH(k0, w.cell0, I, w.cell0, after_cycle);
    if (after_cycle) FX_LAUNCH(k2, w.cell2, I, w.cell2, after_cycle);
}

template <typename T>
void launch_reduce(const Inst<T> *I, InstState *S, int ninst, int count_cycle, hipStream_t st) {
    if (count_cycle) hipLaunchKernelGGL((k_reduce<T, 1>), dim3(ninst), dim3(1024), 0, st, I, S);
    else hipLaunchKernelGGL((k_reduce<T, 0>), dim3(ninst), dim3(1024), 0, st, I, S);
}

template <typename T, int ZT>
struct SmoothSet {
    template <typename F>
    static void pick(int upd, int zero_init, int w8, F go) {
        if (w8) {
            if (upd) go(k_smooth_w8<T, 0, ZT, 1>);
            else if (zero_init) go(k_smooth_w8<T, 1, ZT, 0>);
            else go(k_smooth_w8<T, 0, ZT, 0>);
        } else {
            if (upd) go(k_smooth<T, 0, ZT, 1>);
            else if (zero_init) go(k_smooth<T, 1, ZT, 0>);
            else go(k_smooth<T, 0, ZT, 0>);
        }
    }
};

template <typename T>
void launch_smooth(const Inst<T> *I, const Work &w, int level, int color, int zero_init, int upd, const SmoothCfg &c,
                   double *probe, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, int skip_light) {
    if (w.total <= 0) return;
    const dim3 g = grid_of(w.total);
    const int lbx = c.lbx;
    auto go = [&](auto kern) {
        if (ev0) hipExtLaunchKernelGGL(kern, g, dim3(256), 0, st, ev0, ev1, 0, I, w, level, color, lbx, probe, skip_light);
        else hipLaunchKernelGGL(kern, g, dim3(256), 0, st, I, w, level, color, lbx, probe, skip_light);
    };
    switch (c.zt) {
        case 8: SmoothSet<T, 8>::pick(upd, zero_init, c.w8, go); break;
        case 4: SmoothSet<T, 4>::pick(upd, zero_init, c.w8, go); break;
        case 2: SmoothSet<T, 2>::pick(upd, zero_init, c.w8, go); break;
        default: SmoothSet<T, 1>::pick(upd, zero_init, c.w8, go); break;
    }
}

template <typename T>
void launch_smooth_zpair(const Inst<T> *I, const Work &w, int level, const SmoothCfg &c, hipStream_t st) {
    if (w.total <= 0) return;
    const dim3 g = grid_of(w.total);
    switch (c.zt) {
        case 8: hipLaunchKernelGGL((k_smooth_zpair<T, 8>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
        case 4: hipLaunchKernelGGL((k_smooth_zpair<T, 4>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
        case 2: hipLaunchKernelGGL((k_smooth_zpair<T, 2>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
        default: hipLaunchKernelGGL((k_smooth_zpair<T, 1>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
    }
}

template <typename T>
void launch_prolong_red(const Inst<T> *I, const Work &w, int level, const SmoothCfg &c, hipStream_t st) {
    if (w.total <= 0) return;
    const dim3 g = grid_of(w.total);
    switch (c.zt) {
        case 8: hipLaunchKernelGGL((k_prolong_red<T, 8>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
        case 4: hipLaunchKernelGGL((k_prolong_red<T, 4>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
        case 2: hipLaunchKernelGGL((k_prolong_red<T, 2>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
        default: hipLaunchKernelGGL((k_prolong_red<T, 1>), g, dim3(256), 0, st, I, w, level, c.lbx); break;
    }
}

template <typename T>
void launch_restrict(const Inst<T> *I, const Work &w, int level, hipStream_t st) {
    FX_LAUNCH(k_restrict<T>, w, I, w, level);
}

template <typename T>
void launch_prolong(const Inst<T> *I, const Work &w, int level, hipStream_t st) {
    FX_LAUNCH(k_prolong<T>, w, I, w, level);
}

template <typename T>
void launch_prolong_cc(const Inst<T> *I, const Work &w, int level, int cz, hipStream_t st) {
    FX_LAUNCH(k_prolong_cc<T>, w, I, w, level, cz);
}

template <typename T>
void launch_pre_tb(const Inst<T> *I, const Work &w, int level, int nu, int lds_bytes, hipStream_t st) {
    if (w.total <= 0) return;
    hipLaunchKernelGGL(k_pre_tb<T>, grid_of(w.total), dim3(TbShape<TbCfg<T>::pre_q>::threads), lds_bytes, st, I, w,
                       level, nu);
}
template <typename T>
void launch_post_tb(const Inst<T> *I, const Work &w, int level, int nu, int lds_bytes, hipStream_t st) {
    if (w.total <= 0) return;
    hipLaunchKernelGGL(k_post_tb<T>, grid_of(w.total), dim3(TbShape<TbCfg<T>::post_q>::threads), lds_bytes, st, I, w,
                       level, nu);
}
template <typename T>
void launch_coarse(const Inst<T> *I, InstState *S, int ninst, int lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse<T>, dim3(ninst), dim3(kCoarseThreads), lds_bytes, st, I, S);
}

template <typename T>
void launch_head(const Inst<T> *I, InstState *S, int ninst, int advance, hipStream_t st) {
    hipLaunchKernelGGL(k_head<T>, per_inst(ninst), dim3(64), 0, st, I, S, ninst, advance);
}


template <typename T>
void launch_run_setup(const Inst<T> *I, int ninst, int nsteps, int has_sched, double dt, int first, hipStream_t st) {
    hipLaunchKernelGGL(k_run_setup<T>, per_inst(ninst), dim3(64), 0, st, I, ninst, nsteps, has_sched, dt, first);
}

template <typename T>
void launch_set_vtop(const Inst<T> *I, int ninst, double v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_vtop<T>, per_inst(ninst), dim3(64), 0, st, I, ninst, v);
}

void launch_put_state(InstState *dst, const InstState &v, hipStream_t st) {
    hipLaunchKernelGGL(k_put_state, dim3(1), dim3(64), 0, st, dst, v);
}

void launch_zero(void *x, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4, b = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero32, dim3(b == 0 ? 1 : (b < 4096 ? (unsigned)b : 4096u)), dim3(256), 0, st, (unsigned *)x, n);
}

void launch_fill(double *x, size_t n, double v, hipStream_t st) {
    const size_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3(b == 0 ? 1 : (b < 4096 ? (unsigned)b : 4096u)), dim3(256), 0, st, x, n, v);
}

#define FX_INST(T)                                                                                           \
    template void launch_tdgl<T>(const Inst<T> *, const Work &, int, hipStream_t);                           \
    template void launch_tdgl_corr<T>(const Inst<T> *, const Work &, hipStream_t);                           \
    template void launch_flip<T>(const Inst<T> *, int, hipStream_t);                                        \
    template void launch_qv<T>(const Inst<T> *, int, int, double *, hipStream_t);                            \
    template void launch_begin<T>(const Inst<T> *, InstState *, int, int, hipStream_t);                                  \
    template void launch_extrap<T>(const Inst<T> *, const Work &, hipStream_t);                              \
    template void launch_residual<T>(const Inst<T> *, const ResWork &, int, int, hipStream_t);                    \
    template void launch_reduce<T>(const Inst<T> *, InstState *, int, int, hipStream_t);                                  \
    template void launch_smooth<T>(const Inst<T> *, const Work &, int, int, int, int, const SmoothCfg &,     \
                                   double *, hipStream_t, hipEvent_t, hipEvent_t, int);                      \
    template void launch_smooth_zpair<T>(const Inst<T> *, const Work &, int, const SmoothCfg &, hipStream_t); \
    template void launch_prolong_red<T>(const Inst<T> *, const Work &, int, const SmoothCfg &, hipStream_t);  \
    template void launch_restrict<T>(const Inst<T> *, const Work &, int, hipStream_t);                       \
    template void launch_prolong<T>(const Inst<T> *, const Work &, int, hipStream_t);                        \
    template void launch_prolong_cc<T>(const Inst<T> *, const Work &, int, int, hipStream_t);                \
    template void launch_coarse<T>(const Inst<T> *, InstState *, int, int, hipStream_t);                      \
    template void launch_pre_tb<T>(const Inst<T> *, const Work &, int, int, int, hipStream_t);                 \
    template void launch_post_tb<T>(const Inst<T> *, const Work &, int, int, int, hipStream_t);                                  \
    template void launch_head<T>(const Inst<T> *, InstState *, int, int, hipStream_t);                                    \
    template void launch_run_setup<T>(const Inst<T> *, int, int, int, double, int, hipStream_t);             \
    template void launch_set_vtop<T>(const Inst<T> *, int, double, hipStream_t);
FX_INST(double)
FX_INST(float)

}  // namespace fx
