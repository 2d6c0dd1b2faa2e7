// HIP kernels of the TDGL + Poisson time step (gfx950, wave64).
//
// Layout: fields are z-major with x fastest.  Multigrid levels with an even
// x-extent store their cells split by red/black colour (see LevelArgs), so
// that each half-sweep of the Gauss-Seidel smoother streams two contiguous
// arrays instead of touching every other element.  Workgroups are 64x4
// threads (one wave per row); large launches use a 1D grid whose block
// index is remapped so that each of the 8 XCDs walks one contiguous range of
// tiles (consecutive planes and rows), keeping stencil neighbours in that
// XCD's L2.
#include "fx_internal.h"

#include <hip/hip_ext.h>

namespace fx {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

__device__ __forceinline__ int wrap_p(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }

struct Tile {
    int tx, ty, k, id;
    bool ok;
};

// Tile of a 1D launch whose block count is a multiple of 8: XCD x (= block
// index mod 8 under round-robin dispatch) gets tiles [x*nb/8, (x+1)*nb/8).
__device__ __forceinline__ Tile tile_of(int ntx, int nty, int nz) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int t = (b & 7) * (nb >> 3) + (b >> 3);
    Tile r;
    r.id = t;
    r.ok = t < ntx * nty * nz;
    r.tx = t % ntx;
    const int q = t / ntx;
    r.ty = q % nty;
    r.k = q / nty;
    return r;
}

int tiles(int nxw, int ny, int nz) { return ((nxw + BX - 1) / BX) * ((ny + BY - 1) / BY) * nz; }
dim3 tile_grid(int ntiles) { return dim3((ntiles + 7) / 8 * 8); }

template <typename T>
__device__ __forceinline__ int cidx(const LevelArgs<T> &L, int i, int j, int k) {
    const int lin = (k * L.ny + j) * L.nx + i;
    if (!L.rb) return lin;
    return (((i + j + k) & 1) ? ((L.nx * L.ny * L.nz) >> 1) : 0) + (lin >> 1);
}

template <typename T>
__device__ __forceinline__ bool has_sig(const LevelArgs<T> &L, int k) { return k >= L.sig_lo && k < L.sig_hi; }

template <typename T>
__device__ __forceinline__ int sidx(const LevelArgs<T> &L, int i, int j, int k) {
    const int lin = ((k - L.sig_lo) * L.ny + j) * L.nx + i;
    if (!L.rb) return lin;
    return (((i + j + k) & 1) ? ((L.nx * L.ny * (L.sig_hi - L.sig_lo)) >> 1) : 0) + (lin >> 1);
}

// sum over the 6 neighbours of coefficient * e(neighbour); Dirichlet neighbours are zero
template <typename T>
__device__ __forceinline__ T nb_sum(const LevelArgs<T> &L, const T *e, int i, int j, int k) {
    T s = 0;
    const T cx = L.cxy[k];
    if (L.nx > 1) s += cx * (e[cidx(L, wrap_p(i, L.nx), j, k)] + e[cidx(L, wrap_m(i, L.nx), j, k)]);
    if (L.ny > 1) s += cx * (e[cidx(L, i, wrap_p(j, L.ny), k)] + e[cidx(L, i, wrap_m(j, L.ny), k)]);
    if (k > 0) s += L.czm[k] * e[cidx(L, i, j, k - 1)];
    if (k < L.nz - 1) s += L.czp[k] * e[cidx(L, i, j, k + 1)];
    return s;
}

template <typename T>
__device__ __forceinline__ T diag_of(const LevelArgs<T> &L, int i, int j, int k) {
    T d = L.dg[k];
    if (has_sig(L, k)) d += L.sig[sidx(L, i, j, k)];
    return d;
}

// Gauss-Seidel update of one cell of (L + diag sigma) e = r.
template <typename T>
__device__ __forceinline__ void gs_cell(const LevelArgs<T> &L, int i, int j, int k, int zero_init) {
    const int c = cidx(L, i, j, k);
    const T d = diag_of(L, i, j, k);
    L.e[c] = zero_init ? L.r[c] / d : (L.r[c] + nb_sum(L, L.e, i, j, k)) / d;
}

// Residual of the finer level restricted to one coarse cell: volume-weighted
// mean over the children, likewise sigma.  On a red/black level the black
// children are skipped: right after a black half-sweep their residual is
// zero (each black equation has just been solved exactly).
template <typename T>
__device__ __forceinline__ void restrict_cell(const LevelArgs<T> &F, const LevelArgs<T> &C, const XferArgs<T> &X,
                                              int I, int J, int K) {
    const int nsub = X.xy ? 2 : 1;
    double sr = 0.0, ss = 0.0;
    const int ks = X.cks[K], cnt = X.ccnt[K];
    for (int dz = 0; dz < cnt; ++dz) {
        const int k = ks + dz;
        const double wz = (double)X.fthick[k] / (double)X.cthick[K];
        const bool hs = has_sig(F, k);
        for (int dy = 0; dy < nsub; ++dy) {
            const int j = X.xy ? 2 * J + dy : J;
            for (int dx = 0; dx < nsub; ++dx) {
                const int i = X.xy ? 2 * I + dx : I;
                const T sg = hs ? F.sig[sidx(F, i, j, k)] : T(0);
                ss += wz * (double)sg;
                if (F.rb && ((i + j + k) & 1)) continue;
                const int c = cidx(F, i, j, k);
                const T res = F.r[c] - ((F.dg[k] + sg) * F.e[c] - nb_sum(F, F.e, i, j, k));
                sr += wz * (double)res;
            }
        }
    }
    const double wxy = X.xy ? 0.25 : 1.0;
    C.r[cidx(C, I, J, K)] = (T)(sr * wxy);
    if (has_sig(C, K)) C.sig[sidx(C, I, J, K)] = (T)(ss * wxy);
}

// e_f += I e_c: bilinear in x,y (cell-centred 3/4, 1/4), linear in z between
// coarse plane centres (zero on contact faces).  On a red/black level only
// black cells are corrected: the red values are overwritten by the next red
// half-sweep without being read.
template <typename T>
__device__ __forceinline__ void prolong_cell(const LevelArgs<T> &F, const LevelArgs<T> &C, const XferArgs<T> &X,
                                             int i, int j, int k) {
    if (F.rb && !((i + j + k) & 1)) return;
    int ix[2], jy[2];
    T wx[2], wy[2];
    int ns = 1;
    if (X.xy) {
        const int I = i >> 1, J = j >> 1;
        ix[0] = I; ix[1] = (i & 1) ? wrap_p(I, C.nx) : wrap_m(I, C.nx);
        jy[0] = J; jy[1] = (j & 1) ? wrap_p(J, C.ny) : wrap_m(J, C.ny);
        wx[0] = wy[0] = T(0.75);
        wx[1] = wy[1] = T(0.25);
        ns = 2;
    } else {
        ix[0] = i; jy[0] = j; wx[0] = wy[0] = T(1);
    }
    T v = 0;
    const int kz[2] = {X.pka[k], X.pkb[k]};
    const T wz[2] = {X.pwa[k], X.pwb[k]};
    for (int q = 0; q < 2; ++q) {
        if (kz[q] < 0) continue;
        T s = 0;
        for (int yy = 0; yy < ns; ++yy)
            for (int xx = 0; xx < ns; ++xx) s += wx[xx] * wy[yy] * C.e[cidx(C, ix[xx], jy[yy], kz[q])];
        v += wz[q] * s;
    }
    F.e[cidx(F, i, j, k)] += v;
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

// ------------------------------------------------------------------- TDGL
// eq. (TDGL2) with forward Euler (Step 1a); surface stencils of eqs. (Pbc),
// (PbcFree), (PbcDir) on the two ferroelectric boundary planes.
__device__ __forceinline__ double surface_value(int pbc, double lambda, double h, double p0, double p1) {
    if (pbc == 0) return (9.0 * p0 - p1) * 0.125;
    if (pbc == 1) return 0.0;
    return lambda * (9.0 * p0 - p1) / (8.0 * lambda + 3.0 * h);
}

__global__ __launch_bounds__(256) void k_tdgl(TdglArgs a) {
    const Tile t = tile_of((a.nx + BX - 1) / BX, (a.ny + BY - 1) / BY, a.f1 - a.f0);
    if (!t.ok) return;
    const int i = t.tx * BX + threadIdx.x;
    const int j = t.ty * BY + threadIdx.y;
    const int k = a.f0 + t.k;
    if (i >= a.nx || j >= a.ny) return;
    const size_t nxy = (size_t)a.nx * a.ny;
    const size_t c = (size_t)k * nxy + (size_t)j * a.nx + i;
    const double *P = a.P, *phi = a.phi;
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
    const double dF = landau - a.g44 * (dxx + dyy) - a.g11 * dzz + dphi;
    a.Pn[c] = p - a.dt * a.Gamma * dF;
}

// ------------------------------------------------------ fine-level residual
// MODE 0: residual at phi_in; MODE 2: at phi_in + clip(e), written to phi_out.
// Each thread owns a column of ZT planes.  All loads are issued before any
// arithmetic (clamped indices instead of boundary branches; the z-neighbours
// of the column's planes are loaded once) so a wave makes one memory round
// trip for ZT cells.
template <typename T, int MODE, int ZT>
__global__ __launch_bounds__(256) void k_residual(ResArgs<T> a) {
    __shared__ double lds_r[4];
    __shared__ double lds_f[4];
    if (a.ctrl->done) return;
    const int nx = a.nx, ny = a.ny, nzd = a.nzd;
    const Tile t = tile_of((nx + BX - 1) / BX, (ny + BY - 1) / BY, (nzd + ZT - 1) / ZT);
    if (!t.ok) return;
    const int ii = t.tx * BX + threadIdx.x;
    const int jj = t.ty * BY + threadIdx.y;
    const bool live = ii < nx && jj < ny;
    const int i = live ? ii : 0, j = live ? jj : 0;
    const int k0 = t.k * ZT;
    const int nxy = nx * ny;
    const size_t off = (size_t)a.kb * nxy;
    const double *phi = a.phi_in + off;
    const double *P = a.P + off;
    const int col = j * nx + i;
    const int ox0 = wrap_p(i, nx) - i, ox1 = wrap_m(i, nx) - i;
    const int oy0 = (wrap_p(j, ny) - j) * nx, oy1 = (wrap_m(j, ny) - j) * nx;
    const int rb = a.L0.rb;
    const int half = (nxy * nzd) >> 1;
    const double big = 1e300;
    auto kcl = [&](int k) { return k < 0 ? 0 : (k >= nzd ? nzd - 1 : k); };
    // ---- bound charge: P of the column's planes and their neighbours (ferroelectric tiles only)
    double pz[ZT + 2];
#pragma unroll
    for (int z = 0; z < ZT + 2; ++z) pz[z] = 0.0;
    bool anyP = false;
#pragma unroll
    for (int z = 0; z < ZT; ++z) anyP |= (k0 + z < nzd) && (a.pflags[kcl(k0 + z)] & PF_P);
    if (anyP) {
#pragma unroll
        for (int z = 0; z < ZT + 2; ++z) pz[z] = P[kcl(k0 - 1 + z) * nxy + col];
    }
    // ---- potential at the column (planes k0-1 .. k0+ZT) and the x/y neighbours (k0 .. k0+ZT-1)
    double vc[ZT + 2], vx0[ZT], vx1[ZT], vy0[ZT], vy1[ZT];
    auto at = [&](int k, int o, int par, double *dst) {
        const int c = k * nxy + col + o;
        double v = phi[c];
        if (MODE == 2) {
            const double d = (double)a.e[rb ? (par ? half : 0) + (c >> 1) : c];
            const double lim = (a.pflags[k] & PF_SC) ? a.dmax : big;
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
        at(k, ox0, pn, &vx0[z]);
        at(k, ox1, pn, &vx1[z]);
        at(k, oy0, pn, &vy0[z]);
        at(k, oy1, pn, &vy1[z]);
    }
    // ---- residual, carriers and stores, plane by plane
    double rr = 0.0, ff = 0.0;
    const LevelArgs<T> &L = a.L0;
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = k0 + z;
        if (k >= nzd) break;
        const int fl = a.pflags[k];
        const double v0 = vc[z + 1];
        const double nb = (vx0[z] + vx1[z] - 2.0 * v0) + (vy0[z] + vy1[z] - 2.0 * v0);
        const double dn = k > 0 ? vc[z] : 0.0;
        const double up = k < nzd - 1 ? vc[z + 2] : 0.0;
        const double Lphi = -a.cxy[k] * nb + a.czm[k] * (v0 - dn) + a.czp[k] * (v0 - up);
        double f = 0.0;
        if (fl & PF_P) {
            const double pc = pz[z + 1];
            const double pup = k == nzd - 1 ? pc : a.wl[k] * pc + a.wr[k] * pz[z + 2];
            const double pdn = k == 0 ? pc : a.wl[k - 1] * pz[z] + a.wr[k - 1] * pc;
            f = -(pup - pdn) * a.p_scale;
        }
        if (k == 0) f += a.czm[k] * a.v_b;
        if (k == nzd - 1) f += a.czp[k] * a.v_t;
        double res = f - Lphi;
        if (live) {
            const int cl = k * nxy + col;
            if (MODE != 0) a.phi_out[off + cl] = v0;
            if (fl & PF_SC) {
                const double u = v0 * a.vt_inv;
                const double em = expm1(-u), ep = expm1(u);
                const double p0e = a.p0e[k], n0e = a.n0e[k];
                res += (p0e * em - n0e * ep) * a.rho_scale;                       // + rho_c
                L.sig[sidx(L, i, j, k)] = (T)((p0e * (1.0 + em) + n0e * (1.0 + ep)) * a.sig_scale);
            }
            L.r[cidx(L, i, j, k)] = (T)res;
            rr += res * res;
            ff += f * f;
        }
    }
    const double sr = block_sum(rr, lds_r);
    const double sf = block_sum(ff, lds_f);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        a.part[2 * t.id] = sr;
        a.part[2 * t.id + 1] = sf;
    }
}

// Deterministic final sum of the residual partials and the stop decision.
__global__ __launch_bounds__(1024) void k_reduce(const double *part, int n, SolveCtrl *ctrl, int count_cycle) {
    __shared__ double lr[16];
    __shared__ double lf[16];
    if (ctrl->done) return;
    double r = 0.0, f = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) { r += part[2 * b]; f += part[2 * b + 1]; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) { r += __shfl_down(r, off, 64); f += __shfl_down(f, off, 64); }
    if ((threadIdx.x & 63) == 0) { lr[threadIdx.x >> 6] = r; lf[threadIdx.x >> 6] = f; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { a += lr[q]; b += lf[q]; }
        ctrl->rn2 = a;
        ctrl->fn2 = b;
        if (count_cycle) ctrl->cycles += 1;
        if (!isfinite(a) || !isfinite(b)) ctrl->done = 2;
        else if (a <= ctrl->tol2 * b || a == 0.0 || b == 0.0) ctrl->done = 1;   // b = 0: the host sets phi = 0
        else if (ctrl->cycles >= ctrl->max_cycles) ctrl->done = 3;
    }
}

__global__ void k_ctrl_reset(SolveCtrl *ctrl, int max_cycles, double tol2) {
    ctrl->done = 0;
    ctrl->cycles = 0;
    ctrl->max_cycles = max_cycles;
    ctrl->tol2 = tol2;
    ctrl->rn2 = 0.0;
    ctrl->fn2 = 0.0;
}

// ----------------------------------------------------------------- smoother
// One colour of red-black Gauss-Seidel on a red/black-split level: a thread
// per cell of that colour, all reads and writes contiguous along x.
template <typename T, int ZI, int ZT, int UPD>
__global__ __launch_bounds__(256) void k_smooth_rb(LevelArgs<T> L, int color, const SolveCtrl *ctrl, UpdArgs u) {
    if (ctrl->done) return;
    const int hx = L.nx >> 1;
    const Tile t = tile_of((hx + BX - 1) / BX, (L.ny + BY - 1) / BY, (L.nz + ZT - 1) / ZT);
    if (!t.ok) return;
    const int mm = t.tx * BX + threadIdx.x;
    const int jj = t.ty * BY + threadIdx.y;
    const bool live = mm < hx && jj < L.ny;
    const int m = live ? mm : 0, j = live ? jj : 0;
    const int half = (L.nx * L.ny * L.nz) >> 1;
    const int plane = L.ny * hx;
    const T *eo = L.e + (color ? 0 : half);
    T *es = L.e + (color ? half : 0);
    const T *rs = L.r + (color ? half : 0);
    const int hsz = (L.nx * L.ny * (L.sig_hi - L.sig_lo)) >> 1;
    const int oy0 = L.ny > 1 ? (wrap_p(j, L.ny) - j) * hx : 0;
    const int oy1 = L.ny > 1 ? (wrap_m(j, L.ny) - j) * hx : 0;
    T out[ZT];
    // loads of all ZT planes first
    T rr[ZT], sg[ZT], ex0[ZT], ex1[ZT], ey0[ZT], ey1[ZT], ez0[ZT], ez1[ZT], ep[ZT];
    double2 ph[ZT];
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = min(t.k * ZT + z, L.nz - 1);
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
        if (UPD) {
            ep[z] = eo[q];                       // the red partner of this black cell's pair
            ph[z] = *(const double2 *)(u.phi_in + (size_t)k * L.nx * L.ny + (size_t)j * L.nx + 2 * m);
        }
    }
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = min(t.k * ZT + z, L.nz - 1);
        const bool hs = k >= L.sig_lo && k < L.sig_hi;
        T s = 0;
        if (!ZI) {
            const T cx = L.cxy[k];
            const T cy = L.ny > 1 ? cx : T(0);
            s = cx * (ex0[z] + ex1[z]) + cy * (ey0[z] + ey1[z]) + (k > 0 ? L.czm[k] : T(0)) * ez0[z] +
                (k < L.nz - 1 ? L.czp[k] : T(0)) * ez1[z];
        }
        out[z] = (rr[z] + s) / (L.dg[k] + (hs ? sg[z] : T(0)));
    }
#pragma unroll
    for (int z = 0; z < ZT; ++z) {
        const int k = t.k * ZT + z;
        if (live && k < L.nz) {
            es[k * plane + j * hx + m] = out[z];
            if (UPD) {
                const double lim = (u.pflags[k] & PF_SC) ? u.dmax : 1e300;
                const double db = fmin(fmax((double)out[z], -lim), lim);
                const double dr = fmin(fmax((double)ep[z], -lim), lim);
                const bool odd = ((color + j + k) & 1) != 0;          // black cell at 2m+1
                double2 o;
                o.x = ph[z].x + (odd ? dr : db);
                o.y = ph[z].y + (odd ? db : dr);
                *(double2 *)(u.phi_out + (size_t)k * L.nx * L.ny + (size_t)j * L.nx + 2 * m) = o;
            }
        }
    }
}

// Colour of a cell on a plainly stored level (odd x or y extent).  With an
// odd periodic extent the parity colouring makes the wrap neighbours equal
// coloured, so the last column / row (for odd nx / ny) get colours 2 and 3:
// no two cells of one colour are then neighbours, and a sweep is the four
// colours in turn.
template <typename T>
__device__ __forceinline__ int nat_color(const LevelArgs<T> &L, int i, int j, int k) {
    const int par = (i + j + k) & 1;
    const bool edge = ((L.nx & 1) && i == L.nx - 1) || ((L.ny & 1) && j == L.ny - 1);
    return edge ? 2 + par : par;
}

// One colour of the Gauss-Seidel sweep on a plainly stored level: a thread per cell.
template <typename T>
__global__ __launch_bounds__(256) void k_smooth_nat(LevelArgs<T> L, int color, int zero_init, const SolveCtrl *ctrl) {
    if (ctrl->done) return;
    const Tile t = tile_of((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, L.nz);
    if (!t.ok) return;
    const int i = t.tx * BX + threadIdx.x;
    const int j = t.ty * BY + threadIdx.y;
    const int k = t.k;
    if (i >= L.nx || j >= L.ny) return;
    if (nat_color(L, i, j, k) != color) {
        if (zero_init) L.e[cidx(L, i, j, k)] = T(0);
        return;
    }
    gs_cell(L, i, j, k, zero_init);
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict(LevelArgs<T> F, LevelArgs<T> C, XferArgs<T> X, const SolveCtrl *ctrl) {
    if (ctrl->done) return;
    const Tile t = tile_of((C.nx + BX - 1) / BX, (C.ny + BY - 1) / BY, C.nz);
    if (!t.ok) return;
    const int I = t.tx * BX + threadIdx.x;
    const int J = t.ty * BY + threadIdx.y;
    if (I >= C.nx || J >= C.ny) return;
    restrict_cell(F, C, X, I, J, t.k);
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong(LevelArgs<T> F, LevelArgs<T> C, XferArgs<T> X, const SolveCtrl *ctrl) {
    if (ctrl->done) return;
    int i, j, k;
    if (F.rb) {                       // a thread per black cell
        const int hx = F.nx >> 1;
        const Tile t = tile_of((hx + BX - 1) / BX, (F.ny + BY - 1) / BY, F.nz);
        if (!t.ok) return;
        const int m = t.tx * BX + threadIdx.x;
        j = t.ty * BY + threadIdx.y;
        k = t.k;
        if (m >= hx || j >= F.ny) return;
        i = 2 * m + ((1 + j + k) & 1);
    } else {
        const Tile t = tile_of((F.nx + BX - 1) / BX, (F.ny + BY - 1) / BY, F.nz);
        if (!t.ok) return;
        i = t.tx * BX + threadIdx.x;
        j = t.ty * BY + threadIdx.y;
        k = t.k;
        if (i >= F.nx || j >= F.ny) return;
    }
    prolong_cell(F, C, X, i, j, k);
}

// --------------------------------------------- coarse levels in one workgroup
template <typename T>
__device__ void smooth_color(const LevelArgs<T> &L, int color, int zero_init) {
    if (L.rb) {
        const int hx = L.nx >> 1;
        const int n = hx * L.ny * L.nz;
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int m = q % hx, row = q / hx, j = row % L.ny, k = row / L.ny;
            gs_cell(L, 2 * m + ((color + j + k) & 1), j, k, zero_init);
        }
    } else {
        const int n = L.nx * L.ny * L.nz;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const int i = c % L.nx, row = c / L.nx, j = row % L.ny, k = row / L.ny;
            if (nat_color(L, i, j, k) == color) gs_cell(L, i, j, k, zero_init);
            else if (zero_init) L.e[cidx(L, i, j, k)] = T(0);
        }
    }
}

// One full Gauss-Seidel sweep (2 colours on split levels, 4 otherwise).
template <typename T>
__device__ void smooth_sweep(const LevelArgs<T> &L, int zero_init) {
    const int ncol = L.rb ? 2 : 4;
    for (int c = 0; c < ncol; ++c) {
        smooth_color(L, c, zero_init && c == 0);
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(512) void k_coarse(const CoarseArgs<T> *A, const SolveCtrl *ctrl) {
    extern __shared__ double lds_raw[];
    if (ctrl->done) return;
    unsigned char *lds = (unsigned char *)lds_raw;
    const int nl = A->nlev;
    // level views with LDS-resident e, r, sig
    auto lvl = [&](int l) {
        LevelArgs<T> L = A->lv[l];
        L.e = (T *)(lds + A->off_e[l]);
        L.r = (T *)(lds + A->off_r[l]);
        L.sig = (T *)(lds + A->off_s[l]);
        T *tab = (T *)(lds + A->off_t[l]);
        L.cxy = tab;
        L.czm = tab + L.nz;
        L.czp = tab + 2 * L.nz;
        L.dg = tab + 3 * L.nz;
        return L;
    };
    for (int l = 0; l < nl; ++l) {        // per-plane coefficient tables into LDS
        const LevelArgs<T> G = A->lv[l];
        T *tab = (T *)(lds + A->off_t[l]);
        for (int c = threadIdx.x; c < G.nz; c += blockDim.x) {
            tab[c] = G.cxy[c];
            tab[G.nz + c] = G.czm[c];
            tab[2 * G.nz + c] = G.czp[c];
            tab[3 * G.nz + c] = G.dg[c];
        }
    }
    {
        const LevelArgs<T> L0 = lvl(0);
        const int n = L0.nx * L0.ny * L0.nz;
        const int ns = L0.nx * L0.ny * (L0.sig_hi - L0.sig_lo);
        for (int c = threadIdx.x; c < n; c += blockDim.x) L0.r[c] = A->r_in[c];
        for (int c = threadIdx.x; c < ns; c += blockDim.x) L0.sig[c] = A->sig_in[c];
        __syncthreads();
    }
    for (int l = 0; l < nl - 1; ++l) {
        const LevelArgs<T> L = lvl(l);
        for (int s = 0; s < A->nu1; ++s) smooth_sweep(L, s == 0);
        const LevelArgs<T> C = lvl(l + 1);
        const XferArgs<T> X = A->xf[l];
        const int n = C.nx * C.ny * C.nz;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const int I = c % C.nx, row = c / C.nx;
            restrict_cell(L, C, X, I, row % C.ny, row / C.ny);
        }
        __syncthreads();
    }
    {
        const LevelArgs<T> B = lvl(nl - 1);
        for (int s = 0; s < A->bottom_sweeps; ++s) smooth_sweep(B, s == 0);
    }
    for (int l = nl - 2; l >= 0; --l) {
        const LevelArgs<T> L = lvl(l);
        const LevelArgs<T> C = lvl(l + 1);
        const XferArgs<T> X = A->xf[l];
        const int n = L.nx * L.ny * L.nz;
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const int i = c % L.nx, row = c / L.nx;
            prolong_cell(L, C, X, i, row % L.ny, row / L.ny);
        }
        __syncthreads();
        for (int s = 0; s < A->nu2; ++s) smooth_sweep(L, 0);
    }
    {
        const LevelArgs<T> L0 = lvl(0);
        const int n = L0.nx * L0.ny * L0.nz;
        for (int c = threadIdx.x; c < n; c += blockDim.x) A->e_out[c] = L0.e[c];
    }
}

// out = sum_q c[q] in[q] over n contiguous values (polynomial extrapolation in time).
__global__ __launch_bounds__(256) void k_extrap(double *out, ExtrapArgs a, size_t n) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
        double v = a.c[0] * a.in[0][c];
        for (int q = 1; q < a.nin; ++q) v += a.c[q] * a.in[q][c];
        out[c] = v;
    }
}

__global__ void k_fill(double *x, size_t n, double v) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) x[c] = v;
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_tdgl(const TdglArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_tdgl, tile_grid(tiles(a.nx, a.ny, a.f1 - a.f0)), dim3(BX, BY), 0, st, a);
}

constexpr int kResZ = 4;   // planes per thread in the fine-level residual

template <typename T>
int launch_residual(const ResArgs<T> &a, hipStream_t st) {
    const int n = tiles(a.nx, a.ny, (a.nzd + kResZ - 1) / kResZ);
    if (a.e)
        hipLaunchKernelGGL((k_residual<T, 2, kResZ>), tile_grid(n), dim3(BX, BY), 0, st, a);
    else
        hipLaunchKernelGGL((k_residual<T, 0, kResZ>), tile_grid(n), dim3(BX, BY), 0, st, a);
    return n;
}

template <typename T>
void launch_smooth(const LevelArgs<T> &L, int color, int zero_init, const SolveCtrl *ctrl, hipStream_t st,
                   const UpdArgs *upd, hipEvent_t ev0, hipEvent_t ev1) {
    if (!L.rb) {
        hipLaunchKernelGGL(k_smooth_nat<T>, tile_grid(tiles(L.nx, L.ny, L.nz)), dim3(BX, BY), 0, st, L, color,
                           zero_init, ctrl);
        return;
    }
    // large levels: 4 planes per thread; small ones one plane per thread for parallelism
    const bool deep = (size_t)L.nx * L.ny * L.nz >= (1u << 19) && L.nz >= 8;
    const dim3 g = deep ? tile_grid(tiles(L.nx / 2, L.ny, (L.nz + 3) / 4)) : tile_grid(tiles(L.nx / 2, L.ny, L.nz));
    const UpdArgs u = upd ? *upd : UpdArgs{nullptr, nullptr, nullptr, 0.0};
    auto go = [&](auto kern) {
        if (ev0) hipExtLaunchKernelGGL(kern, g, dim3(BX, BY), 0, st, ev0, ev1, 0, L, color, ctrl, u);
        else hipLaunchKernelGGL(kern, g, dim3(BX, BY), 0, st, L, color, ctrl, u);
    };
    if (upd) {
        if (deep) go(k_smooth_rb<T, 0, 4, 1>);
        else go(k_smooth_rb<T, 0, 1, 1>);
    } else if (zero_init) {
        if (deep) go(k_smooth_rb<T, 1, 4, 0>);
        else go(k_smooth_rb<T, 1, 1, 0>);
    } else {
        if (deep) go(k_smooth_rb<T, 0, 4, 0>);
        else go(k_smooth_rb<T, 0, 1, 0>);
    }
}

template <typename T>
void launch_restrict(const LevelArgs<T> &F, const LevelArgs<T> &C, const XferArgs<T> &X, const SolveCtrl *ctrl,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_restrict<T>, tile_grid(tiles(C.nx, C.ny, C.nz)), dim3(BX, BY), 0, st, F, C, X, ctrl);
}

template <typename T>
void launch_prolong(const LevelArgs<T> &F, const LevelArgs<T> &C, const XferArgs<T> &X, const SolveCtrl *ctrl,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_prolong<T>, tile_grid(tiles(F.rb ? F.nx / 2 : F.nx, F.ny, F.nz)), dim3(BX, BY), 0, st, F, C, X,
                       ctrl);
}

template <typename T>
void launch_coarse(const CoarseArgs<T> *dev_args, int lds_bytes, const SolveCtrl *ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(512), lds_bytes, st, dev_args, ctrl);
}

void launch_reduce(const double *part, int nparts, SolveCtrl *ctrl, int count_cycle, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, part, nparts, ctrl, count_cycle);
}

void launch_ctrl_reset(SolveCtrl *ctrl, int max_cycles, double tol2, hipStream_t st) {
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(1), 0, st, ctrl, max_cycles, tol2);
}

void launch_extrap(double *out, const ExtrapArgs &a, size_t n, hipStream_t st) {
    const size_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_extrap, dim3(b < 8192 ? (unsigned)b : 8192u), dim3(256), 0, st, out, a, n);
}

void launch_fill(double *x, size_t n, double v, hipStream_t st) {
    const size_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3(b == 0 ? 1 : (b < 4096 ? (unsigned)b : 4096u)), dim3(256), 0, st, x, n, v);
}

#define FX_INST(T)                                                                                              \
    template int launch_residual<T>(const ResArgs<T> &, hipStream_t);                                            \
    template void launch_smooth<T>(const LevelArgs<T> &, int, int, const SolveCtrl *, hipStream_t, const UpdArgs *, \
                                   hipEvent_t, hipEvent_t);                                                      \
    template void launch_restrict<T>(const LevelArgs<T> &, const LevelArgs<T> &, const XferArgs<T> &,            \
                                     const SolveCtrl *, hipStream_t);                                            \
    template void launch_prolong<T>(const LevelArgs<T> &, const LevelArgs<T> &, const XferArgs<T> &,             \
                                    const SolveCtrl *, hipStream_t);                                             \
    template void launch_coarse<T>(const CoarseArgs<T> *, int, const SolveCtrl *, hipStream_t);
FX_INST(double)
FX_INST(float)

}  // namespace fx
