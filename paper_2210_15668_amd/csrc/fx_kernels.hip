// HIP kernels of the TDGL + Poisson time step (gfx950, wave64).
//
// Layout: every field is z-major, x fastest, so a wave of 64 lanes along x
// reads 512 contiguous bytes (FP64).  Launches use 64x4 blocks (one wave per
// x-row) over (x, y) and one grid layer per z-plane, so all per-plane
// coefficients are wave-uniform scalar loads.
#include "fx_internal.h"

namespace fx {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

__device__ __forceinline__ int wrap_p(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// Sum over a 256-thread block (4 waves); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
        const int nw = (blockDim.x * blockDim.y + 63) >> 6;
        for (int q = 0; q < nw; ++q) s += lds[q];
    }
    return s;
}

dim3 plane_grid(int nx, int ny, int nz) {
    return dim3((nx + BX - 1) / BX, (ny + BY - 1) / BY, nz);
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
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = a.f0 + blockIdx.z;
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
template <typename T>
__global__ __launch_bounds__(256) void k_residual(ResArgs<T> a) {
    __shared__ double lds_r[4];
    __shared__ double lds_f[4];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;                       // device plane
    double rr = 0.0, ff = 0.0;
    if (i < a.nx && j < a.ny) {
        const size_t nxy = (size_t)a.nx * a.ny;
        const size_t cl = (size_t)k * nxy + (size_t)j * a.nx + i;   // level-0 index
        const size_t c = cl + (size_t)a.kb * nxy;                   // full-grid index
        const double *phi = a.phi;
        const double v = phi[c];
        double nb = 0.0;
        if (a.nx > 1) nb += phi[c - i + wrap_p(i, a.nx)] + phi[c - i + wrap_m(i, a.nx)] - 2.0 * v;
        if (a.ny > 1) {
            const size_t pl = c - (size_t)j * a.nx;
            nb += phi[pl + (size_t)wrap_p(j, a.ny) * a.nx] + phi[pl + (size_t)wrap_m(j, a.ny) * a.nx] - 2.0 * v;
        }
        double Lphi = -a.cxy[k] * nb;
        const double dn = k > 0 ? phi[c - nxy] : 0.0;
        const double up = k < a.nzd - 1 ? phi[c + nxy] : 0.0;
        Lphi += a.czm[k] * (v - dn) + a.czp[k] * (v - up);
        double f = 0.0;
        if (k == 0) f += a.czm[k] * a.v_b;
        if (k == a.nzd - 1) f += a.czp[k] * a.v_t;
        const int fl = a.pflags[k];
        if (fl & PF_P) {
            const double pc = a.P[c];
            const double pup = k == a.nzd - 1 ? pc : a.wl[k] * pc + a.wr[k] * a.P[c + nxy];
            const double pdn = k == 0 ? pc : a.wl[k - 1] * a.P[c - nxy] + a.wr[k - 1] * pc;
            f -= (pup - pdn) * a.p_scale;
        }
        double res = f - Lphi;
        if (fl & PF_SC) {
            const double u = v * a.vt_inv;
            const double em = expm1(-u), ep = expm1(u);
            const double p0e = a.p0e[k], n0e = a.n0e[k];
            res += (p0e * em - n0e * ep) * a.rho_scale;                       // + rho_c
            a.sig[cl - (size_t)a.sig_lo * nxy] = (T)((p0e * (1.0 + em) + n0e * (1.0 + ep)) * a.sig_scale);
        }
        a.r[cl] = (T)res;
        rr = res * res;
        ff = f * f;
    }
    const double sr = block_sum(rr, lds_r);
    const double sf = block_sum(ff, lds_f);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        a.part[2 * b] = sr;
        a.part[2 * b + 1] = sf;
    }
}

// ----------------------------------------------------------------- smoother
// One colour of red-black Gauss-Seidel on (L + diag sigma) e = r.
template <typename T>
__device__ __forceinline__ T diag_at(const LevelArgs<T> &L, int k, size_t c, size_t nxy) {
    T d = L.dg[k];
    if (k >= L.sig_lo && k < L.sig_hi) d += L.sig[c - (size_t)L.sig_lo * nxy];
    return d;
}

template <typename T>
__device__ __forceinline__ T offdiag_sum(const LevelArgs<T> &L, const T *e, int i, int j, int k, size_t c, size_t nxy) {
    T s = 0;
    if (L.nx > 1) s += L.cxy[k] * (e[c - i + wrap_p(i, L.nx)] + e[c - i + wrap_m(i, L.nx)]);
    if (L.ny > 1) {
        const size_t pl = c - (size_t)j * L.nx;
        s += L.cxy[k] * (e[pl + (size_t)wrap_p(j, L.ny) * L.nx] + e[pl + (size_t)wrap_m(j, L.ny) * L.nx]);
    }
    if (k > 0) s += L.czm[k] * e[c - nxy];
    if (k < L.nz - 1) s += L.czp[k] * e[c + nxy];
    return s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_smooth(LevelArgs<T> L, int color, int zero_init) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= L.nx || j >= L.ny) return;
    const size_t nxy = (size_t)L.nx * L.ny;
    const size_t c = (size_t)k * nxy + (size_t)j * L.nx + i;
    if (((i + j + k) & 1) != color) {
        if (zero_init) L.e[c] = T(0);
        return;
    }
    const T d = diag_at(L, k, c, nxy);
    if (zero_init) {
        L.e[c] = L.r[c] / d;
        return;
    }
    L.e[c] = (L.r[c] + offdiag_sum(L, L.e, i, j, k, c, nxy)) / d;
}

// ------------------------------------------------- residual + restriction
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(RestrictArgs<T> a) {
    const int I = blockIdx.x * BX + threadIdx.x;
    const int J = blockIdx.y * BY + threadIdx.y;
    const int K = blockIdx.z;
    if (I >= a.c.nx || J >= a.c.ny) return;
    const LevelArgs<T> &F = a.f;
    const size_t fnxy = (size_t)F.nx * F.ny;
    const int nsub = a.xy ? 2 : 1;
    double sr = 0.0, ss = 0.0;
    const int ks = a.cks[K], cnt = a.ccnt[K];
    for (int dz = 0; dz < cnt; ++dz) {
        const int k = ks + dz;
        const double wz = (double)a.fthick[k] / (double)a.cthick[K];
        const bool has_sig = k >= F.sig_lo && k < F.sig_hi;
        for (int dy = 0; dy < nsub; ++dy) {
            const int j = a.xy ? 2 * J + dy : J;
            for (int dx = 0; dx < nsub; ++dx) {
                const int i = a.xy ? 2 * I + dx : I;
                const size_t c = (size_t)k * fnxy + (size_t)j * F.nx + i;
                T d = F.dg[k];
                T sg = 0;
                if (has_sig) { sg = F.sig[c - (size_t)F.sig_lo * fnxy]; d += sg; }
                const T res = F.r[c] - (d * F.e[c] - offdiag_sum(F, F.e, i, j, k, c, fnxy));
                sr += wz * (double)res;
                ss += wz * (double)sg;
            }
        }
    }
    const double wxy = a.xy ? 0.25 : 1.0;
    const size_t cc = ((size_t)K * a.c.ny + J) * a.c.nx + I;
    a.c.r[cc] = (T)(sr * wxy);
    if (K >= a.c.sig_lo && K < a.c.sig_hi)
        a.c.sig[cc - (size_t)a.c.sig_lo * a.c.nx * a.c.ny] = (T)(ss * wxy);
}

// ----------------------------------------------- prolongation + correction
template <typename T>
__global__ __launch_bounds__(256) void k_prolong(ProlongArgs<T> a) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= a.f.nx || j >= a.f.ny) return;
    const int cnx = a.c.nx, cny = a.c.ny;
    int ix[2], jy[2];
    T wx[2], wy[2];
    int nxs = 1, nys = 1;
    if (a.xy) {
        const int I = i >> 1, J = j >> 1;
        ix[0] = I; ix[1] = (i & 1) ? wrap_p(I, cnx) : wrap_m(I, cnx);
        jy[0] = J; jy[1] = (j & 1) ? wrap_p(J, cny) : wrap_m(J, cny);
        wx[0] = T(0.75); wx[1] = T(0.25); wy[0] = T(0.75); wy[1] = T(0.25);
        nxs = 2; nys = 2;
    } else {
        ix[0] = i; jy[0] = j; wx[0] = T(1); wy[0] = T(1);
    }
    const size_t cnxy = (size_t)cnx * cny;
    T v = 0;
    const int kz[2] = {a.ka[k], a.kb[k]};
    const T wz[2] = {a.wa[k], a.wb[k]};
    for (int q = 0; q < 2; ++q) {
        if (kz[q] < 0) continue;
        const T *ec = a.c.e + (size_t)kz[q] * cnxy;
        T s = 0;
        for (int yy = 0; yy < nys; ++yy)
            for (int xx = 0; xx < nxs; ++xx) s += wx[xx] * wy[yy] * ec[(size_t)jy[yy] * cnx + ix[xx]];
        v += wz[q] * s;
    }
    const size_t c = ((size_t)k * a.f.ny + j) * a.f.nx + i;
    a.f.e[c] += v;
}

// ------------------------------------------------------------ bottom solve
// Coarsest level: LDS-resident red-black sweeps in one workgroup.
constexpr int kBottomMax = 2048;

template <typename T>
__global__ __launch_bounds__(1024) void k_bottom(LevelArgs<T> L, int sweeps) {
    __shared__ T se[kBottomMax];
    __shared__ T sr[kBottomMax];
    __shared__ T sd[kBottomMax];
    const int n = L.nx * L.ny * L.nz;
    const int nxy = L.nx * L.ny;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int k = c / nxy;
        T d = L.dg[k];
        if (k >= L.sig_lo && k < L.sig_hi) d += L.sig[c - L.sig_lo * nxy];
        sd[c] = d;
        sr[c] = L.r[c];
        se[c] = T(0);
    }
    __syncthreads();
    for (int s = 0; s < sweeps; ++s) {
        for (int color = 0; color < 2; ++color) {
            for (int c = threadIdx.x; c < n; c += blockDim.x) {
                const int k = c / nxy, rem = c - k * nxy, j = rem / L.nx, i = rem - j * L.nx;
                if (((i + j + k) & 1) != color) continue;
                T acc = sr[c];
                if (L.nx > 1) acc += L.cxy[k] * (se[c - i + wrap_p(i, L.nx)] + se[c - i + wrap_m(i, L.nx)]);
                if (L.ny > 1) {
                    const int pl = c - j * L.nx;
                    acc += L.cxy[k] * (se[pl + wrap_p(j, L.ny) * L.nx] + se[pl + wrap_m(j, L.ny) * L.nx]);
                }
                if (k > 0) acc += L.czm[k] * se[c - nxy];
                if (k < L.nz - 1) acc += L.czp[k] * se[c + nxy];
                se[c] = acc / sd[c];
            }
            __syncthreads();
        }
    }
    for (int c = threadIdx.x; c < n; c += blockDim.x) L.e[c] = se[c];
}

// ------------------------------------------------------------------ update
template <typename T>
__global__ __launch_bounds__(256) void k_update(double *phi, const T *e, int nx, int ny, int kb, const int *pflags,
                                                double dmax) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const size_t nxy = (size_t)nx * ny;
    const size_t cl = (size_t)k * nxy + (size_t)j * nx + i;
    double d = (double)e[cl];
    if (pflags[k] & PF_SC) d = fmin(fmax(d, -dmax), dmax);
    phi[cl + (size_t)kb * nxy] += d;
}

__global__ __launch_bounds__(1024) void k_reduce_norms(const double *part, int nb, double *out) {
    __shared__ double lr[16];
    __shared__ double lf[16];
    double r = 0.0, f = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) { r += part[2 * b]; f += part[2 * b + 1]; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) { r += __shfl_down(r, off, 64); f += __shfl_down(f, off, 64); }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { lr[w] = r; lf[w] = f; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { a += lr[q]; b += lf[q]; }
        out[0] = a;
        out[1] = b;
    }
}

__global__ void k_fill(double *x, size_t n, double v) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) x[c] = v;
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_tdgl(const TdglArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_tdgl, plane_grid(a.nx, a.ny, a.f1 - a.f0), dim3(BX, BY), 0, st, a);
}

template <typename T>
void launch_residual(const ResArgs<T> &a, hipStream_t st, int *nblocks) {
    dim3 g = plane_grid(a.nx, a.ny, a.nzd);
    *nblocks = (int)(g.x * g.y * g.z);
    hipLaunchKernelGGL(k_residual<T>, g, dim3(BX, BY), 0, st, a);
}

template <typename T>
void launch_smooth(const LevelArgs<T> &L, int color, int zero_init, hipStream_t st) {
    hipLaunchKernelGGL(k_smooth<T>, plane_grid(L.nx, L.ny, L.nz), dim3(BX, BY), 0, st, L, color, zero_init);
}

template <typename T>
void launch_restrict(const RestrictArgs<T> &a, hipStream_t st) {
    hipLaunchKernelGGL(k_restrict<T>, plane_grid(a.c.nx, a.c.ny, a.c.nz), dim3(BX, BY), 0, st, a);
}

template <typename T>
void launch_prolong(const ProlongArgs<T> &a, hipStream_t st) {
    hipLaunchKernelGGL(k_prolong<T>, plane_grid(a.f.nx, a.f.ny, a.f.nz), dim3(BX, BY), 0, st, a);
}

template <typename T>
void launch_bottom(const LevelArgs<T> &L, int sweeps, hipStream_t st) {
    hipLaunchKernelGGL(k_bottom<T>, dim3(1), dim3(1024), 0, st, L, sweeps);
}

template <typename T>
void launch_update(double *phi, const T *e, int nx, int ny, int nzd, int kb, const int *pflags, double dmax,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_update<T>, plane_grid(nx, ny, nzd), dim3(BX, BY), 0, st, phi, e, nx, ny, kb, pflags, dmax);
}

void launch_reduce_norms(const double *part, int nblocks, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_norms, dim3(1), dim3(1024), 0, st, part, nblocks, out);
}

void launch_fill(double *x, size_t n, double v, hipStream_t st) {
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, x, n, v);
}

#define FX_INST(T)                                                                                         \
    template void launch_residual<T>(const ResArgs<T> &, hipStream_t, int *);                               \
    template void launch_smooth<T>(const LevelArgs<T> &, int, int, hipStream_t);                            \
    template void launch_restrict<T>(const RestrictArgs<T> &, hipStream_t);                                 \
    template void launch_prolong<T>(const ProlongArgs<T> &, hipStream_t);                                   \
    template void launch_bottom<T>(const LevelArgs<T> &, int, hipStream_t);                                 \
    template void launch_update<T>(double *, const T *, int, int, int, int, const int *, double, hipStream_t);
FX_INST(double)
FX_INST(float)

}  // namespace fx
