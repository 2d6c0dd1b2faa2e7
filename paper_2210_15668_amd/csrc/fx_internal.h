// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace fx {

// Physical constants (CODATA 2018).
constexpr double kQe = 1.602176634e-19;
constexpr double kKb = 1.380649e-23;
constexpr double kEps0 = 8.8541878128e-12;

// Per-plane flag bits of the finest (device) level.
enum : int { PF_SC = 1, PF_P = 2 };

// --------------------------------------------------------------------- TDGL
struct TdglArgs {
    int nx, ny, f0, f1;          // ferroelectric planes [f0, f1) of the full grid
    double h, dt;
    double alpha, beta, gamma, g11, g44, Gamma;
    int pbc;
    double lambda;
    const double *P;
    const double *phi;
    double *Pn;
};
void launch_tdgl(const TdglArgs &a, hipStream_t st);

// ------------------------------------------------- fine-level residual (FP64)
// r = s (f - N(phi)) on the device slab (planes kb .. kb+nzd-1 of the full
// grid), sigma = s e (p + n) / VT on the semiconductor planes; s = h^2/eps0.
// Coefficient tables are in the same scaled units.  Per-block partial sums
// of r^2 and (s f)^2 go to part[2*b], part[2*b+1].
template <typename T>
struct ResArgs {
    int nx, ny, nzd, kb;
    double v_b, v_t;
    double p_scale;              // h / eps0   (scale * (1/h) for the bound-charge term)
    double rho_scale;            // h^2 / eps0
    double vt_inv;               // 1 / VT
    double sig_scale;            // (h^2/eps0) * e / VT
    const double *cxy, *czm, *czp;   // scaled, per device plane
    const double *wl, *wr;           // P face weights of the face above plane k
    const double *p0e, *n0e;         // e * p0, e * n0 per device plane
    const int *pflags;
    const double *phi;               // full grid
    const double *P;                 // full grid
    T *r;
    T *sig;
    int sig_lo, sig_hi;
    double *part;
};
template <typename T> void launch_residual(const ResArgs<T> &a, hipStream_t st, int *nblocks);

// --------------------------------------------------------------- multigrid
template <typename T>
struct LevelArgs {
    int nx, ny, nz;
    const T *cxy, *czm, *czp, *dg;   // per plane
    T *e;
    T *r;
    T *sig;
    int sig_lo, sig_hi;
};

template <typename T> void launch_smooth(const LevelArgs<T> &L, int color, int zero_init, hipStream_t st);

template <typename T>
struct RestrictArgs {
    LevelArgs<T> f;                  // fine level (e, r, sig read)
    LevelArgs<T> c;                  // coarse level (r, sig written)
    const int *fthick;               // fine plane thickness (finest-level planes)
    const int *cthick;
    const int *cks, *ccnt;           // coarse plane K covers fine planes cks[K] .. cks[K]+ccnt[K]-1
    int xy;                          // 1 if x and y are coarsened
};
template <typename T> void launch_restrict(const RestrictArgs<T> &a, hipStream_t st);

template <typename T>
struct ProlongArgs {
    LevelArgs<T> f;                  // fine level e updated
    LevelArgs<T> c;                  // coarse level e read
    const int *ka, *kb;              // coarse planes for each fine plane (kb = -1: boundary, value 0)
    const T *wa, *wb;
    int xy;
};
template <typename T> void launch_prolong(const ProlongArgs<T> &a, hipStream_t st);

template <typename T> void launch_bottom(const LevelArgs<T> &L, int sweeps, hipStream_t st);

// phi[kb*nxy + c] += clip(e[c]) on the device slab; clip to +-dmax on planes flagged PF_SC.
template <typename T>
void launch_update(double *phi, const T *e, int nx, int ny, int nzd, int kb, const int *pflags, double dmax,
                   hipStream_t st);

void launch_reduce_norms(const double *part, int nblocks, double *out, hipStream_t st);
void launch_fill(double *x, size_t n, double v, hipStream_t st);

}  // namespace fx
