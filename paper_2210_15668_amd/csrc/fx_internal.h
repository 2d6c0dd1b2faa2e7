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

constexpr int kMaxLevels = 24;

// Device-side state of one Poisson solve.  done: 0 running, 1 converged,
// 2 non-finite residual, 3 cycle budget exhausted.  Kernels of a cycle
// return immediately once done != 0, so cycles can be enqueued ahead of the
// host's convergence check.
struct SolveCtrl {
    int done;
    int cycles;
    int max_cycles;
    int pad;
    double tol2;       // tol_rel^2
    double rn2, fn2;   // ||r||^2, ||f||^2 of the latest residual (scaled units)
};

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

// One multigrid level as the kernels see it.  Storage of e and r: with rb
// set (nx even, ny even or 1: a proper red/black colouring under periodic
// wrap) the cells of colour (i+j+k)&1 == 0 come first, then colour 1, each
// in z-major row order; otherwise plain z-major order.  sig holds planes
// [sig_lo, sig_hi) in the same arrangement.  Every level has fewer than
// 2^31 cells, so all indices are 32-bit.
template <typename T>
struct LevelArgs {
    int nx, ny, nz, rb;
    const T *cxy, *czm, *czp, *dg;   // per-plane coefficients (scaled by h^2/eps0)
    T *e;
    T *r;
    T *sig;
    int sig_lo, sig_hi;
};

// Transfer tables between a level and the next coarser one.
template <typename T>
struct XferArgs {
    const int *cks, *ccnt;           // coarse plane K covers fine planes cks[K] .. cks[K]+ccnt[K]-1
    const int *fthick, *cthick;      // plane thickness in finest planes
    const int *pka, *pkb;            // coarse planes interpolated into each fine plane (pkb -1: contact)
    const T *pwa, *pwb;
    int xy;                          // x and y halved
};

// ------------------------------------------------- fine-level residual (FP64)
// phi_out = phi_in + clip(e) (when e is given), then r = s (f - N(phi_out))
// on the device slab and sigma = s e (p + n) / VT on semiconductor planes;
// s = h^2/eps0.  Per-tile partial sums of r^2 and (s f)^2.
template <typename T>
struct ResArgs {
    int nx, ny, nzd, kb;
    double v_b, v_t;
    double p_scale;              // h / eps0
    double rho_scale;            // h^2 / eps0
    double vt_inv;               // 1 / VT
    double sig_scale;            // (h^2/eps0) / VT
    double dmax;                 // Newton update clip on semiconductor planes
    const double *cxy, *czm, *czp;   // scaled, per device plane
    const double *wl, *wr;           // P face weights of the face above plane k
    const double *p0e, *n0e;         // e * p0, e * n0 per device plane
    const int *pflags;
    const double *phi_in;            // full grid
    double *phi_out;                 // full grid (written when e is given)
    const T *e;                      // level-0 correction or nullptr
    const double *P;                 // full grid
    LevelArgs<T> L0;                 // r and sig written
    double *part;
    const SolveCtrl *ctrl;
};
template <typename T> int launch_residual(const ResArgs<T> &a, hipStream_t st);

// Newton update folded into the last black half-sweep of the finest level:
// phi_out = phi_in + clip(e) for each black cell and its red partner (the
// pair 2m, 2m+1 of a row), pointers at the device slab.
struct UpdArgs {
    const double *phi_in;
    double *phi_out;
    const int *pflags;
    double dmax;
};

// ev0/ev1 (optional): HIP events the dispatch itself timestamps.
template <typename T> void launch_smooth(const LevelArgs<T> &L, int color, int zero_init, const SolveCtrl *ctrl,
                                         hipStream_t st, const UpdArgs *upd = nullptr, hipEvent_t ev0 = nullptr,
                                         hipEvent_t ev1 = nullptr);
template <typename T> void launch_restrict(const LevelArgs<T> &F, const LevelArgs<T> &C, const XferArgs<T> &X,
                                           const SolveCtrl *ctrl, hipStream_t st);
template <typename T> void launch_prolong(const LevelArgs<T> &F, const LevelArgs<T> &C, const XferArgs<T> &X,
                                          const SolveCtrl *ctrl, hipStream_t st);

// All levels from the first one handed over down to the coarsest, in one
// workgroup with every level resident in LDS: lv[0] is the handed-over level
// (its r and sig are copied in from r_in / sig_in, its correction copied out
// to e_out), xf[l] links lv[l] and lv[l+1].  off_* are byte offsets of each
// level's arrays in the dynamic LDS allocation of lds_bytes.
template <typename T>
struct CoarseArgs {
    int nlev, nu1, nu2, bottom_sweeps;
    int lds_bytes;
    LevelArgs<T> lv[kMaxLevels];
    XferArgs<T> xf[kMaxLevels];
    int off_e[kMaxLevels], off_r[kMaxLevels], off_s[kMaxLevels], off_t[kMaxLevels];
    const T *r_in;
    const T *sig_in;
    T *e_out;
};
template <typename T> void launch_coarse(const CoarseArgs<T> *dev_args, int lds_bytes, const SolveCtrl *ctrl,
                                         hipStream_t st);
constexpr int kCoarseLdsBytes = 64 * 1024;

void launch_reduce(const double *part, int nparts, SolveCtrl *ctrl, int count_cycle, hipStream_t st);
void launch_ctrl_reset(SolveCtrl *ctrl, int max_cycles, double tol2, hipStream_t st);
struct ExtrapArgs {
    int nin;
    double c[4];
    const double *in[4];
};
void launch_extrap(double *out, const ExtrapArgs &a, size_t n, hipStream_t st);
void launch_fill(double *x, size_t n, double v, hipStream_t st);

}  // namespace fx
