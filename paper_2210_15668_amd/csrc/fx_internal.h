// Internal declarations shared by the HIP kernels and the host engine.
//
// Every kernel is multi-instance: one launch covers the tiles of all
// instances of a batch (a single stack is a batch of one).  A launch gets the
// instance array and a prefix table of per-instance tile counts, and decodes
// its block into (instance, local tile).  All per-solve control -- which phi
// buffer holds which iterate, the stop decision, the stored time levels --
// lives in device memory (InstState), so a whole time step can be enqueued,
// or captured in a HIP graph, without a host decision inside it.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace fx {

// Physical constants (CODATA 2018).
constexpr double kQe = 1.602176634e-19;
constexpr double kKb = 1.380649e-23;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kHbar = 1.054571817e-34;
constexpr double kMe0 = 9.1093837015e-31;

// Fermi-Dirac integral of order 1/2, normalised to e^eta for eta -> -inf, in the
// closed form of Bednarczyk and Bednarczyk (1978): F = 1/(e^-eta + xi),
// xi = (3 sqrt(pi)/4) nu^(-3/8), nu = eta^4 + 50 + 33.6 eta (1 - 0.68 e^(-0.17 (eta+1)^2)),
// and dF/deta of that expression (written so that nothing overflows for eta >= -700).
__host__ __device__ inline void fd_half(double eta, double &F, double &dF) {
    eta = fmax(eta, -700.0);
    const double a = eta + 1.0;
    const double g = exp(-0.17 * a * a);
    const double s = 1.0 - 0.68 * g;
    const double e2 = eta * eta;
    const double nu = e2 * e2 + 50.0 + 33.6 * eta * s;
    const double dnu = 4.0 * e2 * eta + 33.6 * s + 7.76832 * eta * a * g;
    const double xi = 1.329340388179137 * exp(-0.375 * log(nu));
    const double dxi = -0.375 * xi * dnu / nu;
    const double em = exp(-eta);
    const double f = 1.0 / (em + xi);
    F = f;
    dF = (em * f - dxi * f) * f;
}

// Per-plane flag bits of the finest (device) level.
enum : int { PF_SC = 1, PF_P = 2 };

constexpr int kMaxLevels = 24;
constexpr double kLightRatio = 5.0;        // see InstState::light
constexpr double kLightContraction = 6.0;  // the cycle before reduced ||r|| at least this much
constexpr int kMaxOrder = 3;      // highest order of the extrapolated starting iterate
constexpr int kPhiBufs = 8;       // phi^n, up to 3 stored levels, two iterate buffers; for
                                  // predictor-corrector instances a fourth stored level (the
                                  // corrector extrapolates through phi^n .. phi^{n-3}) and
                                  // the last predictor's phi*
constexpr int kMaxHist = 4;       // stored levels of a predictor-corrector instance (Euler: 3)
constexpr int kCoarseLdsBytes = 64 * 1024;
// temporal blocking of the smoothing below the finest level (k_pre_tb / k_post_tb)
constexpr int kTbT = 8;                    // tile edge (cells)
constexpr int kTbH = 4;                    // ring (cells): 2 nu for nu <= 2 sweeps
constexpr int kTbW = kTbT + 2 * kTbH;      // box edge; a thread per box column
constexpr int kTbMaxNz = 30;               // planes of a blocked level (a column's values in registers)
constexpr int kTbLdsBytes = 64 * 1024;     // largest box (all planes of a level) and its tables
constexpr int kQvBlocks = 8;      // blocks per instance of the interface-plane reductions
constexpr int kRecSteps = 1024;   // recorded steps per instance held on the device

// Mutable per-instance state of the current solve and of the time history.
// Every instance runs its own state machine, driven by two kinds of slots:
//  - an advance slot finalizes a solve that has stopped (history, status,
//    step count) and, in a run, starts the next time step of instances that
//    have not reached their target: TDGL update, flip of the P buffers,
//    starting iterate, first residual;
//  - a cycle slot performs one multigrid cycle + residual for every
//    instance whose solve is still running.
// A run is then a fixed sequence of slots (one advance slot, then pairs of
// cycle and advance slots) that needs no host decision between its kernels.
// done: 0 running, 1 converged, 2 non-finite residual, 3 cycle budget used.
struct InstState {
    int done, cycles;
    int cur, start, oth0, oth1;       // phi buffers: phi^n, iterate before cycle 0, cycle outputs
    int prev[kMaxHist], hist;         // stored time levels phi^{n-1..n-4}
    int order;                        // extrapolation order of this solve
    int zpend;                        // right-hand side exactly zero with a nonzero residual
    int zero_fix;                     // the solve finalized in this slot had f = 0 exactly (its
                                      // last iterate was set to 0 when it stopped)
    int status;                       // fx_status of the last finalized solve
    int step, target, sched_base, sched_len;
    int pcur;                         // P buffer holding the current P
    int ts;                           // the running solve belongs to a time step
    int phase;                        // second-order steps: 0 predictor (or Euler), 1 corrector
    int corr;                         // runs the corrector update in this advance slot
    int pstar;                        // buffer of the last step's predictor phi* (-1: none)
    int usestar;                      // this solve starts from the extrapolation + phi* - phi^n
    int stepped;                      // a time step was completed in this advance slot
    int fresh;                        // solve started in this slot (first residual pending)
    int insolve;                      // a solve is running or awaits finalization
    int light;                        // this cycle skips one pre- and one post-smoothing sweep
                                      // per level: the last one left ||r|| within kLightRatio
                                      // of the tolerance after a kLightContraction-fold cut
    int adv;                          // starts a time step in this advance slot
    int parked;                       // run target reached or a solve failed
    int solves, failed, total_cycles, max_cycles_step;
    double v_top;                     // gate potential of the current solve
    double dt;                        // time step of the run
    double rn2, fn2;                  // ||r||^2, ||f||^2 of the latest residual (scaled units)
};

// One multigrid level.  Storage of e and r: with rb set (nx even, ny even or
// 1: a proper red/black colouring under periodic wrap) the cells of colour
// (i+j+k)&1 == 0 come first, then colour 1, each in z-major row order;
// otherwise plain z-major order.  sig holds planes [sig_lo, sig_hi) in the
// same arrangement.  Every level has fewer than 2^31 cells (32-bit indices).
template <typename T>
struct LevelArgs {
    int nx, ny, nz, rb;
    const T *cxy, *czm, *czp, *dg;   // per-plane coefficients (scaled by h^2/eps0)
    T *e;
    T *r;
    T *sig;
    int sig_lo, sig_hi;
    T *ealt;                         // black values between the blocked pre- and post-smoothing (or null)
};

// Transfer tables between a level and the next coarser one.
template <typename T>
struct XferArgs {
    const int *cks, *ccnt;           // coarse plane K covers fine planes cks[K] .. cks[K]+ccnt[K]-1
    const int *fthick, *cthick;      // plane thickness in finest planes
    const int *pka, *pkb;            // coarse planes interpolated into each fine plane (pkb -1: contact)
    const T *pwa, *pwb;
    int xy;                          // lateral transfer: 0 none, 1 x and y halved, 2 x halved (one row)
};

// Constant description of one instance (device memory, read by every kernel).
template <typename T>
struct Inst {
    int nx, ny, nz, kb, nzd, f0, f1;   // full grid, device slab [kb, kb+nzd), ferroelectric [f0, f1)
    int nlev, lc, fold;                // levels; first level of the coarse kernel; update folded into smoothing
    int max_cycles, warm;
    int order2;                        // predictor-corrector time steps
    int nbuf;                          // phi buffers in use (kPhiBufs - 2 without order2)
    int light_ok;                      // light cycles allowed (InstState::light)
    double light_r2, light_c2;         // squares of kLightRatio and kLightContraction
    double tol2;
    // TDGL
    double h, alpha, beta, gamma, g11, g44, Gamma, lambda;
    int pbc;
    // residual (scaled by s = h^2/eps0)
    double v_b, p_scale, rho_scale, vt_inv, sig_scale, dmax;
    const double *cxy0, *czm0, *czp0, *wl, *wr, *p0e, *n0e;
    // Fermi-Dirac carriers (fd): p0e, n0e hold e Nv, e Nc; fdt holds per plane
    // eta_p0, eta_n0, F(eta_p0), F(eta_n0)
    int fd;
    const double *fdt;
    const int *pflags;
    const double *vsched;              // gate potentials of the run's steps (sched_len entries)
    double *phi[kPhiBufs];
    double *P[2];
    double *part;                      // residual partial sums, 2 per residual tile
    // Q-V diagnostics: the ferroelectric/dielectric face between planes qv_kl and qv_kl + 1
    // (qv_kl < 0: none), the ferroelectric on its upper side if qv_fe_up; eps0 eps_r of
    // both planes; partial sums (2 per block) and the per-step record (Q, V_fe pairs)
    int qv_kl, qv_fe_up;
    double qv_el, qv_er;
    double *qv_part;
    double *qv_rec;
    InstState *st;
    // multigrid
    LevelArgs<T> lv[kMaxLevels];
    XferArgs<T> xf[kMaxLevels];
    int nu1, nu2, lds_bytes;
    int off_e[kMaxLevels], off_r[kMaxLevels], off_s[kMaxLevels], off_t[kMaxLevels];
    int off_x[kMaxLevels];             // transfer tables between coarse-kernel levels q and q+1
    // conjugate-gradient bottom solve: search direction, product, reduction scratch (LDS offsets)
    int off_p, off_q, off_red;
    int bottom_iters;
    double bottom_tol2;
};

// A launch over all instances: prefix[i] .. prefix[i+1] are instance i's tiles.
struct Work {
    const int *prefix;
    int ninst;
    int total;
    InstState *st;                     // the instances' states (InstState[ninst])
};

// ------------------------------------------------------------------ launchers
// sel = 1 restricts a launch to the instances starting a time step in the
// current advance slot; sel = 0 covers every instance.
template <typename T> void launch_tdgl(const Inst<T> *I, const Work &w, int sel, hipStream_t st);
// corrector of a second-order step, for the instances flagged in this advance slot:
// P^n := (P^n + P*)/2 + dt/2 f(P*, phi*), in the buffer that holds P^n
template <typename T> void launch_tdgl_corr(const Inst<T> *I, const Work &w, hipStream_t st);
template <typename T> void launch_flip(const Inst<T> *I, int ninst, hipStream_t st);
// Interface charge Q and average ferroelectric voltage V_fe.  record 0: every instance's
// current state into out[2 i], out[2 i + 1] (NaN without an interface); record 1: the
// instances that completed a time step in this advance slot, into their per-step record.
template <typename T> void launch_qv(const Inst<T> *I, int ninst, int record, double *out, hipStream_t st);
template <typename T> void launch_begin(const Inst<T> *I, InstState *S, int ninst, int sel, hipStream_t st);
template <typename T> void launch_extrap(const Inst<T> *I, const Work &w, hipStream_t st);
// Work tables of the residual: cell0 -- every instance (mode 0, the current
// iterate; after a cycle the kernel skips the instances of cell2); cell2 --
// instances whose update is not folded into the smoother (mode 2: forms
// phi_in + clip(e) itself, after a cycle).
struct ResWork {
    Work cell0, cell2;
};
// after_cycle 0: residual at the starting iterate of freshly begun solves;
// 1: at the output of the cycle just run (forming phi_in + clip(e) first
// where the update is not folded into the smoother).
// any_fd: some instance takes Fermi-Dirac carriers (else the kernel without that branch)
template <typename T> void launch_residual(const Inst<T> *I, const ResWork &w, int after_cycle, int any_fd, hipStream_t st);
template <typename T> void launch_reduce(const Inst<T> *I, InstState *S, int ninst, int count_cycle, hipStream_t st);
// Launch shape of one level's smoother: tile of 2^lbx x 2^(8-lbx) threads,
// zt planes per thread, w8: register budget for 8 waves per SIMD.  Only the
// division of the work changes, never a cell's arithmetic.
struct SmoothCfg {
    int lbx, zt, w8;
};
// skip_light: the launch is one of the sweeps a light cycle leaves out
template <typename T> void launch_smooth(const Inst<T> *I, const Work &w, int level, int color, int zero_init,
                                         int upd, const SmoothCfg &c, double *probe, hipStream_t st,
                                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int skip_light = 0);
// the first two half-sweeps of a cycle on a level stored red/black at every
// instance (zero start, red then black) as one launch; the same values as the
// two separate launches
template <typename T> void launch_smooth_zpair(const Inst<T> *I, const Work &w, int level, const SmoothCfg &c,
                                               hipStream_t st);
// prolongation into a level stored red/black at every instance fused with the
// red half-sweep after it (the corrected black values are not stored: the
// black half-sweep that follows overwrites them without reading them)
template <typename T> void launch_prolong_red(const Inst<T> *I, const Work &w, int level, const SmoothCfg &c,
                                              hipStream_t st);
template <typename T> void launch_restrict(const Inst<T> *I, const Work &w, int level, hipStream_t st);
template <typename T> void launch_prolong(const Inst<T> *I, const Work &w, int level, hipStream_t st);
// the same prolongation by coarse columns, for red/black levels halved in x and y and
// paired in z (the work table counts exactly those instances' tiles)
template <typename T> void launch_prolong_cc(const Inst<T> *I, const Work &w, int level, int cz, hipStream_t st);
template <typename T> void launch_coarse(const Inst<T> *I, InstState *S, int ninst, int lds_bytes, hipStream_t st);
// pre-smoothing (nu zero-start sweeps) + restriction of level `level`, and prolongation +
// post-smoothing (nu sweeps), a block per kTbT x kTbT tile with lds_bytes of LDS
template <typename T> void launch_pre_tb(const Inst<T> *I, const Work &w, int level, int nu, int lds_bytes, hipStream_t st);
template <typename T> void launch_post_tb(const Inst<T> *I, const Work &w, int level, int nu, int lds_bytes, hipStream_t st);
template <typename T> void launch_head(const Inst<T> *I, InstState *S, int ninst, int advance, hipStream_t st);
template <typename T> void launch_run_setup(const Inst<T> *I, int ninst, int nsteps, int has_sched, double dt,
                                            int first, hipStream_t st);
template <typename T> void launch_set_vtop(const Inst<T> *I, int ninst, double v, hipStream_t st);
void launch_put_state(InstState *dst, const InstState &v, hipStream_t st);
void launch_fill(double *x, size_t n, double v, hipStream_t st);
void launch_zero(void *x, size_t bytes, hipStream_t st);          // bytes: a multiple of 4

// Host-side tile counts (must match the kernels' decoding).
constexpr int BX = 64;
constexpr int BY = 4;
__host__ __device__ inline int tiles3(int nxw, int ny, int nz) { return ((nxw + BX - 1) / BX) * ((ny + BY - 1) / BY) * nz; }
inline int tiles_cfg(int nxw, int ny, int nz, const SmoothCfg &c) {
    const int bx = 1 << c.lbx, by = 256 >> c.lbx;
    return ((nxw + bx - 1) / bx) * ((ny + by - 1) / by) * ((nz + c.zt - 1) / c.zt);
}
constexpr int kResZ = 4;            // planes per thread in the fine-level residual
constexpr int kProZ = 4;            // planes per thread in the prolongation kernel
constexpr int kProCZ = 4;           // coarse planes per thread in the coarse-column prolongation
                                    // into a level of at least kProCZBig coarse cells (else 1)
constexpr size_t kProCZBig = (size_t)1 << 19;
constexpr int kExtrapChunk = 1024;  // cells per extrapolation tile

}  // namespace fx
