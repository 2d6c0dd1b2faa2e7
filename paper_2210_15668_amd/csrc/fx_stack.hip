// Host driver and C ABI: descriptor validation, multigrid hierarchy and
// per-plane tables, the Newton / multigrid Poisson solve, the time loop.
//
// Poisson discretisation (eq. (Poisson) with eq. (rho), Dirichlet contacts
// and periodic x/y of the "Electrical boundary conditions" section): finite
// volumes with D_z = -eps dphi/dz + P continuous across each z-face.  For a
// face between planes L and R the face permittivity is the series value
// 2 eps_L eps_R / (eps_L + eps_R) and the face polarisation is
// (eps_R P_L + eps_L P_R) / (eps_L + eps_R); contact faces sit at h/2 with
// the cell's own eps and P.  The nonlinear system N(phi) = L phi - rho_c(phi)
// = f is solved by Newton, each Newton correction taking one multigrid
// V-cycle on (L + diag sigma) e = f - N(phi), sigma = -d rho_c/d phi.
//
// Multigrid: cell-centred geometric coarsening.  x and y halve together
// while both are even and >= 4; z pairs planes (the top coarse plane keeps a
// single plane when the count is odd), so coarse cells may have unequal
// thickness.  Because the permittivity only varies with z, every level's
// operator is described by per-plane tables: the x/y coefficient is the
// thickness-mean permittivity over the covered finest planes, and each
// z-face coefficient is the series conductance of the finest half-planes
// between the two coarse cell centres.  Restriction is the volume-weighted
// mean.  Prolongation is bilinear in x/y and, in z, linear in the series
// resistance between the two nearest coarse centres (or the contact face,
// where the correction is zero) -- the flux-continuous interpolant of a
// layered medium, which keeps the V-cycle contraction near 0.1 across the
// permittivity jumps where distance-linear weights stall near 0.2.
#include "fx_internal.h"
#include "fx_unet_internal.h"
#include "../../include/ferrox.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

using namespace fx;

namespace {

thread_local std::string g_err;

fx_status fail(fx_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
fx_status fail(fx_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_OK(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(FX_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)

}  // namespace

void fx::set_error(const char *msg) { g_err = msg; }

namespace {

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

constexpr int kBottomTarget = 8;         // stop coarsening at this many cells

// One multigrid level, host view.
struct HostLevel {
    int nx = 0, ny = 0, nz = 0;
    int xy_from_finer = 0;              // relative to the finer level: 1 x and y halved, 2 x halved
                                        // (a single row: ny = 1), 0 neither
    int z_from_finer = 0;               // z paired relative to the finer level
    std::vector<int> s0, e0;            // covered finest device planes [s0, e0)
    std::vector<double> cxy, czm, czp, dg;
    std::vector<int> ks, cnt;           // restriction map from the finer level
    std::vector<int> pka, pkb;          // prolongation map of the finer level's planes
    std::vector<double> pwa, pwb;
    int sig_lo = 0, sig_hi = 0;
    int rb = 0;                         // red/black-split storage (nx even)
    size_t ncell() const { return (size_t)nx * ny * nz; }
    size_t nsig() const { return (size_t)nx * ny * (sig_hi - sig_lo); }
};

struct Plan {
    int nx, ny, nz, kb, kt, nzd, f0, f1, sc0, sc1;
    int lc;                             // first level handled by the one-workgroup coarse kernel
    std::vector<HostLevel> lv;
};

// Bump allocator over the caller's workspace (256-byte alignment).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    void *take(size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

template <typename T>
struct DevLevel {
    T *e = nullptr, *r = nullptr, *sig = nullptr;
    T *cxy = nullptr, *czm = nullptr, *czp = nullptr, *dg = nullptr;
    T *pwa = nullptr, *pwb = nullptr;
    int *ks = nullptr, *cnt = nullptr, *thick = nullptr, *pka = nullptr, *pkb = nullptr;
    T *ealt = nullptr;                  // blocked smoothing's black values (levels that may use it)
};


fx_status validate(const fx_stack_desc *d, Plan *p) {
    if (!d) return fail(FX_EINVAL, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(FX_EINVAL, "grid sizes must be >= 1");
    if ((double)d->nx * d->ny * d->nz >= 2147483647.0) return fail(FX_EINVAL, "grid must have < 2^31 cells");
    if (!(d->h > 0) || !(d->Gamma > 0) || !(d->gamma > 0))
        return fail(FX_EINVAL, "h, Gamma and gamma must be > 0");
    if (d->pbc < 0 || d->pbc > 2) return fail(FX_EINVAL, "unknown pbc %d", d->pbc);
    if (d->pbc == FX_PBC_LAMBDA && !(d->lambda >= 0)) return fail(FX_EINVAL, "lambda must be >= 0");
    if (!d->plane_mat || !d->plane_eps_r || !d->plane_Na || !d->plane_Nd)
        return fail(FX_EINVAL, "plane tables must not be NULL");
    if (d->prec != FX_PREC_FP64 && d->prec != FX_PREC_MIXED) return fail(FX_EINVAL, "unknown precision");
    if (!(d->tol_rel > 0) || d->max_cycles < 1) return fail(FX_EINVAL, "tol_rel > 0 and max_cycles >= 1 required");
    if (d->warm_start < 0 || d->warm_start > kMaxOrder)
        return fail(FX_EINVAL, "warm_start must be 0..%d", kMaxOrder);
    if (d->time_order < 0 || d->time_order > 2) return fail(FX_EINVAL, "time_order must be 0, 1 or 2");
    if (d->carriers != FX_CARRIERS_BOLTZMANN && d->carriers != FX_CARRIERS_FD)
        return fail(FX_EINVAL, "carriers must be FX_CARRIERS_BOLTZMANN or FX_CARRIERS_FD");
    if (d->carriers == FX_CARRIERS_FD && !(d->m_e > 0 && d->m_p > 0 && d->Eg > 0))
        return fail(FX_EINVAL, "Fermi-Dirac carriers need m_e, m_p, Eg > 0");
    p->nx = d->nx; p->ny = d->ny; p->nz = d->nz;
    p->kb = -1; p->kt = -1; p->f0 = -1; p->f1 = -1; p->sc0 = -1; p->sc1 = -1;
    bool any_sc = false;
    for (int k = 0; k < d->nz; ++k) {
        const int m = d->plane_mat[k];
        if (m < 0 || m > 3) return fail(FX_EINVAL, "plane %d: unknown material %d", k, m);
        if (m != FX_MAT_METAL) {
            if (p->kb < 0) p->kb = k;
            p->kt = k + 1;
            if (!(d->plane_eps_r[k] > 0)) return fail(FX_EINVAL, "plane %d: eps_r must be > 0", k);
        }
        if (m == FX_MAT_SC) any_sc = true;
    }
    if (p->kb < 0) return fail(FX_EINVAL, "no device planes");
    for (int k = p->kb; k < p->kt; ++k)
        if (d->plane_mat[k] == FX_MAT_METAL) return fail(FX_EINVAL, "metal plane %d inside the device", k);
    for (int k = p->kb; k < p->kt; ++k) {
        if (d->plane_mat[k] == FX_MAT_FE) { if (p->f0 < 0) p->f0 = k; p->f1 = k + 1; }
        if (d->plane_mat[k] == FX_MAT_SC) { if (p->sc0 < 0) p->sc0 = k; p->sc1 = k + 1; }
    }
    if (p->f0 >= 0) {
        for (int k = p->f0; k < p->f1; ++k)
            if (d->plane_mat[k] != FX_MAT_FE) return fail(FX_EINVAL, "ferroelectric planes must be contiguous");
        if (p->f1 - p->f0 < 3) return fail(FX_EINVAL, "ferroelectric needs >= 3 planes");
    }
    if (any_sc) {
        if (!(d->T > 0) || (d->carriers != FX_CARRIERS_FD && !(d->ni > 0)))
            return fail(FX_EINVAL, "T (and ni, for Boltzmann carriers) must be > 0 with a semiconductor");
        for (int k = p->sc0; k < p->sc1; ++k)
            if (d->plane_mat[k] != FX_MAT_SC) return fail(FX_EINVAL, "semiconductor planes must be contiguous");
    }
    p->nzd = p->kt - p->kb;
    return FX_OK;
}

// Series resistance (in units of h / eps0) of finest planes over [za, zb] (units of h).
double series_R(const std::vector<double> &epsd, double za, double zb) {
    double R = 0.0;
    const int i0 = (int)std::floor(za), i1 = (int)std::ceil(zb);
    for (int i = i0; i < i1; ++i) {
        const double lo = std::max(za, (double)i), hi = std::min(zb, (double)(i + 1));
        if (hi > lo) R += (hi - lo) / epsd[i];
    }
    return R;
}

void build_plan(const fx_stack_desc *d, Plan *p) {
    std::vector<double> epsd(p->nzd);
    for (int k = 0; k < p->nzd; ++k) epsd[k] = d->plane_eps_r[p->kb + k];
    p->lv.clear();
    HostLevel L0;
    L0.nx = p->nx; L0.ny = p->ny; L0.nz = p->nzd;
    for (int k = 0; k < p->nzd; ++k) { L0.s0.push_back(k); L0.e0.push_back(k + 1); }
    if (p->sc0 >= 0) { L0.sig_lo = p->sc0 - p->kb; L0.sig_hi = p->sc1 - p->kb; }
    p->lv.push_back(L0);
    for (;;) {
        const HostLevel &F = p->lv.back();
        if (F.ncell() <= (size_t)env_int("FERROX_BOTTOM_CELLS", kBottomTarget)) break;
        const bool cxy = F.nx % 2 == 0 && F.ny % 2 == 0 && F.nx >= 4 && F.ny >= 4;
        // a single row (the 2D x-z reduction) halves x alone
        const bool cx1 = !cxy && F.ny == 1 && F.nx % 2 == 0 && F.nx >= 4;
        const bool cz = F.nz >= 2;
        if (!cxy && !cx1 && !cz) break;
        HostLevel C;
        C.xy_from_finer = cxy ? 1 : (cx1 ? 2 : 0);
        C.z_from_finer = cz;
        C.nx = cxy || cx1 ? F.nx / 2 : F.nx;
        C.ny = cxy ? F.ny / 2 : F.ny;
        C.nz = cz ? (F.nz + 1) / 2 : F.nz;
        for (int K = 0; K < C.nz; ++K) {
            const int ks = cz ? 2 * K : K;
            const int cnt = cz ? std::min(2, F.nz - ks) : 1;
            C.ks.push_back(ks); C.cnt.push_back(cnt);
            C.s0.push_back(F.s0[ks]); C.e0.push_back(F.e0[ks + cnt - 1]);
        }
        if (F.sig_hi > F.sig_lo) {
            C.sig_lo = cz ? F.sig_lo / 2 : F.sig_lo;
            C.sig_hi = cz ? (F.sig_hi + 1) / 2 : F.sig_hi;
        }
        p->lv.push_back(C);
        if ((int)p->lv.size() >= kMaxLevels) break;
    }
    const int nlev = (int)p->lv.size();
    // red/black split storage needs a proper 2-colouring under periodic wrap
    for (int l = 0; l < nlev; ++l)
        p->lv[l].rb = p->lv[l].nx % 2 == 0 && (p->lv[l].ny % 2 == 0 || p->lv[l].ny == 1);
    // the coarse kernel keeps levels lc.. in LDS
    const size_t w = d->prec == FX_PREC_MIXED ? sizeof(float) : sizeof(double);
    p->lc = nlev - 1;
    size_t tail = 0;
    for (int l = nlev - 1; l >= 0; --l) {
        const HostLevel &L = p->lv[l];
        tail += (2 * L.ncell() + L.nsig() + 4 * L.nz) * w + 64;
        if (l == nlev - 1) tail += 2 * L.ncell() * w + 16 * sizeof(double) + 64;   // bottom-solve vectors
        else tail += 3 * (L.nz + p->lv[l + 1].nz) * sizeof(int) + 2 * L.nz * w + 48;  // transfer tables
        if (tail > (size_t)kCoarseLdsBytes) break;
        p->lc = l;
    }
    int xy_pow = 0;
    for (int l = 0; l < nlev; ++l) {
        HostLevel &L = p->lv[l];
        if (l > 0 && L.xy_from_finer) ++xy_pow;
        const double hxy2 = std::pow(4.0, xy_pow);
        L.cxy.assign(L.nz, 0); L.czm.assign(L.nz, 0); L.czp.assign(L.nz, 0); L.dg.assign(L.nz, 0);
        std::vector<double> zc(L.nz);
        for (int K = 0; K < L.nz; ++K) zc[K] = 0.5 * (L.s0[K] + L.e0[K]);
        for (int K = 0; K < L.nz; ++K) {
            const double t = L.e0[K] - L.s0[K];
            double em = 0.0;
            for (int i = L.s0[K]; i < L.e0[K]; ++i) em += epsd[i];
            L.cxy[K] = em / t / hxy2;
            const double Rm = K == 0 ? series_R(epsd, 0.0, zc[0]) : series_R(epsd, zc[K - 1], zc[K]);
            const double Rp = K == L.nz - 1 ? series_R(epsd, zc[K], (double)p->nzd) : series_R(epsd, zc[K], zc[K + 1]);
            L.czm[K] = 1.0 / (Rm * t);
            L.czp[K] = 1.0 / (Rp * t);
            L.dg[K] = (L.nx > 1 ? 2.0 : 0.0) * L.cxy[K] + (L.ny > 1 ? 2.0 : 0.0) * L.cxy[K] + L.czm[K] + L.czp[K];
        }
        // prolongation map of the finer level l-1's planes from this level
        if (l > 0) {
            HostLevel &F = p->lv[l - 1];
            F.pka.assign(F.nz, 0); F.pkb.assign(F.nz, -1); F.pwa.assign(F.nz, 1.0); F.pwb.assign(F.nz, 0.0);
            for (int k = 0; k < F.nz; ++k) {
                const int K = L.z_from_finer ? k / 2 : k;
                const double zf = 0.5 * (F.s0[k] + F.e0[k]);
                F.pka[k] = K;
                if (zf == zc[K]) continue;
                double zn;
                int kn;
                if (zf < zc[K]) { kn = K - 1; zn = kn >= 0 ? zc[kn] : 0.0; }
                else { kn = K + 1 < L.nz ? K + 1 : -1; zn = kn >= 0 ? zc[kn] : (double)p->nzd; }
                // operator-dependent weights: linear in the series resistance
                // (potential of a constant D_z flux) between the two centres,
                // exact for the layered 1D problem across permittivity jumps
                const double ra = series_R(epsd, std::min(zf, zc[K]), std::max(zf, zc[K]));
                const double rn = series_R(epsd, std::min(zf, zn), std::max(zf, zn));
                const double wa = rn / (ra + rn);
                F.pwa[k] = wa;
                F.pwb[k] = 1.0 - wa;
                F.pkb[k] = kn;
            }
        }
    }
}


// ---------------------------------------------------------------- instances
// Host view of one instance: its plan, scaled constants and the device
// addresses carved from its region of the workspace.
struct InstHost {
    fx_stack_desc d{};
    std::vector<int> mat;
    std::vector<double> eps_r, Na, Nd;
    Plan plan{};
    double VT = 0.0, scale = 0.0, dmax = 0.0;
    // P: [0] the caller's array, [1] workspace.  phi: [0] the caller's array,
    // [1..5] workspace; which buffer holds phi^n and the stored time levels is
    // device state (InstState).
    double *P[2] = {nullptr, nullptr};
    double *phi[kPhiBufs] = {};
    double *t_cxy = nullptr, *t_czm = nullptr, *t_czp = nullptr, *t_wl = nullptr, *t_wr = nullptr;
    double *t_p0e = nullptr, *t_n0e = nullptr;
    double *t_fd = nullptr;             // Fermi-Dirac: 4 values per device plane
    int *t_flags = nullptr;
    std::vector<DevLevel<double>> L64;
    std::vector<DevLevel<float>> L32;
    double *part = nullptr;
    double *qv_part = nullptr, *qv_rec = nullptr;
    int lds = 0;                        // LDS bytes of this instance's coarse levels
    double filled_top = NAN;            // contact value last written into the caller's top metal planes
};

constexpr int kSchedChunk = 1024;       // schedule entries per instance held on the device
static_assert(kRecSteps == kSchedChunk, "the Q-V record covers one schedule chunk");
constexpr int kProbeMax = 4096;         // timed launches per probe
constexpr int kMaxBatch = 4096;
constexpr int kUnitPow = 5;             // captured unit graphs: 1, 2, 4, 8, 16 units

// A batch of instances (a single stack is a batch of one) sharing one
// precision, one stream and one launch sequence.
struct Engine {
    int n = 0;
    int prec = FX_PREC_FP64;
    hipStream_t st = nullptr;
    std::vector<InstHost> in;
    void *inst_dev = nullptr;           // Inst<T>[n]
    InstState *st_dev = nullptr;        // InstState[n]
    InstState *mir = nullptr;           // host mirror of the states, valid between calls: pinned,
                                        // or ordinary memory (mir_plain) for poisson_solve_static
    std::vector<InstState> mir_plain;
    int no_alloc = 0;                   // allocates no device or pinned memory (poisson_solve_static)
    int *prefix_dev = nullptr;
    double *sched_dev = nullptr;        // n x kSchedChunk gate potentials
    double *probe_dev = nullptr;        // kProbeMax byte counters
    double *qv_out = nullptr;           // n x (Q, V_fe) of the current state
    int rec = 0;                        // advance slots record Q and V_fe of completed steps
    int graphs_rec = 0;                 // the captured unit graphs include the recording
    std::vector<int> prefix_host;
    Work w_tdgl{}, w_ext{};
    ResWork w_res{};
    std::vector<Work> w_sm, w_rs, w_pr, w_prc;   // w_pr / w_prc: prolongation by fine or by coarse columns
    std::vector<Work> w_tb;             // blocked smoothing: a block per tile
    std::vector<int> tb, tb_lds;        // level smoothed in blocks; LDS bytes of its box
    std::vector<int> prc_cz;            // coarse planes per thread of w_prc, per level
    std::vector<SmoothCfg> scfg;        // smoother launch shape per level
    std::vector<int> ncol;
    std::vector<char> small;            // per level: few enough cells that launch latency dominates
    int max_lc = 0, lds_max = 0, max_cycles = 1;
    int any_order2 = 0;                 // some instance takes predictor-corrector steps
    int any_fd = 0;                     // some instance takes Fermi-Dirac carriers
    int nu1 = 2, nu2 = 2;               // sweeps before / after the coarse correction, finest level
    int nu1c = 2, nu2c = 2;             // the same on every coarser level
    int fuse = 1;                       // fused launches below the finest level (same values)
    int k_pred = 4;                     // cycles enqueued before the first check of a plain solve
    int trace = 0;
    int ucap = 16;                      // units enqueued between host checks of a run
    int mode = FX_LAUNCH_STREAM;
    // kernel-duration probe of the finest-level smoother
    int probe = 0;
    int probe_stride = 1, probe_seen = 0;
    std::vector<hipEvent_t> ev;         // pairs (start, stop)
    int ev_used = 0;
    // unit graphs (2^q units each) captured on a private stream
    hipStream_t cap = nullptr;
    hipGraphExec_t unit_exec[kUnitPow] = {};
};

fx_status validate_all(const fx_stack_desc *descs, int n, Engine *e) {
    if (!descs) return fail(FX_EINVAL, "desc is NULL");
    if (n < 1 || n > kMaxBatch) return fail(FX_EINVAL, "instance count %d outside 1..%d", n, kMaxBatch);
    e->n = n;
    e->in.assign(n, InstHost());
    e->prec = descs[0].prec;
    for (int i = 0; i < n; ++i) {
        InstHost &h = e->in[i];
        fx_status st = validate(&descs[i], &h.plan);
        if (st) {
            if (n > 1) g_err = "instance " + std::to_string(i) + ": " + g_err;
            return st;
        }
        if (descs[i].prec != e->prec) return fail(FX_EINVAL, "instance %d: all instances need one precision", i);
        h.d = descs[i];
        const int nz = descs[i].nz;
        h.mat.assign(descs[i].plane_mat, descs[i].plane_mat + nz);
        h.eps_r.assign(descs[i].plane_eps_r, descs[i].plane_eps_r + nz);
        h.Na.assign(descs[i].plane_Na, descs[i].plane_Na + nz);
        h.Nd.assign(descs[i].plane_Nd, descs[i].plane_Nd + nz);
        h.d.plane_mat = h.mat.data();
        h.d.plane_eps_r = h.eps_r.data();
        h.d.plane_Na = h.Na.data();
        h.d.plane_Nd = h.Nd.data();
        build_plan(&h.d, &h.plan);
        h.scale = h.d.h * h.d.h / kEps0;
        h.VT = kKb * h.d.T / kQe;
        h.dmax = h.VT > 0 ? 40.0 * h.VT : 0.0;
    }
    return FX_OK;
}

// Coarse-kernel LDS layout of levels lc.. of one instance (16-byte slots).
template <typename T>
int coarse_layout(const Plan &p, Inst<T> *a) {
    int off = 0;
    auto take = [&](size_t bytes) { const int o = off; off += (int)((bytes + 15) & ~(size_t)15); return o; };
    const int nl = (int)p.lv.size() - p.lc;
    for (int q = 0; q < nl; ++q) {
        const HostLevel &H = p.lv[p.lc + q];
        const int oe = take(H.ncell() * sizeof(T)), orr = take(H.ncell() * sizeof(T));
        const int os = take(H.nsig() * sizeof(T)), ot = take(4 * H.nz * sizeof(T));
        if (a) { a->off_e[q] = oe; a->off_r[q] = orr; a->off_s[q] = os; a->off_t[q] = ot; }
    }
    // transfer tables: 3 ints per coarse plane (cks, ccnt, cthick), 3 ints and
    // 2 values per fine plane (fthick, pka, pkb; pwa, pwb)
    for (int q = 0; q + 1 < nl; ++q) {
        const int nf = p.lv[p.lc + q].nz, nc = p.lv[p.lc + q + 1].nz;
        const int ox = take(3 * nc * sizeof(int) + 3 * nf * sizeof(int) + 2 * nf * sizeof(T) + 16);
        if (a) a->off_x[q] = ox;
    }
    const HostLevel &B = p.lv.back();
    const int op = take(B.ncell() * sizeof(T)), oq = take(B.ncell() * sizeof(T));
    const int ored = take(16 * sizeof(double));
    if (a) { a->off_p = op; a->off_q = oq; a->off_red = ored; }
    return off;
}

// The Newton update is folded into the finest level's last black half-sweep (red/black
// storage and levels of its own above the coarse kernel); else the residual kernel
// forms it.
bool fold_of(const Plan &p) { return p.lv[0].rb && p.lc > 0; }

// LDS of a blocked level's box (every plane), its per-plane tables and z-transfer tables.
size_t tb_lds_bytes(const HostLevel &H, size_t w) {
    return ((size_t)H.nz * kTbW * kTbW + 6 * (size_t)H.nz) * w + 2 * (size_t)H.nz * sizeof(int);
}

// Level l of p may be smoothed in blocks (k_pre_tb / k_post_tb): a red/black level
// below the finest with launches of its own, small enough for its launches to be
// latency-bound (the blocks recompute their rings), halved in x and y into the next,
// tiles that divide both extents, no column twice in one box (extents of at least a
// box edge), at most kTbMaxNz planes, and the box in kTbLdsBytes of LDS.
bool tb_geom(const Plan &p, int l, size_t w) {
    if (l < 1 || l >= p.lc) return false;
    const HostLevel &H = p.lv[l];
    return H.rb && p.lv[l + 1].xy_from_finer == 1 && H.ncell() < ((size_t)1 << 18) && H.nx % kTbT == 0 &&
           H.ny % kTbT == 0 && H.nx >= kTbW && H.ny >= kTbW && H.nz <= kTbMaxNz &&
           tb_lds_bytes(H, w) <= (size_t)kTbLdsBytes &&
           // the coarse values under a box fit above the interpolants (k_post_tb)
           (size_t)p.lv[l + 1].nz * (kTbW * kTbW + (kTbW / 2 + 2) * (kTbW / 2 + 2)) <= (size_t)H.nz * kTbW * kTbW;
}

int tiles_smooth(const HostLevel &H, const SmoothCfg &c) { return tiles_cfg(H.rb ? H.nx / 2 : H.nx, H.ny, H.nz, c); }

// Launch shapes that depend on all instances: levels with their own
// kernels, planes per smoother thread, colours per sweep.
void plan_launches(Engine *e) {
    e->max_lc = 0;
    e->max_cycles = 1;
    e->any_order2 = 0;
    e->any_fd = 0;
    for (const InstHost &h : e->in) {
        e->max_lc = std::max(e->max_lc, h.plan.lc);
        e->max_cycles = std::max(e->max_cycles, h.d.max_cycles);
        if (h.d.time_order == 2) e->any_order2 = 1;
        if (h.d.carriers == FX_CARRIERS_FD) e->any_fd = 1;
    }
    e->scfg.assign(e->max_lc, SmoothCfg{6, 1, 0});
    e->ncol.assign(e->max_lc, 2);
    e->small.assign(e->max_lc, 0);
    const int zt_env = env_int("FERROX_ZT", 0);
    for (int l = 0; l < e->max_lc; ++l) {
        size_t cells = 0;
        int min_nz = 1 << 30;
        for (const InstHost &h : e->in) {
            if (l >= h.plan.lc) continue;
            const HostLevel &H = h.plan.lv[l];
            cells += H.ncell();
            min_nz = std::min(min_nz, H.nz);
            if (!H.rb) e->ncol[l] = 4;
        }
        // before tuning: large levels 4 planes per thread, small ones one plane per
        // thread for parallelism, 64 x 4 tiles
        e->scfg[l].zt = cells >= ((size_t)1 << 19) && min_nz >= 8 ? 4 : 1;
        e->small[l] = cells < ((size_t)1 << 18);
        if (zt_env == 1 || zt_env == 2 || zt_env == 4 || zt_env == 8) e->scfg[l].zt = zt_env;
    }
}

// (E_F - E_c)/kT of a semiconductor plane at phi = 0 under Fermi-Dirac statistics:
// the root of Nv F(-x - Eg/kT) - Nc F(x) + Nd - Na = 0 (falling in x), by bisection
// down to adjacent doubles.
double fd_neutral_eta(double Nc, double Nv, double egkt, double Na, double Nd) {
    double lo = -egkt - 100.0, hi = 100.0;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double Fp, Fn, d;
        fd_half(-mid - egkt, Fp, d);
        fd_half(mid, Fn, d);
        if (Nv * Fp - Nc * Fn + Nd - Na > 0.0) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// Lay out (or, with ws == nullptr, only size) the workspace: one region per
// instance, then the shared tables.
size_t carve(Engine *e, void *ws) {
    Carver cv(ws);
    const bool mixed = e->prec == FX_PREC_MIXED;
    for (InstHost &h : e->in) {
        const Plan &p = h.plan;
        const size_t nfull = (size_t)p.nx * p.ny * p.nz;
        h.P[1] = (double *)cv.take(nfull * sizeof(double));
        const int nbuf = h.d.time_order == 2 ? kPhiBufs : kPhiBufs - 2;
        for (int b = 1; b < nbuf; ++b) h.phi[b] = (double *)cv.take(nfull * sizeof(double));
        const int nzd = p.nzd;
        h.t_cxy = (double *)cv.take(nzd * sizeof(double));
        h.t_czm = (double *)cv.take(nzd * sizeof(double));
        h.t_czp = (double *)cv.take(nzd * sizeof(double));
        h.t_wl = (double *)cv.take(nzd * sizeof(double));
        h.t_wr = (double *)cv.take(nzd * sizeof(double));
        h.t_p0e = (double *)cv.take(nzd * sizeof(double));
        h.t_n0e = (double *)cv.take(nzd * sizeof(double));
        h.t_fd = (double *)cv.take(4 * (size_t)nzd * sizeof(double));
        h.t_flags = (int *)cv.take(nzd * sizeof(int));
        const int nlev = (int)p.lv.size();
        h.L64.assign(mixed ? 0 : nlev, DevLevel<double>());
        h.L32.assign(mixed ? nlev : 0, DevLevel<float>());
        auto lay = [&](auto &D, const HostLevel &H, size_t w) {
            using TT = std::remove_pointer_t<decltype(D.e)>;
            const size_t nc = H.ncell(), ns = H.nsig();
            const int nz = H.nz;
            D.e = (TT *)cv.take(nc * w); D.r = (TT *)cv.take(nc * w); D.sig = (TT *)cv.take(std::max<size_t>(ns, 1) * w);
            D.cxy = (TT *)cv.take(nz * w); D.czm = (TT *)cv.take(nz * w);
            D.czp = (TT *)cv.take(nz * w); D.dg = (TT *)cv.take(nz * w);
            D.pwa = (TT *)cv.take(nz * w); D.pwb = (TT *)cv.take(nz * w);
            D.ks = (int *)cv.take(nz * sizeof(int)); D.cnt = (int *)cv.take(nz * sizeof(int));
            D.thick = (int *)cv.take(nz * sizeof(int)); D.pka = (int *)cv.take(nz * sizeof(int));
            D.pkb = (int *)cv.take(nz * sizeof(int));
        };
        for (int l = 0; l < nlev; ++l) {
            if (mixed) lay(h.L32[l], p.lv[l], 4);
            else lay(h.L64[l], p.lv[l], 8);
            const size_t w = mixed ? 4 : 8;
            if (tb_geom(p, l, w)) {
                void *ea = cv.take(p.lv[l].ncell() * w);
                if (mixed) h.L32[l].ealt = (float *)ea;
                else h.L64[l].ealt = (double *)ea;
            }
        }
        // residual partial sums: one pair per residual tile
        const size_t nres = (size_t)tiles3(p.nx, p.ny, (p.nzd + kResZ - 1) / kResZ);
        h.part = (double *)cv.take(2 * nres * sizeof(double));
        h.qv_part = (double *)cv.take(2 * kQvBlocks * sizeof(double));
        h.qv_rec = (double *)cv.take(2 * (size_t)kRecSteps * sizeof(double));
    }
    const size_t inst_bytes = mixed ? sizeof(Inst<float>) : sizeof(Inst<double>);
    e->inst_dev = cv.take((size_t)e->n * inst_bytes);
    e->st_dev = (InstState *)cv.take((size_t)e->n * sizeof(InstState));
    const size_t ntab = 4 + 5 * (size_t)e->max_lc;
    e->prefix_dev = (int *)cv.take(ntab * (e->n + 1) * sizeof(int));
    e->sched_dev = (double *)cv.take((size_t)e->n * kSchedChunk * sizeof(double));
    e->probe_dev = (double *)cv.take(kProbeMax * sizeof(double));
    e->qv_out = (double *)cv.take(2 * (size_t)e->n * sizeof(double));
    return cv.off + 256;
}

// Prefix tables of per-instance tile counts, one per launch kind.
fx_status build_work(Engine *e) {
    const int n = e->n;
    e->prefix_host.clear();
    int tab = 0;
    fx_status bad = FX_OK;
    auto mk = [&](auto count) -> Work {
        Work w;
        w.prefix = e->prefix_dev + (size_t)tab * (n + 1);
        w.ninst = n;
        w.st = e->st_dev;
        long long tot = 0;
        e->prefix_host.push_back(0);
        for (int i = 0; i < n; ++i) {
            tot += count(e->in[i]);
            if (tot > (1LL << 30)) bad = FX_EINVAL;
            e->prefix_host.push_back((int)std::min<long long>(tot, 1LL << 30));
        }
        w.total = (int)std::min<long long>(tot, 1LL << 30);
        ++tab;
        return w;
    };
    e->w_tdgl = mk([](const InstHost &h) { const Plan &p = h.plan; return p.f0 >= 0 ? tiles3(p.nx, p.ny, p.f1 - p.f0) : 0; });
    e->w_ext = mk([](const InstHost &h) {
        const Plan &p = h.plan;
        return (int)(((size_t)p.nx * p.ny * p.nzd + kExtrapChunk - 1) / kExtrapChunk);
    });
    // residual: every instance in mode 0; after the cycles of unfolded instances, mode 2
    auto nzc = [](const Plan &p) { return (p.nzd + kResZ - 1) / kResZ; };
    e->w_res.cell0 = mk([&](const InstHost &h) { const Plan &p = h.plan; return tiles3(p.nx, p.ny, nzc(p)); });
    e->w_res.cell2 = mk([&](const InstHost &h) { const Plan &p = h.plan; return fold_of(p) ? 0 : tiles3(p.nx, p.ny, nzc(p)); });
    e->w_sm.clear(); e->w_rs.clear(); e->w_pr.clear(); e->w_prc.clear(); e->prc_cz.clear();
    e->w_tb.clear(); e->tb.clear(); e->tb_lds.clear();
    const int cc_ok = env_int("FERROX_PROLONG_CC", 1) != 0;
    // the coarse-column prolongation: red/black fine level, x and y halved, z paired
    auto by_cc = [cc_ok](const Plan &p, int l) {
        return cc_ok && p.lv[l].rb && p.lv[l + 1].xy_from_finer == 1 && p.lv[l + 1].z_from_finer;
    };
    for (int l = 0; l < e->max_lc; ++l) {
        const SmoothCfg c = e->scfg[l];
        e->w_sm.push_back(mk([&](const InstHost &h) { return l < h.plan.lc ? tiles_smooth(h.plan.lv[l], c) : 0; }));
        e->w_rs.push_back(mk([&](const InstHost &h) {
            if (l >= h.plan.lc) return 0;
            const HostLevel &C = h.plan.lv[l + 1];
            return tiles3(C.nx, C.ny, C.nz);
        }));
        e->w_pr.push_back(mk([&](const InstHost &h) {
            if (l >= h.plan.lc || by_cc(h.plan, l)) return 0;
            const HostLevel &F = h.plan.lv[l];
            const int zt = (F.nz + kProZ - 1) / kProZ;
            return F.rb ? tiles3(F.nx / 2, F.ny, zt) : tiles3(F.nx, F.ny, zt);
        }));
        // several coarse planes per thread where the coarse level is large, one where
        // more threads are needed to fill the chip
        size_t ccells = 0;
        for (const InstHost &h : e->in)
            if (l < h.plan.lc && by_cc(h.plan, l)) ccells += h.plan.lv[l + 1].ncell();
        const int cz = ccells >= kProCZBig ? kProCZ : 1;
        e->prc_cz.push_back(cz);
        e->w_prc.push_back(mk([&](const InstHost &h) {
            if (l >= h.plan.lc || !by_cc(h.plan, l)) return 0;
            const HostLevel &C = h.plan.lv[l + 1];
            return tiles3(C.nx, C.ny, (C.nz + cz - 1) / cz);
        }));
        // blocked smoothing where every instance that has this level qualifies
        const size_t w = e->prec == FX_PREC_MIXED ? 4 : 8;
        bool ok = e->fuse && env_int("FERROX_TB", 1) != 0 && e->nu1c <= 2 && e->nu2c <= 2;
        bool any = false;
        int lds = 0;
        for (const InstHost &h : e->in) {
            if (l >= h.plan.lc) continue;
            any = true;
            ok = ok && tb_geom(h.plan, l, w);
            lds = std::max(lds, (int)tb_lds_bytes(h.plan.lv[l], w));
        }
        e->tb.push_back(ok && any);
        e->tb_lds.push_back(lds);
        e->w_tb.push_back(mk([&](const InstHost &h) {
            if (!e->tb[l] || l >= h.plan.lc) return 0;
            return (h.plan.lv[l].nx / kTbT) * (h.plan.lv[l].ny / kTbT);
        }));
    }
    if (bad) return fail(FX_EINVAL, "a launch would exceed 2^30 tiles");
    HIP_OK(hipMemcpy(e->prefix_dev, e->prefix_host.data(), e->prefix_host.size() * sizeof(int), hipMemcpyHostToDevice));
    return FX_OK;
}

template <typename T>
fx_status upload_level(const HostLevel &H, DevLevel<T> &D) {
    std::vector<T> a(H.nz);
    auto up = [&](T *dst, const std::vector<double> &src) -> fx_status {
        for (int K = 0; K < H.nz; ++K) a[K] = (T)src[K];
        HIP_OK(hipMemcpy(dst, a.data(), H.nz * sizeof(T), hipMemcpyHostToDevice));
        return FX_OK;
    };
    auto upi = [&](int *dst, std::vector<int> v, int fillv) -> fx_status {
        v.resize(H.nz, fillv);
        HIP_OK(hipMemcpy(dst, v.data(), H.nz * sizeof(int), hipMemcpyHostToDevice));
        return FX_OK;
    };
    fx_status st;
    if ((st = up(D.cxy, H.cxy)) || (st = up(D.czm, H.czm)) || (st = up(D.czp, H.czp)) || (st = up(D.dg, H.dg)))
        return st;
    std::vector<double> pwa(H.pwa), pwb(H.pwb);
    pwa.resize(H.nz, 1.0); pwb.resize(H.nz, 0.0);
    if ((st = up(D.pwa, pwa)) || (st = up(D.pwb, pwb))) return st;
    std::vector<int> thick(H.nz);
    for (int K = 0; K < H.nz; ++K) thick[K] = H.e0[K] - H.s0[K];
    if ((st = upi(D.ks, H.ks, 0)) || (st = upi(D.cnt, H.cnt, 1)) || (st = upi(D.thick, thick, 1)) ||
        (st = upi(D.pka, H.pka, 0)) || (st = upi(D.pkb, H.pkb, -1)))
        return st;
    return FX_OK;
}

template <typename T>
const std::vector<DevLevel<T>> &levels(const InstHost &h) {
    if constexpr (std::is_same<T, float>::value) return h.L32;
    else return h.L64;
}

template <typename T>
Inst<T> make_inst(const Engine *e, int i) {
    const InstHost &h = e->in[i];
    const Plan &p = h.plan;
    const fx_stack_desc &d = h.d;
    const std::vector<DevLevel<T>> &D = levels<T>(h);
    Inst<T> a;
    memset(&a, 0, sizeof a);
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.kb = p.kb; a.nzd = p.nzd;
    a.f0 = p.f0 >= 0 ? p.f0 : 0;
    a.f1 = p.f0 >= 0 ? p.f1 : 0;
    a.nlev = (int)p.lv.size();
    a.lc = p.lc;
    a.fold = fold_of(p);
    a.max_cycles = d.max_cycles;
    a.warm = d.warm_start;
    a.order2 = d.time_order == 2;
    a.nbuf = a.order2 ? kPhiBufs : kPhiBufs - 2;
    a.light_ok = env_int("FERROX_LIGHT", 1) != 0;
    {
        const char *lr = getenv("FERROX_LIGHT_RATIO"), *lc = getenv("FERROX_LIGHT_CUT");
        const double r = lr ? atof(lr) : kLightRatio, c = lc ? atof(lc) : kLightContraction;
        a.light_r2 = r * r;
        a.light_c2 = c * c;
    }
    a.tol2 = d.tol_rel * d.tol_rel;
    a.h = d.h; a.alpha = d.alpha; a.beta = d.beta; a.gamma = d.gamma;
    a.g11 = d.g11; a.g44 = d.g44; a.Gamma = d.Gamma; a.lambda = d.lambda; a.pbc = d.pbc;
    a.v_b = d.v_bottom;
    a.p_scale = d.h / kEps0;
    a.rho_scale = h.scale;
    a.vt_inv = h.VT > 0 ? 1.0 / h.VT : 0.0;
    a.sig_scale = h.VT > 0 ? h.scale / h.VT : 0.0;
    a.dmax = h.dmax;
    a.cxy0 = h.t_cxy; a.czm0 = h.t_czm; a.czp0 = h.t_czp; a.wl = h.t_wl; a.wr = h.t_wr;
    a.p0e = h.t_p0e; a.n0e = h.t_n0e; a.pflags = h.t_flags;
    a.fd = d.carriers == FX_CARRIERS_FD;
    a.fdt = h.t_fd;
    a.vsched = e->sched_dev + (size_t)i * kSchedChunk;
    for (int b = 0; b < kPhiBufs; ++b) a.phi[b] = h.phi[b];
    a.P[0] = h.P[0]; a.P[1] = h.P[1];
    a.part = h.part;
    a.st = e->st_dev + i;
    // the ferroelectric/dielectric face: below the ferroelectric if that plane is
    // dielectric, else above it
    a.qv_kl = -1;
    a.qv_fe_up = 0;
    if (p.f0 >= 0) {
        if (p.f0 - 1 >= p.kb && h.mat[p.f0 - 1] == FX_MAT_DE) { a.qv_kl = p.f0 - 1; a.qv_fe_up = 1; }
        else if (p.f1 < p.kt && h.mat[p.f1] == FX_MAT_DE) { a.qv_kl = p.f1 - 1; a.qv_fe_up = 0; }
    }
    if (a.qv_kl >= 0) {
        a.qv_el = kEps0 * h.eps_r[a.qv_kl];
        a.qv_er = kEps0 * h.eps_r[a.qv_kl + 1];
    }
    a.qv_part = h.qv_part;
    a.qv_rec = h.qv_rec;
    for (int l = 0; l < a.nlev; ++l) {
        const HostLevel &H = p.lv[l];
        LevelArgs<T> &L = a.lv[l];
        L.nx = H.nx; L.ny = H.ny; L.nz = H.nz; L.rb = H.rb;
        L.cxy = D[l].cxy; L.czm = D[l].czm; L.czp = D[l].czp; L.dg = D[l].dg;
        L.e = D[l].e; L.r = D[l].r; L.sig = D[l].sig;
        L.sig_lo = H.sig_lo; L.sig_hi = H.sig_hi;
        L.ealt = D[l].ealt;
        if (l + 1 < a.nlev) {
            XferArgs<T> &X = a.xf[l];
            X.cks = D[l + 1].ks; X.ccnt = D[l + 1].cnt;
            X.fthick = D[l].thick; X.cthick = D[l + 1].thick;
            X.pka = D[l].pka; X.pkb = D[l].pkb; X.pwa = D[l].pwa; X.pwb = D[l].pwb;
            X.xy = p.lv[l + 1].xy_from_finer;
        }
    }
    a.nu1 = e->nu1c;
    a.nu2 = e->nu2c;
    // CG in exact arithmetic ends within ncell steps; the cap only guards rounding
    a.bottom_iters = (int)std::min<size_t>(2 * p.lv.back().ncell() + 8, 512);
    {
        // relative residual the bottom solve reaches (FERROX_BOTTOM_RTOL overrides)
        const char *v = getenv("FERROX_BOTTOM_RTOL");
        const double rt = v && *v ? atof(v) : (std::is_same<T, float>::value ? 1e-5 : 1e-7);
        a.bottom_tol2 = rt * rt;
    }
    a.lds_bytes = coarse_layout<T>(p, &a);
    return a;
}

// Per-plane tables of the finest level and of every multigrid level, the
// instance array and the initial states.
template <typename T>
fx_status upload_all(Engine *e) {
    std::vector<Inst<T>> host(e->n);
    for (int i = 0; i < e->n; ++i) {
        InstHost &h = e->in[i];
        const Plan &p = h.plan;
        const fx_stack_desc &d = h.d;
        const int nzd = p.nzd;
        // finest-level tables: scaled coefficients, P face weights, carrier densities
        std::vector<double> wl(nzd, 1.0), wr(nzd, 0.0), p0e(nzd, 0.0), n0e(nzd, 0.0), fdt(4 * (size_t)nzd, 0.0);
        std::vector<int> fl(nzd, 0);
        for (int k = 0; k < nzd; ++k) {
            const int K = p.kb + k;
            if (k + 1 < nzd) {
                const double eL = d.plane_eps_r[K], eR = d.plane_eps_r[K + 1];
                wl[k] = eR / (eL + eR);
                wr[k] = eL / (eL + eR);
            }
            const bool fe_near = d.plane_mat[K] == FX_MAT_FE || (k > 0 && d.plane_mat[K - 1] == FX_MAT_FE) ||
                                 (k + 1 < nzd && d.plane_mat[K + 1] == FX_MAT_FE);
            if (fe_near) fl[k] |= PF_P;
            if (d.plane_mat[K] == FX_MAT_SC) {
                fl[k] |= PF_SC;
                if (d.carriers == FX_CARRIERS_FD) {
                    const double kT = kKb * d.T;
                    const double Nc = 2.0 * std::pow(d.m_e * kMe0 * kT / (2.0 * M_PI * kHbar * kHbar), 1.5);
                    const double Nv = 2.0 * std::pow(d.m_p * kMe0 * kT / (2.0 * M_PI * kHbar * kHbar), 1.5);
                    const double egkt = d.Eg / h.VT;
                    const double etn = fd_neutral_eta(Nc, Nv, egkt, d.plane_Na[K], d.plane_Nd[K]);
                    double F, dF;
                    fdt[4 * k + 0] = -etn - egkt;
                    fdt[4 * k + 1] = etn;
                    fd_half(-etn - egkt, F, dF);
                    fdt[4 * k + 2] = F;
                    fd_half(etn, F, dF);
                    fdt[4 * k + 3] = F;
                    p0e[k] = kQe * Nv;
                    n0e[k] = kQe * Nc;
                } else {
                    const double net = d.plane_Nd[K] - d.plane_Na[K], ni = d.ni;
                    double pp, nn;
                    if (net >= 0) { nn = 0.5 * net + std::sqrt(0.25 * net * net + ni * ni); pp = ni * ni / nn; }
                    else { pp = -0.5 * net + std::sqrt(0.25 * net * net + ni * ni); nn = ni * ni / pp; }
                    p0e[k] = kQe * pp;
                    n0e[k] = kQe * nn;
                }
            }
        }
        const HostLevel &H0 = p.lv[0];
        HIP_OK(hipMemcpy(h.t_cxy, H0.cxy.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_czm, H0.czm.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_czp, H0.czp.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_wl, wl.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_wr, wr.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_p0e, p0e.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_n0e, n0e.data(), nzd * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_fd, fdt.data(), fdt.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h.t_flags, fl.data(), nzd * sizeof(int), hipMemcpyHostToDevice));
        const std::vector<DevLevel<T>> &D = levels<T>(h);
        for (size_t l = 0; l < p.lv.size(); ++l) {
            fx_status st = upload_level(p.lv[l], const_cast<DevLevel<T> &>(D[l]));
            if (st) return st;
        }
        host[i] = make_inst<T>(e, i);
        h.lds = host[i].lds_bytes;
        if (h.lds > kCoarseLdsBytes) return fail(FX_EINVAL, "coarse levels need %d bytes of LDS", h.lds);
        e->lds_max = std::max(e->lds_max, h.lds);
    }
    HIP_OK(hipMemcpy(e->inst_dev, host.data(), (size_t)e->n * sizeof(Inst<T>), hipMemcpyHostToDevice));
    for (int i = 0; i < e->n; ++i) {
        InstState &s = e->mir[i];
        memset(&s, 0, sizeof s);
        s.done = 1;                     // idle: no solve running
        s.cur = 0;
        for (int m = 0; m < kMaxHist; ++m) s.prev[m] = m + 1;
        s.pstar = -1;
        s.parked = 1;
        s.v_top = e->in[i].d.v_top;
    }
    HIP_OK(hipMemcpy(e->st_dev, e->mir, (size_t)e->n * sizeof(InstState), hipMemcpyHostToDevice));
    return FX_OK;
}

// ------------------------------------------------------------ launch slots
template <typename T>
const Inst<T> *idev(const Engine *e) { return (const Inst<T> *)e->inst_dev; }

// One smoother colour at level l; finest-level launches are timed while the
// probe is on.
template <typename T>
void smooth_l(Engine *e, int l, int color, int zi, int upd, int skip_light = 0) {
    const Work &w = e->w_sm[l];
    if (w.total <= 0) return;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double *pb = nullptr;
    if (l == 0 && e->probe && e->ev_used + 2 <= (int)e->ev.size() && (e->probe_seen++ % e->probe_stride) == 0) {
        e0 = e->ev[e->ev_used];
        e1 = e->ev[e->ev_used + 1];
        pb = e->probe_dev + e->ev_used / 2;
        e->ev_used += 2;
    }
    launch_smooth(idev<T>(e), w, l, color, zi, upd, e->scfg[l], pb, e->st, e0, e1, skip_light);
}

// One V(nu1, nu2) cycle over every running instance.  Levels 0 .. lc-1 of an
// instance have their own launches; the coarse kernel takes the rest.  On
// the finest level the last black half-sweep also forms phi_out = phi_in +
// clip(e) where the update is folded in.
template <typename T>
void enq_vcycle(Engine *e) {
    const Inst<T> *I = idev<T>(e);
    for (int l = 0; l < e->max_lc; ++l) {
        if (e->tb[l]) {                                  // sweeps and restriction in blocks
            launch_pre_tb(I, e->w_tb[l], l, e->nu1c, e->tb_lds[l], e->st);
            continue;
        }
        const int nu1 = l == 0 ? e->nu1 : e->nu1c;
        // below the finest level (whose launches the probe times one by one) the
        // zero-start red and black half-sweeps of a red/black level are one launch
        const bool zpair = e->fuse && l > 0 && e->ncol[l] == 2 && e->w_sm[l].total > 0;
        // a light cycle (InstState::light) leaves out the sweeps after the first
        for (int q = 0; q < nu1; ++q) {
            if (q == 0 && zpair) {
                launch_smooth_zpair(I, e->w_sm[l], l, e->scfg[l], e->st);
                continue;
            }
            for (int c = 0; c < e->ncol[l]; ++c) smooth_l<T>(e, l, c, q == 0 && c == 0, 0, q > 0);
        }
        launch_restrict(I, e->w_rs[l], l, e->st);
    }
    launch_coarse(I, e->st_dev, e->n, e->lds_max, e->st);
    for (int l = e->max_lc - 1; l >= 0; --l) {
        if (e->tb[l]) {                                  // prolongation and sweeps in blocks
            launch_post_tb(I, e->w_tb[l], l, e->nu2c, e->tb_lds[l], e->st);
            continue;
        }
        const int nu2 = l == 0 ? e->nu2 : e->nu2c;
        // on a small red/black level the correction is formed inside the first
        // red half-sweep: one launch fewer, where launches cost more than the
        // six interpolations per red cell the fused kernel repeats
        const bool pred = e->fuse && l > 0 && e->small[l] && e->ncol[l] == 2 && e->w_sm[l].total > 0;
        if (pred) {
            launch_prolong_red(I, e->w_sm[l], l, e->scfg[l], e->st);
        } else {
            launch_prolong_cc(I, e->w_prc[l], l, e->prc_cz[l], e->st);
            launch_prolong(I, e->w_pr[l], l, e->st);
        }
        // a light cycle leaves out one sweep: on the finest level one before the
        // last (which folds the update in), elsewhere one after the first (whose red
        // half holds the fused prolongation)
        for (int q = 0; q < nu2; ++q) {
            const int skip = nu2 > 1 && (l == 0 ? q == nu2 - 2 : q == nu2 - 1);
            for (int c = 0; c < e->ncol[l]; ++c) {
                if (pred && q == 0 && c == 0) continue;
                smooth_l<T>(e, l, c, 0, l == 0 && q == nu2 - 1 && c == 1, skip);
            }
        }
    }
}

// Cycle slot: one cycle and its residual for every running solve.
template <typename T>
void enq_cycle(Engine *e) {
    enq_vcycle<T>(e);
    launch_residual(idev<T>(e), e->w_res, 1, e->any_fd, e->st);
    launch_reduce(idev<T>(e), e->st_dev, e->n, 1, e->st);
}

// Advance slot: finalize stopped solves, start the next time step where due.
template <typename T>
void enq_advance(Engine *e) {
    const Inst<T> *I = idev<T>(e);
    launch_head(I, e->st_dev, e->n, 1, e->st);
    if (e->rec) launch_qv(I, e->n, 1, nullptr, e->st);
    launch_tdgl(I, e->w_tdgl, 1, e->st);
    if (e->any_order2) launch_tdgl_corr(I, e->w_tdgl, e->st);
    launch_begin(I, e->st_dev, e->n, 1, e->st);
    launch_extrap(I, e->w_ext, e->st);
    launch_residual(I, e->w_res, 0, e->any_fd, e->st);
    launch_reduce(I, e->st_dev, e->n, 0, e->st);
}

template <typename T>
void enq_units(Engine *e, int units) {
    for (int u = 0; u < units; ++u) {
        enq_cycle<T>(e);
        enq_advance<T>(e);
    }
}

// Capture the unit sequences as graphs (once; a private stream records them).
void drop_graphs(Engine *e);

template <typename T>
fx_status capture_units(Engine *e) {
    if (e->unit_exec[0] && e->graphs_rec == e->rec) return FX_OK;
    drop_graphs(e);
    e->graphs_rec = e->rec;
    if (!e->cap) HIP_OK(hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking));
    hipStream_t user = e->st;
    for (int q = 0; q < kUnitPow; ++q) {
        hipGraph_t g = nullptr;
        e->st = e->cap;
        hipError_t err = hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) {
            enq_units<T>(e, 1 << q);
            err = hipStreamEndCapture(e->cap, &g);
        }
        e->st = user;
        if (err != hipSuccess) return fail(FX_EDEVICE, "graph capture failed: %s", hipGetErrorString(err));
        err = hipGraphInstantiate(&e->unit_exec[q], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (err != hipSuccess) return fail(FX_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(err));
    }
    return FX_OK;
}

template <typename T>
fx_status launch_units(Engine *e, int units) {
    if (e->mode == FX_LAUNCH_GRAPH && !e->probe) {
        fx_status st = capture_units<T>(e);
        if (st) return st;
        for (int q = kUnitPow - 1; q >= 0; --q)
            while (units >= (1 << q)) {
                HIP_OK(hipGraphLaunch(e->unit_exec[q], e->st));
                units -= 1 << q;
            }
        return FX_OK;
    }
    enq_units<T>(e, units);
    return FX_OK;
}

fx_status read_states(Engine *e) {
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(e->mir, e->st_dev, (size_t)e->n * sizeof(InstState), hipMemcpyDeviceToHost, e->st));
    HIP_OK(hipStreamSynchronize(e->st));
    return FX_OK;
}

// Plain solve of every instance from its current phi (Step 0, poisson_solve).
template <typename T>
fx_status solve_plain_t(Engine *e) {
    const Inst<T> *I = idev<T>(e);
    launch_begin(I, e->st_dev, e->n, 0, e->st);
    launch_residual(I, e->w_res, 0, e->any_fd, e->st);
    launch_reduce(I, e->st_dev, e->n, 0, e->st);
    int enq = 0;
    int batch = e->trace ? 0 : std::max(1, e->k_pred);
    fx_status st;
    for (;;) {
        for (int q = 0; q < batch && enq < e->max_cycles; ++q, ++enq) enq_cycle<T>(e);
        if ((st = read_states(e))) return st;
        bool all = true;
        for (int i = 0; i < e->n; ++i) all &= e->mir[i].done != 0;
        if (e->trace) {
            const InstState &c = e->mir[0];
            fprintf(stderr, "[ferrox] cycle %d |r|/|f| = %.3e\n", c.cycles, c.fn2 > 0 ? std::sqrt(c.rn2 / c.fn2) : 0.0);
        }
        if (all) break;
        if (enq >= e->max_cycles) return fail(FX_EDEVICE, "solver state did not stop after %d cycles", enq);
        batch = 1;
    }
    launch_head(I, e->st_dev, e->n, 0, e->st);
    if ((st = read_states(e))) return st;
    int kmax = 1;
    for (int i = 0; i < e->n; ++i)
        if (e->mir[i].status != FX_ENONFINITE) kmax = std::max(kmax, e->mir[i].cycles);
    e->k_pred = kmax;
    return FX_OK;
}

fx_status solve_plain(Engine *e) { return e->prec == FX_PREC_MIXED ? solve_plain_t<float>(e) : solve_plain_t<double>(e); }

// nsteps time steps of every instance (Steps 1a + 1b each, and 2a + 2b for
// predictor-corrector instances, whose steps take two solves).  The
// schedule (host arrays of nsteps gate potentials per instance, or NULL)
// is staged through the device in chunks; inside a chunk the host only
// checks, every few units, whether all instances have parked.
template <typename T>
fx_status run_t(Engine *e, int nsteps, double dt, const double *const *sched, double *const *q_out,
                double *const *v_out) {
    const Inst<T> *I = idev<T>(e);
    fx_status st;
    e->rec = q_out != nullptr;
    std::vector<int> step0(e->n);
    std::vector<double> stage;
    for (int done = 0, first = 1; done < nsteps; first = 0) {
        const int chunk = std::min(kSchedChunk, nsteps - done);
        if (e->rec)
            for (int i = 0; i < e->n; ++i) {
                step0[i] = e->mir[i].step;
                launch_fill(e->in[i].qv_rec, 2 * (size_t)kRecSteps, NAN, e->st);
            }
        if (sched) {
            HIP_OK(hipStreamSynchronize(e->st));
            for (int i = 0; i < e->n; ++i)
                HIP_OK(hipMemcpyAsync(e->sched_dev + (size_t)i * kSchedChunk, sched[i] + done, chunk * sizeof(double),
                                      hipMemcpyHostToDevice, e->st));
        }
        launch_run_setup(I, e->n, chunk, sched ? 1 : 0, dt, first, e->st);
        enq_advance<T>(e);
        long long budget = (long long)chunk * (e->any_order2 ? 2 : 1) * (e->max_cycles + 1) + 1;
        int units = std::min(e->ucap, chunk);
        for (;;) {
            if ((st = launch_units<T>(e, units))) return st;
            budget -= units;
            if ((st = read_states(e))) return st;
            int rem = 0;
            bool all = true;
            for (int i = 0; i < e->n; ++i) {
                const InstState &s = e->mir[i];
                if (s.parked) continue;
                all = false;
                const int solves = e->in[i].d.time_order == 2 ? 2 * (s.target - s.step) - s.phase
                                                              : s.target - s.step;
                rem = std::max(rem, solves);
            }
            if (all) break;
            if (budget <= 0) return fail(FX_EDEVICE, "time steps did not finish within the cycle budget");
            units = std::max(1, std::min(e->ucap, rem));
        }
        if (e->rec) {
            stage.resize(2 * (size_t)kRecSteps);
            for (int i = 0; i < e->n; ++i) {
                const int got = std::min(e->mir[i].step - step0[i], chunk);
                if (got <= 0) continue;
                HIP_OK(hipMemcpyAsync(stage.data(), e->in[i].qv_rec, 2 * (size_t)got * sizeof(double),
                                      hipMemcpyDeviceToHost, e->st));
                HIP_OK(hipStreamSynchronize(e->st));
                for (int q = 0; q < got; ++q) {
                    q_out[i][done + q] = stage[2 * q];
                    v_out[i][done + q] = stage[2 * q + 1];
                }
            }
        }
        done += chunk;
        bool any_ok = false;
        for (int i = 0; i < e->n; ++i) any_ok |= e->mir[i].status == FX_OK;
        if (!any_ok) break;
    }
    return FX_OK;
}

fx_status run(Engine *e, int nsteps, double dt, const double *const *sched, double *const *q_out = nullptr,
              double *const *v_out = nullptr) {
    return e->prec == FX_PREC_MIXED ? run_t<float>(e, nsteps, dt, sched, q_out, v_out)
                                    : run_t<double>(e, nsteps, dt, sched, q_out, v_out);
}

// The ferroelectric has a dielectric plane next to it (the face Q and V_fe are read on).
bool has_interface(const InstHost &h) {
    const Plan &p = h.plan;
    if (p.f0 < 0) return false;
    return (p.f0 - 1 >= p.kb && h.mat[p.f0 - 1] == FX_MAT_DE) || (p.f1 < p.kt && h.mat[p.f1] == FX_MAT_DE);
}

// Q and V_fe of every instance's current state into host arrays of n entries.
fx_status qv_now(Engine *e, double *h_Q, double *h_V) {
    if (e->prec == FX_PREC_MIXED) launch_qv(idev<float>(e), e->n, 0, e->qv_out, e->st);
    else launch_qv(idev<double>(e), e->n, 0, e->qv_out, e->st);
    std::vector<double> b(2 * (size_t)e->n);
    HIP_OK(hipMemcpyAsync(b.data(), e->qv_out, b.size() * sizeof(double), hipMemcpyDeviceToHost, e->st));
    HIP_OK(hipStreamSynchronize(e->st));
    for (int i = 0; i < e->n; ++i) {
        h_Q[i] = b[2 * i];
        h_V[i] = b[2 * i + 1];
    }
    return FX_OK;
}

// Write the host mirror of instance i back to the device (stream-ordered).
void put_state(Engine *e, int i) { launch_put_state(e->st_dev + i, e->mir[i], e->st); }

// Buffer b holds a stored time level or the last predictor's phi*.
bool holds_history(const InstState &s, int b) {
    for (int m = 0; m < s.hist; ++m)
        if (s.prev[m] == b) return true;
    return s.pstar == b;
}

void fill_contacts(Engine *e, int i, bool force) {
    InstHost &h = e->in[i];
    const Plan &p = h.plan;
    const size_t nxy = (size_t)p.nx * p.ny;
    const double vt = e->mir[i].v_top;
    if (force && p.kb > 0) launch_fill(h.phi[0], (size_t)p.kb * nxy, h.d.v_bottom, e->st);
    if (p.kt < p.nz && (force || !(h.filled_top == vt)))
        launch_fill(h.phi[0] + (size_t)p.kt * nxy, (size_t)(p.nz - p.kt) * nxy, vt, e->st);
    h.filled_top = vt;
}

// Make the caller's arrays hold the current P and phi (mirror must be valid).
fx_status sync_to_caller(Engine *e) {
    for (int i = 0; i < e->n; ++i) {
        InstHost &h = e->in[i];
        InstState &s = e->mir[i];
        const Plan &p = h.plan;
        const size_t nxy = (size_t)p.nx * p.ny;
        bool changed = false;
        if (s.pcur != 0) {
            if (p.f0 >= 0)
                HIP_OK(hipMemcpyAsync(h.P[0] + p.f0 * nxy, h.P[1] + p.f0 * nxy, (p.f1 - p.f0) * nxy * sizeof(double),
                                      hipMemcpyDeviceToDevice, e->st));
            s.pcur = 0;
            changed = true;
        }
        if (s.cur != 0) {
            // buffer 0 is the caller's: if it holds a stored level (or the last
            // predictor's phi*), move that first
            for (int m = -1; m < s.hist; ++m) {
                int &slot = m < 0 ? s.pstar : s.prev[m];
                if (slot != 0) continue;
                int spare = 1;
                while (spare == s.cur || holds_history(s, spare)) ++spare;
                HIP_OK(hipMemcpyAsync(h.phi[spare] + p.kb * nxy, h.phi[0] + p.kb * nxy,
                                      (size_t)p.nzd * nxy * sizeof(double), hipMemcpyDeviceToDevice, e->st));
                slot = spare;
            }
            HIP_OK(hipMemcpyAsync(h.phi[0] + p.kb * nxy, h.phi[s.cur] + p.kb * nxy,
                                  (size_t)p.nzd * nxy * sizeof(double), hipMemcpyDeviceToDevice, e->st));
            s.cur = 0;
            changed = true;
        }
        if (changed) put_state(e, i);
        fill_contacts(e, i, false);
    }
    HIP_OK(hipGetLastError());
    return FX_OK;
}

int env_mode(int dflt) {
    const int m = env_int("FERROX_LAUNCH", dflt);
    return m == FX_LAUNCH_GRAPH ? FX_LAUNCH_GRAPH : FX_LAUNCH_STREAM;
}

// Common set-up of stacks and batches, then Step 0 for every instance.
fx_status engine_init(Engine *e, double *const *d_P, double *const *d_phi, void *d_ws, size_t ws_bytes,
                      void *stream) {
    const size_t need = carve(e, nullptr);
    if (ws_bytes < need) return fail(FX_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    carve(e, d_ws);
    e->st = (hipStream_t)stream;
    e->nu1 = std::max(1, env_int("FERROX_NU1", 2));
    e->nu2 = std::max(1, env_int("FERROX_NU2", 2));
    e->nu1c = std::max(1, env_int("FERROX_NU1C", e->nu1));
    e->nu2c = std::max(1, env_int("FERROX_NU2C", e->nu2));
    e->fuse = env_int("FERROX_FUSE", 1) != 0;
    e->trace = env_int("FERROX_TRACE", 0);
    e->ucap = std::max(1, std::min(1 << (kUnitPow - 1), env_int("FERROX_UNITS", 16)));
    for (int i = 0; i < e->n; ++i) {
        e->in[i].P[0] = d_P[i];
        e->in[i].phi[0] = d_phi[i];
    }
    if (e->no_alloc) {
        e->mir_plain.assign(e->n, InstState{});
        e->mir = e->mir_plain.data();
    } else if (hipHostMalloc((void **)&e->mir, (size_t)e->n * sizeof(InstState), 0) != hipSuccess) {
        return fail(FX_EDEVICE, "hipHostMalloc failed");
    }
    fx_status st = build_work(e);
    if (st) return st;
    st = e->prec == FX_PREC_MIXED ? upload_all<float>(e) : upload_all<double>(e);
    if (st) return st;
    for (int i = 0; i < e->n; ++i) {
        InstHost &h = e->in[i];
        const Plan &p = h.plan;
        // P: zero off the ferroelectric in both buffers
        const size_t nfull = (size_t)p.nx * p.ny * p.nz, nxy = (size_t)p.nx * p.ny;
        launch_fill(h.P[1], nfull, 0.0, e->st);
        if (p.f0 >= 0) {
            if (p.f0 > 0) launch_fill(h.P[0], (size_t)p.f0 * nxy, 0.0, e->st);
            if (p.f1 < p.nz) launch_fill(h.P[0] + (size_t)p.f1 * nxy, (size_t)(p.nz - p.f1) * nxy, 0.0, e->st);
        } else {
            launch_fill(h.P[0], nfull, 0.0, e->st);
        }
        // Step 0: phi^{0,(0)} = 0, then solve
        for (int b = 0; b < kPhiBufs; ++b)
            if (h.phi[b]) launch_fill(h.phi[b], nfull, 0.0, e->st);
        // level arrays start defined (the autotuner may sweep them before any solve)
        const size_t w = e->prec == FX_PREC_MIXED ? sizeof(float) : sizeof(double);
        for (size_t l = 0; l < p.lv.size(); ++l) {
            const HostLevel &H = p.lv[l];
            void *ee = e->prec == FX_PREC_MIXED ? (void *)h.L32[l].e : (void *)h.L64[l].e;
            void *rr = e->prec == FX_PREC_MIXED ? (void *)h.L32[l].r : (void *)h.L64[l].r;
            void *ss = e->prec == FX_PREC_MIXED ? (void *)h.L32[l].sig : (void *)h.L64[l].sig;
            launch_zero(ee, H.ncell() * w, e->st);
            launch_zero(rr, H.ncell() * w, e->st);
            launch_zero(ss, std::max<size_t>(H.nsig(), 1) * w, e->st);
        }
        fill_contacts(e, i, true);
    }
    launch_fill(e->probe_dev, kProbeMax, 0.0, e->st);
    return solve_plain(e);
}

void engine_release(Engine *e) {
    if (e->st) (void)hipStreamSynchronize(e->st); else (void)hipDeviceSynchronize();
    for (int q = 0; q < kUnitPow; ++q)
        if (e->unit_exec[q]) (void)hipGraphExecDestroy(e->unit_exec[q]);
    for (int q = 0; q < kUnitPow; ++q) e->unit_exec[q] = nullptr;
    if (e->cap) (void)hipStreamDestroy(e->cap);
    if (e->mir && !e->no_alloc) (void)hipHostFree(e->mir);
    e->mir = nullptr;
    for (hipEvent_t ev : e->ev) (void)hipEventDestroy(ev);
}

fx_status status_message(const InstState &s, int inst) {
    const char *who = inst >= 0 ? "instance " : "";
    char idx[32] = "";
    if (inst >= 0) snprintf(idx, sizeof idx, "%d: ", inst);
    if (s.status == FX_ENOCONV)
        return fail(FX_ENOCONV, "%s%sno convergence in %d cycles: |r|/|f| = %.3e", who, idx, s.cycles,
                    s.fn2 > 0 ? std::sqrt(s.rn2 / s.fn2) : 0.0);
    if (s.status == FX_ENONFINITE) return fail(FX_ENONFINITE, "%s%snon-finite residual", who, idx);
    return FX_OK;
}

fx_status get_field_impl(Engine *e, int i, int which, double *h_out) {
    if (which < FX_FIELD_P || which > FX_FIELD_PHI_PREV3) return fail(FX_EINVAL, "unknown field %d", which);
    fx_status st = sync_to_caller(e);
    if (st) return st;
    const InstHost &h = e->in[i];
    const InstState &s = e->mir[i];
    const Plan &p = h.plan;
    const size_t nxy = (size_t)p.nx * p.ny, n = nxy * p.nz;
    if (which >= FX_FIELD_PHI_PREV) {
        const int m = which - FX_FIELD_PHI_PREV;
        if (m >= s.hist) return fail(FX_ESTATE, "time level n-%d is not held", m + 1);
        // device planes from the history buffer, contacts from the caller's array
        HIP_OK(hipMemcpyAsync(h_out, h.phi[0], n * sizeof(double), hipMemcpyDeviceToHost, e->st));
        HIP_OK(hipMemcpyAsync(h_out + p.kb * nxy, h.phi[s.prev[m]] + p.kb * nxy, (size_t)p.nzd * nxy * sizeof(double),
                              hipMemcpyDeviceToHost, e->st));
    } else {
        HIP_OK(hipMemcpyAsync(h_out, which == FX_FIELD_P ? h.P[0] : h.phi[0], n * sizeof(double),
                              hipMemcpyDeviceToHost, e->st));
    }
    HIP_OK(hipStreamSynchronize(e->st));
    return FX_OK;
}

fx_status set_field_impl(Engine *e, int i, int which, const double *h_in) {
    if (which < FX_FIELD_P || which > FX_FIELD_PHI_PREV3) return fail(FX_EINVAL, "unknown field %d", which);
    fx_status st = sync_to_caller(e);
    if (st) return st;
    InstHost &h = e->in[i];
    InstState &s = e->mir[i];
    const Plan &p = h.plan;
    const size_t nxy = (size_t)p.nx * p.ny, n = nxy * p.nz;
    if (which >= FX_FIELD_PHI_PREV) {
        const int m = which - FX_FIELD_PHI_PREV;
        if (m != s.hist) return fail(FX_ESTATE, "set time level n-%d after n-1 .. n-%d", m + 1, m);
        int b = 1;                      // cur is 0 after sync_to_caller
        while (holds_history(s, b)) ++b;
        HIP_OK(hipMemcpyAsync(h.phi[b] + p.kb * nxy, h_in + p.kb * nxy, (size_t)p.nzd * nxy * sizeof(double),
                              hipMemcpyHostToDevice, e->st));
        HIP_OK(hipStreamSynchronize(e->st));
        s.prev[m] = b;
        s.hist = m + 1;
        put_state(e, i);
        return FX_OK;
    }
    s.hist = 0;
    s.pstar = -1;
    put_state(e, i);
    if (which == FX_FIELD_P) {
        HIP_OK(hipMemcpyAsync(h.P[0], h_in, n * sizeof(double), hipMemcpyHostToDevice, e->st));
        HIP_OK(hipStreamSynchronize(e->st));
        if (p.f0 >= 0) {
            if (p.f0 > 0) launch_fill(h.P[0], (size_t)p.f0 * nxy, 0.0, e->st);
            if (p.f1 < p.nz) launch_fill(h.P[0] + (size_t)p.f1 * nxy, (size_t)(p.nz - p.f1) * nxy, 0.0, e->st);
        } else {
            launch_fill(h.P[0], n, 0.0, e->st);
        }
    } else {
        HIP_OK(hipMemcpyAsync(h.phi[0], h_in, n * sizeof(double), hipMemcpyHostToDevice, e->st));
        HIP_OK(hipStreamSynchronize(e->st));
        fill_contacts(e, i, true);
    }
    return FX_OK;
}

fx_status probe_on(Engine *e, int kernel, int max_launches, int stride) {
    if (kernel != FX_PROBE_OFF && kernel != FX_PROBE_SMOOTH_FINE) return fail(FX_EINVAL, "unknown probe %d", kernel);
    if (kernel == FX_PROBE_OFF) { e->probe = 0; return FX_OK; }
    if (max_launches < 1 || max_launches > kProbeMax)
        return fail(FX_EINVAL, "max_launches must be in 1..%d", kProbeMax);
    if (stride < 1) return fail(FX_EINVAL, "stride must be >= 1");
    HIP_OK(hipStreamSynchronize(e->st));
    while ((int)e->ev.size() < 2 * max_launches) {
        hipEvent_t ev;
        HIP_OK(hipEventCreate(&ev));
        e->ev.push_back(ev);
    }
    e->ev.resize(2 * max_launches);
    launch_fill(e->probe_dev, kProbeMax, 0.0, e->st);
    HIP_OK(hipStreamSynchronize(e->st));
    e->probe = kernel;
    e->probe_stride = stride;
    e->probe_seen = 0;
    e->ev_used = 0;
    return FX_OK;
}

// Launches in which no instance worked (all solves stopped) carry no bytes
// and are left out.
fx_status probe_read(Engine *e, double *total_ms, int *launches, double *bytes) {
    HIP_OK(hipStreamSynchronize(e->st));
    const int nl = e->ev_used / 2;
    std::vector<double> b(std::max(nl, 1));
    if (nl > 0) HIP_OK(hipMemcpy(b.data(), e->probe_dev, nl * sizeof(double), hipMemcpyDeviceToHost));
    double tot = 0.0, by = 0.0;
    int cnt = 0;
    for (int q = 0; q < nl; ++q) {
        if (!(b[q] > 0)) continue;
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, e->ev[2 * q], e->ev[2 * q + 1]));
        tot += ms;
        by += b[q];
        ++cnt;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    if (bytes) *bytes = by;
    return FX_OK;
}

// ---------------------------------------------------------------- autotuner
// For every level with its own smoother launches, the candidate launch shapes
// (tile 32x8, 64x4 or 128x2 threads; 1, 2, 4 or 8 planes per thread; the
// compiler's register budget or one for 8 waves per SIMD) are timed on the
// live level arrays, and the fastest is kept.  The arithmetic of a cell does
// not depend on the shape, so results are bitwise unchanged.  Choices are
// cached in a text file, one line per (device, precision, level composition):
//   <key> -> <log2 tile x> <planes per thread> <8-wave budget> <us per half-sweep>
constexpr int kTuneVersion = 1;
constexpr int kTuneReps = 10;

uint64_t fnv1a(const std::string &t) {
    uint64_t h = 1469598103934665603ULL;
    for (unsigned char c : t) { h ^= c; h *= 1099511628211ULL; }
    return h;
}

std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t pr;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    for (char &c : a)
        if (c == ' ') c = '_';
    return a + "/" + std::to_string(pr.multiProcessorCount);
}

std::string tune_key(const Engine *e, int l, const std::string &dev) {
    std::string sig;
    size_t cells = 0;
    for (const InstHost &h : e->in) {
        if (l >= h.plan.lc) continue;
        const HostLevel &H = h.plan.lv[l];
        sig += std::to_string(H.nx) + "x" + std::to_string(H.ny) + "x" + std::to_string(H.nz) + (H.rb ? "r" : "n") +
               std::to_string(H.sig_hi - H.sig_lo) + ";";
        cells += H.ncell();
    }
    char buf[256];
    snprintf(buf, sizeof buf, "v%d %s %s smooth %016llx %zu", kTuneVersion, dev.c_str(),
             e->prec == FX_PREC_MIXED ? "f32" : "f64", (unsigned long long)fnv1a(sig), cells);
    return buf;
}

struct TuneEntry {
    SmoothCfg c;
    double us;
};

std::vector<std::pair<std::string, TuneEntry>> read_tune_cache(const char *path) {
    std::vector<std::pair<std::string, TuneEntry>> out;
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f) return out;
    char line[1024];
    while (fgets(line, sizeof line, f)) {
        std::string t(line);
        const size_t arrow = t.find(" -> ");
        if (arrow == std::string::npos) continue;
        TuneEntry te;
        if (sscanf(t.c_str() + arrow + 4, "%d %d %d %lf", &te.c.lbx, &te.c.zt, &te.c.w8, &te.us) != 4) continue;
        const bool ok = te.c.lbx >= 5 && te.c.lbx <= 7 && (te.c.zt == 1 || te.c.zt == 2 || te.c.zt == 4 || te.c.zt == 8) &&
                        (te.c.w8 == 0 || te.c.w8 == 1);
        if (ok) out.emplace_back(t.substr(0, arrow), te);
    }
    fclose(f);
    return out;
}

// Prefix table of level l's smoother launches for launch shape c.
fx_status set_smooth_work(Engine *e, int l, const SmoothCfg &c) {
    const int n = e->n;
    // this level's smoother table, wherever build_work placed it
    const size_t tab = (size_t)(e->w_sm[l].prefix - e->prefix_dev) / (size_t)(n + 1);
    int *hp = e->prefix_host.data() + tab * (n + 1);
    long long tot = 0;
    hp[0] = 0;
    for (int i = 0; i < n; ++i) {
        const InstHost &h = e->in[i];
        tot += l < h.plan.lc ? tiles_smooth(h.plan.lv[l], c) : 0;
        if (tot > (1LL << 30)) return fail(FX_EINVAL, "a launch would exceed 2^30 tiles");
        hp[i + 1] = (int)tot;
    }
    HIP_OK(hipStreamSynchronize(e->st));
    HIP_OK(hipMemcpy(e->prefix_dev + tab * (n + 1), hp, (n + 1) * sizeof(int), hipMemcpyHostToDevice));
    e->w_sm[l].total = (int)tot;
    return FX_OK;
}

template <typename T>
fx_status time_smooth(Engine *e, int l, const SmoothCfg &c, hipEvent_t ev0, hipEvent_t ev1, double *us) {
    fx_status st = set_smooth_work(e, l, c);
    if (st) return st;
    const Inst<T> *I = idev<T>(e);
    double best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
        for (int q = 0; q < 2; ++q) launch_smooth(I, e->w_sm[l], l, q & 1, 0, 0, c, nullptr, e->st);
        HIP_OK(hipEventRecord(ev0, e->st));
        for (int q = 0; q < kTuneReps; ++q) launch_smooth(I, e->w_sm[l], l, q & 1, 0, 0, c, nullptr, e->st);
        HIP_OK(hipEventRecord(ev1, e->st));
        HIP_OK(hipEventSynchronize(ev1));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, ev0, ev1));
        best = std::min(best, 1e3 * ms / kTuneReps);
    }
    *us = best;
    return FX_OK;
}

void drop_graphs(Engine *e) {
    for (int q = 0; q < kUnitPow; ++q)
        if (e->unit_exec[q]) {
            (void)hipGraphExecDestroy(e->unit_exec[q]);
            e->unit_exec[q] = nullptr;
        }
}

template <typename T>
fx_status autotune_t(Engine *e, const char *path, int flags, fx_tune_info *info) {
    fx_tune_info ti{};
    HIP_OK(hipStreamSynchronize(e->st));
    // every instance's kernels must run while timing: done = 0, restored after
    std::vector<InstState> saved(e->mir, e->mir + e->n);
    for (int i = 0; i < e->n; ++i) {
        InstState t = saved[i];
        t.done = 0;
        launch_put_state(e->st_dev + i, t, e->st);
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    HIP_OK(hipEventCreate(&ev0));
    HIP_OK(hipEventCreate(&ev1));
    const std::string dev = device_tag();
    const auto cache = read_tune_cache(path);
    FILE *out = nullptr;
    fx_status st = FX_OK;
    for (int l = 0; l < e->max_lc && !st; ++l) {
        ++ti.levels;
        const std::string key = tune_key(e, l, dev);
        const TuneEntry *hit = nullptr;
        for (const auto &kv : cache)
            if (kv.first == key) hit = &kv.second;          // the last entry wins
        SmoothCfg pick = e->scfg[l];
        if (hit && !(flags & FX_TUNE_FORCE)) {
            pick = hit->c;
            ++ti.from_cache;
        } else {
            int min_nz = 1 << 30;
            for (const InstHost &h : e->in)
                if (l < h.plan.lc) min_nz = std::min(min_nz, h.plan.lv[l].nz);
            double def_us = 0.0, best_us;
            if ((st = time_smooth<T>(e, l, pick, ev0, ev1, &def_us))) break;
            best_us = def_us;
            ++ti.configs_timed;
            for (int lbx = 5; lbx <= 7 && !st; ++lbx)
                for (int zt : {1, 2, 4, 8})
                    for (int w8 = 0; w8 <= 1; ++w8) {
                        if (zt > 1 && zt > min_nz) continue;
                        const SmoothCfg c{lbx, zt, w8};
                        if (c.lbx == pick.lbx && c.zt == pick.zt && c.w8 == pick.w8) continue;
                        double us = 0.0;
                        if ((st = time_smooth<T>(e, l, c, ev0, ev1, &us))) break;
                        ++ti.configs_timed;
                        if (us < 0.98 * best_us) { best_us = us; pick = c; }
                    }
            if (st) break;
            ti.default_us += def_us;
            ti.tuned_us += best_us;
            if (path) {
                if (!out) out = fopen(path, "a");
                if (out) {
                    fprintf(out, "%s -> %d %d %d %.3f\n", key.c_str(), pick.lbx, pick.zt, pick.w8, best_us);
                    ti.cache_written = 1;
                }
            }
        }
        e->scfg[l] = pick;
        if (!st) st = set_smooth_work(e, l, pick);
    }
    if (out) fclose(out);
    for (int i = 0; i < e->n; ++i) launch_put_state(e->st_dev + i, saved[i], e->st);
    hipError_t er = hipStreamSynchronize(e->st);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    drop_graphs(e);
    if (st) return st;
    if (er != hipSuccess) return fail(FX_EDEVICE, "autotune: %s", hipGetErrorString(er));
    if (info) *info = ti;
    return FX_OK;
}

fx_status autotune(Engine *e, const char *path, int flags, fx_tune_info *info) {
    return e->prec == FX_PREC_MIXED ? autotune_t<float>(e, path, flags, info) : autotune_t<double>(e, path, flags, info);
}

}  // namespace

struct fx_stack {
    Engine e;
};

struct fx_batch {
    Engine e;
};

// ------------------------------------------------- learned start helpers
namespace {

fx_status check_unet(const Engine *e, fx_unet *u) {
    if (!u) return fail(FX_EINVAL, "network is NULL");
    int nx, ny, nz;
    hipStream_t ust;
    unet_geometry(u, &nx, &ny, &nz, &ust);
    const Plan &p = e->in[0].plan;
    if (nx != p.nx || ny != p.ny || nz != p.nzd)
        return fail(FX_EINVAL, "network slab %dx%dx%d differs from the stack's device slab %dx%dx%d", nx, ny, nz, p.nx,
                    p.ny, p.nzd);
    return FX_OK;
}

// Per-plane tables of the stack's device planes for the network.
fx_status unet_tables(const Engine *e, fx_unet *u, double v_top, bool doping) {
    const InstHost &h = e->in[0];
    const Plan &p = h.plan;
    std::vector<double> eps(p.nzd), dop(p.nzd);
    for (int k = 0; k < p.nzd; ++k) {
        eps[k] = h.eps_r[p.kb + k];
        dop[k] = h.mat[p.kb + k] == FX_MAT_SC ? h.Nd[p.kb + k] - h.Na[p.kb + k] : 0.0;
    }
    fx_status st = unet_upload_lin(u, eps.data(), h.d.v_bottom, v_top);
    if (!st && doping) st = unet_upload_doping(u, dop.data());
    return st;
}

}  // namespace


// ------------------------------------------- workspace without allocation
// The workspace of poisson_solve_static: a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends.  Host code never
// uses the array's name as an address: each device's copy is looked up once,
// with that device current, and that address is what the kernels receive.
constexpr size_t kStaticWsBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of the static workspace.
fx_status static_workspace(void **out) {
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FX_EDEVICE, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t err = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr)
            return fail(FX_EDEVICE, "hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(err));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FX_OK;
}

}  // namespace

extern "C" {

size_t stack_workspace_bytes(const fx_stack_desc *desc) {
    g_err.clear();
    Engine tmp;
    if (validate_all(desc, 1, &tmp)) return 0;
    plan_launches(&tmp);
    return carve(&tmp, nullptr);
}

fx_status init_stack(const fx_stack_desc *desc, double *d_P, double *d_phi, void *d_ws, size_t ws_bytes,
                     void *stream, fx_stack **out) {
    g_err.clear();
    if (!out) return fail(FX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_P || !d_phi || !d_ws) return fail(FX_EINVAL, "device pointers must not be NULL");
    if (((uintptr_t)d_ws & 255) != 0) return fail(FX_EINVAL, "workspace must be 256-byte aligned");
    if (((uintptr_t)d_P & 15) != 0 || ((uintptr_t)d_phi & 15) != 0)
        return fail(FX_EINVAL, "d_P and d_phi must be 16-byte aligned");
    fx_stack *s = new (std::nothrow) fx_stack();
    if (!s) return fail(FX_ENOMEM, "host allocation failed");
    Engine *e = &s->e;
    fx_status st = validate_all(desc, 1, e);
    if (st) { delete s; return st; }
    plan_launches(e);
    e->mode = env_mode(FX_LAUNCH_STREAM);
    st = engine_init(e, &d_P, &d_phi, d_ws, ws_bytes, stream);
    if (st == FX_ENOMEM || st == FX_EINVAL || (st == FX_EDEVICE && !e->mir)) {
        engine_release(e);
        delete s;
        return st;
    }
    *out = s;
    if (st) return st;
    fx_status st2 = sync_to_caller(e);
    if (!st2) st2 = status_message(e->mir[0], -1);
    return st2;
}

fx_status poisson_solve_static(const fx_stack_desc *desc, double *d_P, double *d_phi, void *stream,
                               fx_solve_info *info) {
    g_err.clear();
    if (!d_P || !d_phi) return fail(FX_EINVAL, "device pointers must not be NULL");
    if (((uintptr_t)d_P & 15) != 0 || ((uintptr_t)d_phi & 15) != 0)
        return fail(FX_EINVAL, "d_P and d_phi must be 16-byte aligned");
    Engine e;
    e.no_alloc = 1;
    fx_status st = validate_all(desc, 1, &e);
    if (st) return st;
    plan_launches(&e);
    e.mode = FX_LAUNCH_STREAM;                     // no graphs: capturing one would allocate
    const size_t need = carve(&e, nullptr);
    if (need > kStaticWsBytes)
        return fail(FX_ENOMEM, "this stack needs %zu bytes of workspace; the static workspace holds %zu", need,
                    kStaticWsBytes);
    void *ws = nullptr;
    if ((st = static_workspace(&ws))) return st;
    st = engine_init(&e, &d_P, &d_phi, ws, kStaticWsBytes, stream);
    if (!st || st == FX_ENOCONV || st == FX_ENONFINITE) {
        const fx_status st2 = sync_to_caller(&e);
        if (!st2 && e.mir) {
            const InstState &c = e.mir[0];
            if (info) {
                info->cycles = c.cycles;
                info->status = c.status;
                info->res_norm = c.status == FX_OK && c.zero_fix ? 0.0 : std::sqrt(c.rn2);
                info->rhs_norm = std::sqrt(c.fn2);
            }
            if (!st) st = status_message(c, -1);
        } else if (st2) {
            st = st2;
        }
    }
    engine_release(&e);
    return st;
}

fx_status tdgl_step(fx_stack *s, double dt) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (!(dt > 0)) return fail(FX_EINVAL, "dt must be > 0");
    Engine *e = &s->e;
    e->mir[0].dt = dt;
    put_state(e, 0);
    if (e->prec == FX_PREC_MIXED) {
        launch_tdgl(idev<float>(e), e->w_tdgl, 0, e->st);
        launch_flip(idev<float>(e), 1, e->st);
    } else {
        launch_tdgl(idev<double>(e), e->w_tdgl, 0, e->st);
        launch_flip(idev<double>(e), 1, e->st);
    }
    e->mir[0].pcur ^= 1;
    e->mir[0].hist = 0;
    e->mir[0].pstar = -1;
    return sync_to_caller(e);
}

fx_status poisson_solve(fx_stack *s, double v_top, fx_solve_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (!std::isfinite(v_top)) return fail(FX_EINVAL, "v_top must be finite");
    Engine *e = &s->e;
    e->mir[0].v_top = v_top;
    put_state(e, 0);
    fx_status st = solve_plain(e);
    if (st) return st;
    const InstState c = e->mir[0];
    if (info) {
        info->cycles = c.cycles;
        info->status = c.status;
        info->res_norm = c.status == FX_OK && c.zero_fix ? 0.0 : std::sqrt(c.rn2);
        info->rhs_norm = std::sqrt(c.fn2);
    }
    st = sync_to_caller(e);
    if (st) return st;
    return status_message(c, -1);
}

static fx_status run_steps_impl(fx_stack *s, int nsteps, double dt, const double *h_v_top_sched, double *h_Q,
                                double *h_V_fe, fx_run_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (nsteps < 0 || !(dt > 0)) return fail(FX_EINVAL, "nsteps >= 0 and dt > 0 required");
    Engine *e = &s->e;
    const InstState before = e->mir[0];
    fx_status st = run(e, nsteps, dt, h_v_top_sched ? &h_v_top_sched : nullptr, h_Q ? &h_Q : nullptr,
                       h_V_fe ? &h_V_fe : nullptr);
    if (st) return st;
    const InstState c = e->mir[0];
    fx_run_info ri{};
    if (nsteps > 0) {
        ri.steps_done = c.step - before.step;
        ri.total_cycles = c.total_cycles - before.total_cycles;
        ri.max_cycles_step = c.max_cycles_step;
        ri.last_res_rel = c.fn2 > 0 && !(c.status == FX_OK && c.zero_fix) ? std::sqrt(c.rn2 / c.fn2) : 0.0;
    }
    if (info) *info = ri;
    st = sync_to_caller(e);
    if (st) return st;
    return nsteps > 0 ? status_message(c, -1) : FX_OK;
}

fx_status run_steps(fx_stack *s, int nsteps, double dt, const double *h_v_top_sched, fx_run_info *info) {
    return run_steps_impl(s, nsteps, dt, h_v_top_sched, nullptr, nullptr, info);
}

fx_status run_steps_qv(fx_stack *s, int nsteps, double dt, const double *h_v_top_sched, double *h_Q,
                       double *h_V_fe, fx_run_info *info) {
    if (!h_Q || !h_V_fe) return fail(FX_EINVAL, "Q and V_fe arrays are required");
    if (s && !has_interface(s->e.in[0]))
        return fail(FX_EINVAL, "the ferroelectric has no dielectric neighbour");
    return run_steps_impl(s, nsteps, dt, h_v_top_sched, h_Q, h_V_fe, info);
}

fx_status stack_qv(fx_stack *s, double *h_Q, double *h_V_fe) {
    g_err.clear();
    if (!s || !h_Q || !h_V_fe) return fail(FX_EINVAL, "NULL argument");
    if (!has_interface(s->e.in[0])) return fail(FX_EINVAL, "the ferroelectric has no dielectric neighbour");
    return qv_now(&s->e, h_Q, h_V_fe);
}

fx_status get_field(fx_stack *s, int which, double *h_out) {
    g_err.clear();
    if (!s || !h_out) return fail(FX_EINVAL, "NULL argument");
    return get_field_impl(&s->e, 0, which, h_out);
}

fx_status set_field(fx_stack *s, int which, const double *h_in) {
    g_err.clear();
    if (!s || !h_in) return fail(FX_EINVAL, "NULL argument");
    return set_field_impl(&s->e, 0, which, h_in);
}

fx_status stack_set_launch(fx_stack *s, int mode) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (mode != FX_LAUNCH_STREAM && mode != FX_LAUNCH_GRAPH) return fail(FX_EINVAL, "unknown launch mode %d", mode);
    s->e.mode = mode;
    return FX_OK;
}

fx_status stack_autotune(fx_stack *s, const char *cache_path, int flags, fx_tune_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (flags & ~FX_TUNE_FORCE) return fail(FX_EINVAL, "unknown flags %d", flags);
    return autotune(&s->e, cache_path, flags, info);
}

fx_status stack_tune_config(const fx_stack *s, int level, int *tile_x, int *zt, int *waves8) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (level < 0 || level >= s->e.max_lc) return fail(FX_EINVAL, "level %d has no smoother launches", level);
    const SmoothCfg &c = s->e.scfg[level];
    if (tile_x) *tile_x = 1 << c.lbx;
    if (zt) *zt = c.zt;
    if (waves8) *waves8 = c.w8;
    return FX_OK;
}

fx_status stack_probe(fx_stack *s, int kernel, int max_launches, int stride) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    return probe_on(&s->e, kernel, max_launches, stride);
}

fx_status stack_probe_read(fx_stack *s, double *total_ms, int *launches, double *bytes) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    return probe_read(&s->e, total_ms, launches, bytes);
}

int stack_num_levels(const fx_stack *s) { return s ? (int)s->e.in[0].plan.lv.size() : 0; }

fx_status stack_level_shape(const fx_stack *s, int level, int *nx, int *ny, int *nz) {
    if (!s || level < 0 || level >= (int)s->e.in[0].plan.lv.size()) return fail(FX_EINVAL, "bad level");
    const HostLevel &H = s->e.in[0].plan.lv[level];
    if (nx) *nx = H.nx;
    if (ny) *ny = H.ny;
    if (nz) *nz = H.nz;
    return FX_OK;
}

fx_status stack_level_mode(const fx_stack *s, int level, int *mode) {
    if (!s || !mode || level < 0 || level >= (int)s->e.in[0].plan.lv.size()) return fail(FX_EINVAL, "bad level");
    const Engine &e = s->e;
    if (level >= e.in[0].plan.lc) *mode = FX_LEVEL_COARSE;
    else if (level < (int)e.tb.size() && e.tb[level]) *mode = FX_LEVEL_BLOCKED;
    else *mode = FX_LEVEL_LAUNCHES;
    return FX_OK;
}

fx_status destroy_stack(fx_stack *s) {
    if (!s) return FX_OK;
    engine_release(&s->e);
    delete s;
    return FX_OK;
}

// ------------------------------------------------------------------ batches
size_t batch_workspace_bytes(const fx_stack_desc *descs, int n) {
    g_err.clear();
    Engine tmp;
    if (validate_all(descs, n, &tmp)) return 0;
    plan_launches(&tmp);
    return carve(&tmp, nullptr);
}

fx_status init_batch(const fx_stack_desc *descs, int n, double *const *d_P, double *const *d_phi, void *d_ws,
                     size_t ws_bytes, void *stream, fx_batch **out) {
    g_err.clear();
    if (!out) return fail(FX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_P || !d_phi || !d_ws) return fail(FX_EINVAL, "pointers must not be NULL");
    if (((uintptr_t)d_ws & 255) != 0) return fail(FX_EINVAL, "workspace must be 256-byte aligned");
    if (n >= 1 && n <= kMaxBatch)
        for (int i = 0; i < n; ++i) {
            if (!d_P[i] || !d_phi[i]) return fail(FX_EINVAL, "instance %d: device pointers must not be NULL", i);
            if (((uintptr_t)d_P[i] & 15) != 0 || ((uintptr_t)d_phi[i] & 15) != 0)
                return fail(FX_EINVAL, "instance %d: P and phi must be 16-byte aligned", i);
        }
    fx_batch *b = new (std::nothrow) fx_batch();
    if (!b) return fail(FX_ENOMEM, "host allocation failed");
    Engine *e = &b->e;
    fx_status st = validate_all(descs, n, e);
    if (st) { delete b; return st; }
    plan_launches(e);
    e->mode = env_mode(FX_LAUNCH_GRAPH);
    st = engine_init(e, d_P, d_phi, d_ws, ws_bytes, stream);
    if (st == FX_ENOMEM || st == FX_EINVAL || (st == FX_EDEVICE && !e->mir)) {
        engine_release(e);
        delete b;
        return st;
    }
    *out = b;
    if (st) return st;
    st = sync_to_caller(e);
    if (st) return st;
    for (int i = 0; i < n; ++i)
        if (e->mir[i].status != FX_OK) return status_message(e->mir[i], i);
    return FX_OK;
}

static fx_status run_batch_impl(fx_batch *b, int nsteps, double dt, const double *const *h_v_top_sched,
                                double *const *h_Q, double *const *h_V_fe, fx_batch_info *info) {
    g_err.clear();
    if (!b) return fail(FX_EINVAL, "batch is NULL");
    if (nsteps < 0 || !(dt > 0)) return fail(FX_EINVAL, "nsteps >= 0 and dt > 0 required");
    Engine *e = &b->e;
    if (h_v_top_sched)
        for (int i = 0; i < e->n; ++i)
            if (!h_v_top_sched[i]) return fail(FX_EINVAL, "instance %d: schedule is NULL", i);
    if (h_Q)
        for (int i = 0; i < e->n; ++i)
            if (!h_Q[i] || !h_V_fe[i]) return fail(FX_EINVAL, "instance %d: Q or V_fe array is NULL", i);
    std::vector<InstState> before(e->mir, e->mir + e->n);
    fx_status st = run(e, nsteps, dt, h_v_top_sched, h_Q, h_V_fe);
    if (st) return st;
    if (info)
        for (int i = 0; i < e->n; ++i) {
            const InstState &c = e->mir[i];
            fx_batch_info &r = info[i];
            r.status = nsteps > 0 ? c.status : FX_OK;
            r.steps_done = c.step - before[i].step;
            r.total_cycles = c.total_cycles - before[i].total_cycles;
            r.max_cycles_step = nsteps > 0 ? c.max_cycles_step : 0;
            r.last_res_rel = nsteps > 0 && c.fn2 > 0 && !(c.status == FX_OK && c.zero_fix) ? std::sqrt(c.rn2 / c.fn2) : 0.0;
        }
    std::vector<InstState> after(e->mir, e->mir + e->n);
    st = sync_to_caller(e);
    if (st) return st;
    if (nsteps > 0)
        for (int i = 0; i < e->n; ++i)
            if (after[i].status != FX_OK) return status_message(after[i], i);
    return FX_OK;
}

fx_status run_batch(fx_batch *b, int nsteps, double dt, const double *const *h_v_top_sched, fx_batch_info *info) {
    return run_batch_impl(b, nsteps, dt, h_v_top_sched, nullptr, nullptr, info);
}

fx_status run_batch_qv(fx_batch *b, int nsteps, double dt, const double *const *h_v_top_sched,
                       double *const *h_Q, double *const *h_V_fe, fx_batch_info *info) {
    if (!h_Q || !h_V_fe) return fail(FX_EINVAL, "Q and V_fe arrays are required");
    return run_batch_impl(b, nsteps, dt, h_v_top_sched, h_Q, h_V_fe, info);
}

fx_status batch_qv(fx_batch *b, double *h_Q, double *h_V_fe) {
    g_err.clear();
    if (!b || !h_Q || !h_V_fe) return fail(FX_EINVAL, "NULL argument");
    return qv_now(&b->e, h_Q, h_V_fe);
}

fx_status batch_get_field(fx_batch *b, int inst, int which, double *h_out) {
    g_err.clear();
    if (!b || !h_out) return fail(FX_EINVAL, "NULL argument");
    if (inst < 0 || inst >= b->e.n) return fail(FX_EINVAL, "instance %d outside 0..%d", inst, b->e.n - 1);
    return get_field_impl(&b->e, inst, which, h_out);
}

fx_status batch_autotune(fx_batch *b, const char *cache_path, int flags, fx_tune_info *info) {
    g_err.clear();
    if (!b) return fail(FX_EINVAL, "batch is NULL");
    if (flags & ~FX_TUNE_FORCE) return fail(FX_EINVAL, "unknown flags %d", flags);
    return autotune(&b->e, cache_path, flags, info);
}

fx_status batch_set_launch(fx_batch *b, int mode) {
    g_err.clear();
    if (!b) return fail(FX_EINVAL, "batch is NULL");
    if (mode != FX_LAUNCH_STREAM && mode != FX_LAUNCH_GRAPH) return fail(FX_EINVAL, "unknown launch mode %d", mode);
    b->e.mode = mode;
    return FX_OK;
}

fx_status batch_level_mode(const fx_batch *b, int level, int *mode) {
    if (!b || !mode || level < 0) return fail(FX_EINVAL, "bad level");
    const Engine &e = b->e;
    if (level >= e.max_lc) *mode = FX_LEVEL_COARSE;
    else *mode = level < (int)e.tb.size() && e.tb[level] ? FX_LEVEL_BLOCKED : FX_LEVEL_LAUNCHES;
    return FX_OK;
}

fx_status destroy_batch(fx_batch *b) {
    if (!b) return FX_OK;
    engine_release(&b->e);
    delete b;
    return FX_OK;
}

fx_status stack_unet_input(fx_stack *s, fx_unet *u, double v_top) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    fx_status st = check_unet(&s->e, u);
    if (st) return st;
    if (!std::isfinite(v_top)) return fail(FX_EINVAL, "v_top must be finite");
    HIP_OK(hipStreamSynchronize(s->e.st));
    if ((st = unet_tables(&s->e, u, v_top, true))) return st;
    const InstHost &h = s->e.in[0];
    const size_t nxy = (size_t)h.plan.nx * h.plan.ny;
    unet_pack_from_f64(u, h.P[0] + h.plan.kb * nxy, v_top);
    HIP_OK(hipGetLastError());
    return FX_OK;
}

fx_status stack_unet_target(fx_stack *s, fx_unet *u, double v_top, float *d_target) {
    g_err.clear();
    if (!s || !d_target) return fail(FX_EINVAL, "NULL argument");
    fx_status st = check_unet(&s->e, u);
    if (st) return st;
    if (!std::isfinite(v_top)) return fail(FX_EINVAL, "v_top must be finite");
    HIP_OK(hipStreamSynchronize(s->e.st));
    if ((st = unet_tables(&s->e, u, v_top, false))) return st;
    const InstHost &h = s->e.in[0];
    const size_t nxy = (size_t)h.plan.nx * h.plan.ny;
    unet_make_target(u, h.phi[0] + h.plan.kb * nxy, d_target);
    int nx, ny, nz;
    hipStream_t ust;
    unet_geometry(u, &nx, &ny, &nz, &ust);
    HIP_OK(hipStreamSynchronize(ust));
    return FX_OK;
}

fx_status stack_learned_solve(fx_stack *s, fx_unet *u, double v_top, fx_solve_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    Engine *e = &s->e;
    fx_status st = check_unet(e, u);
    if (st) return st;
    if (!std::isfinite(v_top)) return fail(FX_EINVAL, "v_top must be finite");
    HIP_OK(hipStreamSynchronize(e->st));
    if ((st = unet_tables(e, u, v_top, true))) return st;
    InstHost &h = e->in[0];
    const size_t nxy = (size_t)h.plan.nx * h.plan.ny;
    unet_pack_from_f64(u, h.P[0] + h.plan.kb * nxy, v_top);
    unet_forward_enqueue(u);
    unet_apply(u, h.phi[0] + h.plan.kb * nxy);
    int nx, ny, nz;
    hipStream_t ust;
    unet_geometry(u, &nx, &ny, &nz, &ust);
    HIP_OK(hipStreamSynchronize(ust));
    HIP_OK(hipGetLastError());
    // phi^n was replaced: the stored time levels no longer precede it
    e->mir[0].hist = 0;
    e->mir[0].pstar = -1;
    put_state(e, 0);
    return poisson_solve(s, v_top, info);
}

const char *last_error(void) { return g_err.c_str(); }

}  // extern "C"
