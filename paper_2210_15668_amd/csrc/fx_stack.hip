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
// mean, prolongation is linear between cell centres (bilinear in x/y,
// distance-weighted in z with a zero correction on contact faces).
#include "fx_internal.h"
#include "../../include/ferrox.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
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

constexpr int kBottomMaxCells = 2048;   // must not exceed the bottom kernel's LDS arrays
constexpr int kBottomTarget = 64;

// One multigrid level, host view.
struct HostLevel {
    int nx = 0, ny = 0, nz = 0;
    int xy_from_finer = 0;              // x,y halved relative to the finer level
    int z_from_finer = 0;               // z paired relative to the finer level
    std::vector<int> s0, e0;            // covered finest device planes [s0, e0)
    std::vector<double> cxy, czm, czp, dg;
    std::vector<int> ks, cnt;           // restriction map from the finer level
    std::vector<int> pka, pkb;          // prolongation map of the finer level's planes
    std::vector<double> pwa, pwb;
    int sig_lo = 0, sig_hi = 0;
    size_t ncell() const { return (size_t)nx * ny * nz; }
    size_t nsig() const { return (size_t)nx * ny * (sig_hi - sig_lo); }
};

struct Plan {
    int nx, ny, nz, kb, kt, nzd, f0, f1, sc0, sc1;
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
};

fx_status validate(const fx_stack_desc *d, Plan *p) {
    if (!d) return fail(FX_EINVAL, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(FX_EINVAL, "grid sizes must be >= 1");
    if (!(d->h > 0) || !(d->Gamma > 0) || !(d->gamma > 0))
        return fail(FX_EINVAL, "h, Gamma and gamma must be > 0");
    if (d->pbc < 0 || d->pbc > 2) return fail(FX_EINVAL, "unknown pbc %d", d->pbc);
    if (d->pbc == FX_PBC_LAMBDA && !(d->lambda >= 0)) return fail(FX_EINVAL, "lambda must be >= 0");
    if (!d->plane_mat || !d->plane_eps_r || !d->plane_Na || !d->plane_Nd)
        return fail(FX_EINVAL, "plane tables must not be NULL");
    if (d->prec != FX_PREC_FP64 && d->prec != FX_PREC_MIXED) return fail(FX_EINVAL, "unknown precision");
    if (!(d->tol_rel > 0) || d->max_cycles < 1) return fail(FX_EINVAL, "tol_rel > 0 and max_cycles >= 1 required");
    if (d->flags != 0) return fail(FX_EINVAL, "flags must be 0");
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
        if (!(d->T > 0) || !(d->ni > 0)) return fail(FX_EINVAL, "T and ni must be > 0 with a semiconductor");
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
        if (F.ncell() <= (size_t)kBottomTarget) break;
        const bool cxy = F.nx % 2 == 0 && F.ny % 2 == 0 && F.nx >= 4 && F.ny >= 4;
        const bool cz = F.nz >= 2;
        if (!cxy && !cz) break;
        HostLevel C;
        C.xy_from_finer = cxy; C.z_from_finer = cz;
        C.nx = cxy ? F.nx / 2 : F.nx;
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
        if (p->lv.size() > 40) break;
    }
    // If the coarsest level is still too big for the one-workgroup bottom
    // solve, drop nothing: the driver smooths it with the general kernels.
    const int nlev = (int)p->lv.size();
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
                const double wa = (zf - zn) / (zc[K] - zn);
                F.pwa[k] = wa;
                F.pwb[k] = 1.0 - wa;
                F.pkb[k] = kn;
            }
        }
    }
}

}  // namespace

struct fx_stack {
    fx_stack_desc d{};
    std::vector<int> mat;
    std::vector<double> eps_r, Na, Nd;
    Plan plan;
    hipStream_t st = nullptr;
    double *P[2] = {nullptr, nullptr};
    int pcur = 0;
    double *phi = nullptr;
    // finest-level FP64 tables
    double *t_cxy, *t_czm, *t_czp, *t_wl, *t_wr, *t_p0e, *t_n0e;
    int *t_flags;
    std::vector<DevLevel<double>> L64;
    std::vector<DevLevel<float>> L32;
    double *part = nullptr;
    int part_n = 0;
    double *norms_dev = nullptr;
    double *norms_host = nullptr;     // pinned
    double *phi_save = nullptr;
    double VT = 0.0, scale = 0.0;
    double dmax = 0.0;
    int nu1 = 2, nu2 = 2, bottom_sweeps = 40;
};

namespace {

// Lay out (or size) the workspace.  With s->... pointers null it only counts.
size_t carve(fx_stack *s, void *ws) {
    Carver cv(ws);
    const Plan &p = s->plan;
    const size_t nfull = (size_t)p.nx * p.ny * p.nz;
    s->P[1] = (double *)cv.take(nfull * sizeof(double));
    s->phi_save = (double *)cv.take(nfull * sizeof(double));
    const int nzd = p.nzd;
    s->t_cxy = (double *)cv.take(nzd * sizeof(double));
    s->t_czm = (double *)cv.take(nzd * sizeof(double));
    s->t_czp = (double *)cv.take(nzd * sizeof(double));
    s->t_wl = (double *)cv.take(nzd * sizeof(double));
    s->t_wr = (double *)cv.take(nzd * sizeof(double));
    s->t_p0e = (double *)cv.take(nzd * sizeof(double));
    s->t_n0e = (double *)cv.take(nzd * sizeof(double));
    s->t_flags = (int *)cv.take(nzd * sizeof(int));
    const int nlev = (int)p.lv.size();
    const bool mixed = s->d.prec == FX_PREC_MIXED;
    s->L64.assign(nlev, DevLevel<double>());
    s->L32.assign(nlev, DevLevel<float>());
    for (int l = 0; l < nlev; ++l) {
        const HostLevel &H = p.lv[l];
        const size_t n = H.ncell(), ns = H.nsig();
        const int nz = H.nz;
        auto ints = [&](int **dst) { *dst = (int *)cv.take(nz * sizeof(int)); };
        if (!mixed) {
            DevLevel<double> &D = s->L64[l];
            D.e = (double *)cv.take(n * 8); D.r = (double *)cv.take(n * 8); D.sig = (double *)cv.take(ns * 8);
            D.cxy = (double *)cv.take(nz * 8); D.czm = (double *)cv.take(nz * 8);
            D.czp = (double *)cv.take(nz * 8); D.dg = (double *)cv.take(nz * 8);
            D.pwa = (double *)cv.take(nz * 8); D.pwb = (double *)cv.take(nz * 8);
            ints(&D.ks); ints(&D.cnt); ints(&D.thick); ints(&D.pka); ints(&D.pkb);
        } else {
            DevLevel<float> &D = s->L32[l];
            D.e = (float *)cv.take(n * 4); D.r = (float *)cv.take(n * 4); D.sig = (float *)cv.take(ns * 4);
            D.cxy = (float *)cv.take(nz * 4); D.czm = (float *)cv.take(nz * 4);
            D.czp = (float *)cv.take(nz * 4); D.dg = (float *)cv.take(nz * 4);
            D.pwa = (float *)cv.take(nz * 4); D.pwb = (float *)cv.take(nz * 4);
            ints(&D.ks); ints(&D.cnt); ints(&D.thick); ints(&D.pka); ints(&D.pkb);
        }
    }
    // residual partial sums: one pair per 64x4 block of the finest level
    const size_t nb = (size_t)((p.nx + 63) / 64) * ((p.ny + 3) / 4) * nzd;
    s->part_n = (int)nb;
    s->part = (double *)cv.take(2 * nb * sizeof(double));
    s->norms_dev = (double *)cv.take(4 * sizeof(double));
    return cv.off + 256;
}

template <typename T>
fx_status upload_level(const HostLevel &H, DevLevel<T> &D) {
    std::vector<T> a(H.nz);
    auto up = [&](T *dst, const std::vector<double> &src) -> fx_status {
        for (int K = 0; K < H.nz; ++K) a[K] = (T)src[K];
        HIP_OK(hipMemcpy(dst, a.data(), H.nz * sizeof(T), hipMemcpyHostToDevice));
        return FX_OK;
    };
    auto upi = [&](int *dst, const std::vector<int> &src) -> fx_status {
        std::vector<int> v(src);
        v.resize(H.nz, 0);
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
    std::vector<int> pkb(H.pkb);
    pkb.resize(H.nz, -1);
    if ((st = upi(D.ks, H.ks)) || (st = upi(D.cnt, H.cnt)) || (st = upi(D.thick, thick)) ||
        (st = upi(D.pka, H.pka)) || (st = upi(D.pkb, pkb)))
        return st;
    return FX_OK;
}

template <typename T>
LevelArgs<T> level_args(const fx_stack *s, const std::vector<DevLevel<T>> &LV, int l) {
    const HostLevel &H = s->plan.lv[l];
    LevelArgs<T> a;
    a.nx = H.nx; a.ny = H.ny; a.nz = H.nz;
    a.cxy = LV[l].cxy; a.czm = LV[l].czm; a.czp = LV[l].czp; a.dg = LV[l].dg;
    a.e = LV[l].e; a.r = LV[l].r; a.sig = LV[l].sig;
    a.sig_lo = H.sig_lo; a.sig_hi = H.sig_hi;
    return a;
}

template <typename T>
void vcycle(fx_stack *s, const std::vector<DevLevel<T>> &LV, int l) {
    const int nlev = (int)s->plan.lv.size();
    hipStream_t st = s->st;
    LevelArgs<T> A = level_args(s, LV, l);
    if (l == nlev - 1) {
        if (s->plan.lv[l].ncell() <= (size_t)kBottomMaxCells) {
            launch_bottom(A, s->bottom_sweeps, st);
        } else {
            launch_smooth(A, 0, 1, st);
            launch_smooth(A, 1, 0, st);
            for (int q = 1; q < 4 * s->bottom_sweeps; ++q) { launch_smooth(A, 0, 0, st); launch_smooth(A, 1, 0, st); }
        }
        return;
    }
    launch_smooth(A, 0, 1, st);
    launch_smooth(A, 1, 0, st);
    for (int q = 1; q < s->nu1; ++q) { launch_smooth(A, 0, 0, st); launch_smooth(A, 1, 0, st); }
    RestrictArgs<T> R;
    R.f = A;
    R.c = level_args(s, LV, l + 1);
    R.fthick = LV[l].thick; R.cthick = LV[l + 1].thick;
    R.cks = LV[l + 1].ks; R.ccnt = LV[l + 1].cnt;
    R.xy = s->plan.lv[l + 1].xy_from_finer;
    launch_restrict(R, st);
    vcycle(s, LV, l + 1);
    ProlongArgs<T> Pg;
    Pg.f = A;
    Pg.c = R.c;
    Pg.ka = LV[l].pka; Pg.kb = LV[l].pkb; Pg.wa = LV[l].pwa; Pg.wb = LV[l].pwb;
    Pg.xy = R.xy;
    launch_prolong(Pg, st);
    for (int q = 0; q < s->nu2; ++q) { launch_smooth(A, 0, 0, st); launch_smooth(A, 1, 0, st); }
}

template <typename T>
void residual(fx_stack *s, T *r0, T *sig0) {
    const Plan &p = s->plan;
    ResArgs<T> a;
    a.nx = p.nx; a.ny = p.ny; a.nzd = p.nzd; a.kb = p.kb;
    a.v_b = s->d.v_bottom; a.v_t = s->d.v_top;
    a.p_scale = s->d.h / kEps0;
    a.rho_scale = s->scale;
    a.vt_inv = s->VT > 0 ? 1.0 / s->VT : 0.0;
    a.sig_scale = s->VT > 0 ? s->scale / s->VT : 0.0;
    a.cxy = s->t_cxy; a.czm = s->t_czm; a.czp = s->t_czp;
    a.wl = s->t_wl; a.wr = s->t_wr; a.p0e = s->t_p0e; a.n0e = s->t_n0e; a.pflags = s->t_flags;
    a.phi = s->phi; a.P = s->P[s->pcur];
    a.r = r0; a.sig = sig0;
    a.sig_lo = p.lv[0].sig_lo; a.sig_hi = p.lv[0].sig_hi;
    a.part = s->part;
    int nb = 0;
    launch_residual(a, s->st, &nb);
    launch_reduce_norms(s->part, nb, s->norms_dev, s->st);
}

fx_status read_norms(fx_stack *s, double *rn, double *fn) {
    HIP_OK(hipMemcpyAsync(s->norms_host, s->norms_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    *rn = std::sqrt(s->norms_host[0]);
    *fn = std::sqrt(s->norms_host[1]);
    return FX_OK;
}

template <typename T>
fx_status solve_impl(fx_stack *s, const std::vector<DevLevel<T>> &LV, fx_solve_info *info) {
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny;
    double rn = 0, fn = 0;
    HIP_OK(hipMemcpyAsync(s->phi_save + p.kb * nxy, s->phi + p.kb * nxy, p.nzd * nxy * sizeof(double),
                          hipMemcpyDeviceToDevice, s->st));
    residual<T>(s, LV[0].r, LV[0].sig);
    fx_status st = read_norms(s, &rn, &fn);
    if (st) return st;
    if (fn == 0.0 && std::isfinite(rn)) {
        // N(0) = 0 exactly, so phi = 0 is the root of N(phi) = 0
        launch_fill(s->phi + p.kb * nxy, p.nzd * nxy, 0.0, s->st);
        residual<T>(s, LV[0].r, LV[0].sig);
        if ((st = read_norms(s, &rn, &fn))) return st;
    }
    int cyc = 0;
    fx_status res = FX_ENOCONV;
    for (;;) {
        if (!std::isfinite(rn) || !std::isfinite(fn)) { res = FX_ENONFINITE; break; }
        if (rn <= s->d.tol_rel * fn || rn == 0.0) { res = FX_OK; break; }
        if (cyc >= s->d.max_cycles) break;
        vcycle<T>(s, LV, 0);
        launch_update<T>(s->phi, LV[0].e, p.nx, p.ny, p.nzd, p.kb, s->t_flags, s->dmax, s->st);
        residual<T>(s, LV[0].r, LV[0].sig);
        if ((st = read_norms(s, &rn, &fn))) return st;
        ++cyc;
    }
    if (res == FX_ENONFINITE)
        HIP_OK(hipMemcpyAsync(s->phi + p.kb * nxy, s->phi_save + p.kb * nxy, p.nzd * nxy * sizeof(double),
                              hipMemcpyDeviceToDevice, s->st));
    if (info) { info->cycles = cyc; info->status = res; info->res_norm = rn; info->rhs_norm = fn; }
    if (res == FX_ENOCONV) return fail(res, "no convergence in %d cycles: |r|/|f| = %.3e", cyc, rn / fn);
    if (res == FX_ENONFINITE) return fail(res, "non-finite residual");
    return FX_OK;
}

fx_status solve(fx_stack *s, fx_solve_info *info) {
    if (s->d.prec == FX_PREC_MIXED) return solve_impl<float>(s, s->L32, info);
    return solve_impl<double>(s, s->L64, info);
}

fx_status set_contacts(fx_stack *s) {
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny;
    if (p.kb > 0) launch_fill(s->phi, (size_t)p.kb * nxy, s->d.v_bottom, s->st);
    if (p.kt < p.nz) launch_fill(s->phi + (size_t)p.kt * nxy, (size_t)(p.nz - p.kt) * nxy, s->d.v_top, s->st);
    return FX_OK;
}

fx_status tdgl_impl(fx_stack *s, double dt) {
    const Plan &p = s->plan;
    if (p.f0 < 0) return FX_OK;
    TdglArgs a;
    a.nx = p.nx; a.ny = p.ny; a.f0 = p.f0; a.f1 = p.f1;
    a.h = s->d.h; a.dt = dt;
    a.alpha = s->d.alpha; a.beta = s->d.beta; a.gamma = s->d.gamma;
    a.g11 = s->d.g11; a.g44 = s->d.g44; a.Gamma = s->d.Gamma;
    a.pbc = s->d.pbc; a.lambda = s->d.lambda;
    a.P = s->P[s->pcur]; a.phi = s->phi; a.Pn = s->P[1 - s->pcur];
    launch_tdgl(a, s->st);
    s->pcur = 1 - s->pcur;
    return FX_OK;
}

fx_status sync_P_to_caller(fx_stack *s) {
    if (s->pcur == 0) return FX_OK;
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny;
    if (p.f0 >= 0)
        HIP_OK(hipMemcpyAsync(s->P[0] + p.f0 * nxy, s->P[1] + p.f0 * nxy, (p.f1 - p.f0) * nxy * sizeof(double),
                              hipMemcpyDeviceToDevice, s->st));
    s->pcur = 0;
    return FX_OK;
}

}  // namespace

extern "C" {

size_t stack_workspace_bytes(const fx_stack_desc *desc) {
    fx_stack tmp;
    if (validate(desc, &tmp.plan)) return 0;
    tmp.d = *desc;
    build_plan(desc, &tmp.plan);
    return carve(&tmp, nullptr);
}

fx_status init_stack(const fx_stack_desc *desc, double *d_P, double *d_phi, void *d_ws, size_t ws_bytes,
                     void *stream, fx_stack **out) {
    g_err.clear();
    if (!out) return fail(FX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_P || !d_phi || !d_ws) return fail(FX_EINVAL, "device pointers must not be NULL");
    if (((uintptr_t)d_ws & 255) != 0) return fail(FX_EINVAL, "workspace must be 256-byte aligned");
    fx_stack *s = new (std::nothrow) fx_stack();
    if (!s) return fail(FX_ENOMEM, "host allocation failed");
    fx_status st = validate(desc, &s->plan);
    if (st) { delete s; return st; }
    s->d = *desc;
    s->mat.assign(desc->plane_mat, desc->plane_mat + desc->nz);
    s->eps_r.assign(desc->plane_eps_r, desc->plane_eps_r + desc->nz);
    s->Na.assign(desc->plane_Na, desc->plane_Na + desc->nz);
    s->Nd.assign(desc->plane_Nd, desc->plane_Nd + desc->nz);
    s->d.plane_mat = s->mat.data(); s->d.plane_eps_r = s->eps_r.data();
    s->d.plane_Na = s->Na.data(); s->d.plane_Nd = s->Nd.data();
    build_plan(&s->d, &s->plan);
    const size_t need = carve(s, nullptr);
    if (ws_bytes < need) { delete s; return fail(FX_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need); }
    carve(s, d_ws);
    s->st = (hipStream_t)stream;
    s->P[0] = d_P;
    s->phi = d_phi;
    s->pcur = 0;
    s->scale = desc->h * desc->h / kEps0;
    s->VT = kKb * desc->T / kQe;
    s->dmax = s->VT > 0 ? 40.0 * s->VT : 0.0;
    const Plan &p = s->plan;
    const int nzd = p.nzd;
    // finest-level tables: scaled coefficients, P face weights, carrier densities
    std::vector<double> wl(nzd, 1.0), wr(nzd, 0.0), p0e(nzd, 0.0), n0e(nzd, 0.0);
    std::vector<int> fl(nzd, 0);
    for (int k = 0; k < nzd; ++k) {
        const int K = p.kb + k;
        if (k + 1 < nzd) {
            const double eL = desc->plane_eps_r[K], eR = desc->plane_eps_r[K + 1];
            wl[k] = eR / (eL + eR);
            wr[k] = eL / (eL + eR);
        }
        const bool fe_near = desc->plane_mat[K] == FX_MAT_FE || (k > 0 && desc->plane_mat[K - 1] == FX_MAT_FE) ||
                             (k + 1 < nzd && desc->plane_mat[K + 1] == FX_MAT_FE);
        if (fe_near) fl[k] |= PF_P;
        if (desc->plane_mat[K] == FX_MAT_SC) {
            fl[k] |= PF_SC;
            const double net = desc->plane_Nd[K] - desc->plane_Na[K], ni = desc->ni;
            double pp, nn;
            if (net >= 0) { nn = 0.5 * net + std::sqrt(0.25 * net * net + ni * ni); pp = ni * ni / nn; }
            else { pp = -0.5 * net + std::sqrt(0.25 * net * net + ni * ni); nn = ni * ni / pp; }
            p0e[k] = kQe * pp;
            n0e[k] = kQe * nn;
        }
    }
    const HostLevel &H0 = p.lv[0];
#define UP(dst, v, T) HIP_OK(hipMemcpy(dst, (v).data(), nzd * sizeof(T), hipMemcpyHostToDevice))
    UP(s->t_cxy, H0.cxy, double); UP(s->t_czm, H0.czm, double); UP(s->t_czp, H0.czp, double);
    UP(s->t_wl, wl, double); UP(s->t_wr, wr, double); UP(s->t_p0e, p0e, double); UP(s->t_n0e, n0e, double);
    UP(s->t_flags, fl, int);
#undef UP
    for (size_t l = 0; l < p.lv.size(); ++l) {
        st = s->d.prec == FX_PREC_MIXED ? upload_level(p.lv[l], s->L32[l]) : upload_level(p.lv[l], s->L64[l]);
        if (st) { delete s; return st; }
    }
    if (hipHostMalloc((void **)&s->norms_host, 4 * sizeof(double), 0) != hipSuccess) {
        delete s;
        return fail(FX_EDEVICE, "hipHostMalloc failed");
    }
    // P: ping-pong buffer starts as a copy with zeros off the ferroelectric
    const size_t nfull = (size_t)p.nx * p.ny * p.nz, nxy = (size_t)p.nx * p.ny;
    launch_fill(s->P[1], nfull, 0.0, s->st);
    if (p.f0 >= 0) {
        if (p.f0 > 0) launch_fill(s->P[0], (size_t)p.f0 * nxy, 0.0, s->st);
        if (p.f1 < p.nz) launch_fill(s->P[0] + (size_t)p.f1 * nxy, (size_t)(p.nz - p.f1) * nxy, 0.0, s->st);
    } else {
        launch_fill(s->P[0], nfull, 0.0, s->st);
    }
    // Step 0: phi^{0,(0)} = 0, then solve
    launch_fill(s->phi, nfull, 0.0, s->st);
    set_contacts(s);
    *out = s;
    return solve(s, nullptr);
}

fx_status tdgl_step(fx_stack *s, double dt) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (!(dt > 0)) return fail(FX_EINVAL, "dt must be > 0");
    tdgl_impl(s, dt);
    return sync_P_to_caller(s);
}

fx_status poisson_solve(fx_stack *s, double v_top, fx_solve_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (!std::isfinite(v_top)) return fail(FX_EINVAL, "v_top must be finite");
    s->d.v_top = v_top;
    set_contacts(s);
    return solve(s, info);
}

fx_status run_steps(fx_stack *s, int nsteps, double dt, const double *h_v_top_sched, fx_run_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (nsteps < 0 || !(dt > 0)) return fail(FX_EINVAL, "nsteps >= 0 and dt > 0 required");
    fx_run_info ri{};
    fx_status st = FX_OK;
    for (int n = 0; n < nsteps; ++n) {
        tdgl_impl(s, dt);
        if (h_v_top_sched) { s->d.v_top = h_v_top_sched[n]; set_contacts(s); }
        fx_solve_info si{};
        st = solve(s, &si);
        ri.total_cycles += si.cycles;
        if (si.cycles > ri.max_cycles_step) ri.max_cycles_step = si.cycles;
        ri.last_res_rel = si.rhs_norm > 0 ? si.res_norm / si.rhs_norm : 0.0;
        if (st) break;
        ri.steps_done = n + 1;
    }
    fx_status st2 = sync_P_to_caller(s);
    if (info) *info = ri;
    return st ? st : st2;
}

fx_status get_field(fx_stack *s, int which, double *h_out) {
    g_err.clear();
    if (!s || !h_out) return fail(FX_EINVAL, "NULL argument");
    const size_t n = (size_t)s->plan.nx * s->plan.ny * s->plan.nz;
    const double *src = which == FX_FIELD_P ? s->P[s->pcur] : which == FX_FIELD_PHI ? s->phi : nullptr;
    if (!src) return fail(FX_EINVAL, "unknown field %d", which);
    HIP_OK(hipMemcpyAsync(h_out, src, n * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    return FX_OK;
}

fx_status set_field(fx_stack *s, int which, const double *h_in) {
    g_err.clear();
    if (!s || !h_in) return fail(FX_EINVAL, "NULL argument");
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny, n = nxy * p.nz;
    if (which == FX_FIELD_P) {
        fx_status sp = sync_P_to_caller(s);
        if (sp) return sp;
        HIP_OK(hipMemcpyAsync(s->P[0], h_in, n * sizeof(double), hipMemcpyHostToDevice, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        if (p.f0 >= 0) {
            if (p.f0 > 0) launch_fill(s->P[0], (size_t)p.f0 * nxy, 0.0, s->st);
            if (p.f1 < p.nz) launch_fill(s->P[0] + (size_t)p.f1 * nxy, (size_t)(p.nz - p.f1) * nxy, 0.0, s->st);
        } else {
            launch_fill(s->P[0], n, 0.0, s->st);
        }
    } else if (which == FX_FIELD_PHI) {
        HIP_OK(hipMemcpyAsync(s->phi, h_in, n * sizeof(double), hipMemcpyHostToDevice, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        set_contacts(s);
    } else {
        return fail(FX_EINVAL, "unknown field %d", which);
    }
    return FX_OK;
}

int stack_num_levels(const fx_stack *s) { return s ? (int)s->plan.lv.size() : 0; }

fx_status stack_level_shape(const fx_stack *s, int level, int *nx, int *ny, int *nz) {
    if (!s || level < 0 || level >= (int)s->plan.lv.size()) return fail(FX_EINVAL, "bad level");
    const HostLevel &H = s->plan.lv[level];
    if (nx) *nx = H.nx;
    if (ny) *ny = H.ny;
    if (nz) *nz = H.nz;
    return FX_OK;
}

fx_status destroy_stack(fx_stack *s) {
    if (!s) return FX_OK;
    if (s->st) (void)hipStreamSynchronize(s->st); else (void)hipDeviceSynchronize();
    if (s->norms_host) (void)hipHostFree(s->norms_host);
    delete s;
    return FX_OK;
}

const char *last_error(void) { return g_err.c_str(); }

}  // extern "C"
