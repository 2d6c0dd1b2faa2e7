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
#include "../../include/ferrox.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <type_traits>

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

constexpr int kBottomTarget = 8;         // stop coarsening at this many cells

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
};

template <typename T>
struct DevSet {
    std::vector<DevLevel<T>> lv;
    CoarseArgs<T> *coarse = nullptr;    // device copy of the coarse-kernel arguments
    int coarse_lds = 0;
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
    if (d->warm_start < 0 || d->warm_start > 3) return fail(FX_EINVAL, "warm_start must be 0..3");
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

}  // namespace


struct fx_stack {
    fx_stack_desc d{};
    std::vector<int> mat;
    std::vector<double> eps_r, Na, Nd;
    Plan plan;
    hipStream_t st = nullptr;
    // P: [0] the caller's array, [1] workspace; pcur holds P^n
    double *P[2] = {nullptr, nullptr};
    int pcur = 0;
    // phi: [0] the caller's array, [1..5] workspace; phicur holds phi^n and
    // prev[0..hist-1] hold phi^{n-1}, phi^{n-2}, phi^{n-3} of the previous time
    // steps.  A solve writes its iterates into two buffers that are none of
    // these, so the entry state survives a failed solve.
    static constexpr int kPhiBufs = 6, kMaxHist = 3;
    double *phi[kPhiBufs] = {};
    int phicur = 0;
    int prev[kMaxHist] = {1, 2, 3};
    int hist = 0;
    // finest-level FP64 tables
    double *t_cxy = nullptr, *t_czm = nullptr, *t_czp = nullptr, *t_wl = nullptr, *t_wr = nullptr;
    double *t_p0e = nullptr, *t_n0e = nullptr;
    int *t_flags = nullptr;
    DevSet<double> D64;
    DevSet<float> D32;
    double *part = nullptr;
    int part_n = 0;
    SolveCtrl *ctrl = nullptr;          // device
    SolveCtrl *ctrl_host = nullptr;     // pinned
    double VT = 0.0, scale = 0.0;
    double dmax = 0.0;
    int nu1 = 2, nu2 = 2, bottom_sweeps = 12;
    int k_pred = 4;                     // cycles enqueued before the first convergence check
    int trace = 0;
    // kernel-duration probe of the finest-level smoother
    int probe = 0;
    std::vector<hipEvent_t> ev;         // pairs (start, stop)
    int ev_used = 0;
    double probe_bytes = 0.0;
};

namespace {

// Lay out (or, with ws == nullptr, only size) the workspace.
size_t carve(fx_stack *s, void *ws) {
    Carver cv(ws);
    const Plan &p = s->plan;
    const size_t nfull = (size_t)p.nx * p.ny * p.nz;
    s->P[1] = (double *)cv.take(nfull * sizeof(double));
    for (int b = 1; b < fx_stack::kPhiBufs; ++b) s->phi[b] = (double *)cv.take(nfull * sizeof(double));
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
    s->D64.lv.assign(mixed ? 0 : nlev, DevLevel<double>());
    s->D32.lv.assign(mixed ? nlev : 0, DevLevel<float>());
    auto lay = [&](auto &D, const HostLevel &H, size_t w) {
        using TT = std::remove_pointer_t<decltype(D.e)>;
        const size_t n = H.ncell(), ns = H.nsig();
        const int nz = H.nz;
        D.e = (TT *)cv.take(n * w); D.r = (TT *)cv.take(n * w); D.sig = (TT *)cv.take(std::max<size_t>(ns, 1) * w);
        D.cxy = (TT *)cv.take(nz * w); D.czm = (TT *)cv.take(nz * w);
        D.czp = (TT *)cv.take(nz * w); D.dg = (TT *)cv.take(nz * w);
        D.pwa = (TT *)cv.take(nz * w); D.pwb = (TT *)cv.take(nz * w);
        D.ks = (int *)cv.take(nz * sizeof(int)); D.cnt = (int *)cv.take(nz * sizeof(int));
        D.thick = (int *)cv.take(nz * sizeof(int)); D.pka = (int *)cv.take(nz * sizeof(int));
        D.pkb = (int *)cv.take(nz * sizeof(int));
    };
    for (int l = 0; l < nlev; ++l) {
        if (mixed) lay(s->D32.lv[l], p.lv[l], 4);
        else lay(s->D64.lv[l], p.lv[l], 8);
    }
    if (mixed) s->D32.coarse = (CoarseArgs<float> *)cv.take(sizeof(CoarseArgs<float>));
    else s->D64.coarse = (CoarseArgs<double> *)cv.take(sizeof(CoarseArgs<double>));
    // residual partial sums: one pair per 64x4 tile of the finest level (an upper bound
    // for tiles spanning several planes)
    const size_t nb = (size_t)((p.nx + 63) / 64) * ((p.ny + 3) / 4) * nzd;
    s->part_n = (int)nb;
    s->part = (double *)cv.take(2 * nb * sizeof(double));
    s->ctrl = (SolveCtrl *)cv.take(sizeof(SolveCtrl));
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
LevelArgs<T> level_args(const fx_stack *s, const DevSet<T> &D, int l) {
    const HostLevel &H = s->plan.lv[l];
    LevelArgs<T> a;
    a.nx = H.nx; a.ny = H.ny; a.nz = H.nz; a.rb = H.rb;
    a.cxy = D.lv[l].cxy; a.czm = D.lv[l].czm; a.czp = D.lv[l].czp; a.dg = D.lv[l].dg;
    a.e = D.lv[l].e; a.r = D.lv[l].r; a.sig = D.lv[l].sig;
    a.sig_lo = H.sig_lo; a.sig_hi = H.sig_hi;
    return a;
}

// Transfer tables between level l (fine) and l+1 (coarse).
template <typename T>
XferArgs<T> xfer_args(const fx_stack *s, const DevSet<T> &D, int l) {
    XferArgs<T> x;
    x.cks = D.lv[l + 1].ks; x.ccnt = D.lv[l + 1].cnt;
    x.fthick = D.lv[l].thick; x.cthick = D.lv[l + 1].thick;
    x.pka = D.lv[l].pka; x.pkb = D.lv[l].pkb; x.pwa = D.lv[l].pwa; x.pwb = D.lv[l].pwb;
    x.xy = s->plan.lv[l + 1].xy_from_finer;
    return x;
}

template <typename T>
fx_status upload_coarse(fx_stack *s, DevSet<T> &D) {
    const Plan &p = s->plan;
    CoarseArgs<T> A;
    memset(&A, 0, sizeof A);
    A.nlev = (int)p.lv.size() - p.lc;
    A.nu1 = s->nu1; A.nu2 = s->nu2;
    const HostLevel &B = p.lv.back();
    A.bottom_sweeps = std::max(4, 2 * std::max(B.nx, std::max(B.ny, B.nz)));
    int off = 0;
    auto take = [&](size_t bytes) { const int o = off; off += (int)((bytes + 15) & ~(size_t)15); return o; };
    for (int q = 0; q < A.nlev; ++q) {
        const HostLevel &H = p.lv[p.lc + q];
        A.lv[q] = level_args(s, D, p.lc + q);
        A.off_e[q] = take(H.ncell() * sizeof(T));
        A.off_r[q] = take(H.ncell() * sizeof(T));
        A.off_s[q] = take(H.nsig() * sizeof(T));
        A.off_t[q] = take(4 * H.nz * sizeof(T));
        if (q + 1 < A.nlev) A.xf[q] = xfer_args(s, D, p.lc + q);
    }
    A.lds_bytes = off;
    A.r_in = D.lv[p.lc].r;
    A.sig_in = D.lv[p.lc].sig;
    A.e_out = D.lv[p.lc].e;
    if (off > kCoarseLdsBytes) return fail(FX_EINVAL, "coarse levels need %d bytes of LDS", off);
    D.coarse_lds = off;
    HIP_OK(hipMemcpy(D.coarse, &A, sizeof A, hipMemcpyHostToDevice));
    return FX_OK;
}

// Launch one smoother colour; finest-level launches are timestamped while
// the probe is on, and their algorithmic bytes accumulated (one touch of each
// array: the other colour's e, this colour's r, sigma and e; plus the phi
// pair read and write when the Newton update is folded in).
template <typename T>
void smooth(fx_stack *s, const LevelArgs<T> &A, int l, int color, int zi, const UpdArgs *upd = nullptr) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (l == 0 && s->probe && s->ev_used + 2 <= (int)s->ev.size()) {
        e0 = s->ev[s->ev_used];
        e1 = s->ev[s->ev_used + 1];
        s->ev_used += 2;
        const double n = (double)A.nx * A.ny * A.nz, ns = (double)A.nx * A.ny * (A.sig_hi - A.sig_lo);
        double b = sizeof(T) * (0.5 * n + 0.5 * ns + 0.5 * n);       // r, sigma, e of this colour
        if (!zi) b += sizeof(T) * 0.5 * n;                            // the other colour's e
        if (upd) b += 16.0 * n;                                       // phi read + write
        s->probe_bytes += b;
    }
    launch_smooth(A, color, zi, s->ctrl, s->st, upd, e0, e1);
}

// V-cycle from level l.  On the finest level (l = 0) with red/black storage
// the last black half-sweep also writes phi_out = phi_in + clip(e).
template <typename T>
void vcycle(fx_stack *s, const DevSet<T> &D, int l, const UpdArgs *upd = nullptr) {
    hipStream_t st = s->st;
    if (l == s->plan.lc) {
        launch_coarse(D.coarse, D.coarse_lds, s->ctrl, st);
        return;
    }
    const LevelArgs<T> A = level_args(s, D, l);
    const LevelArgs<T> C = level_args(s, D, l + 1);
    const XferArgs<T> X = xfer_args(s, D, l);
    const int ncol = A.rb ? 2 : 4;
    for (int q = 0; q < s->nu1; ++q)
        for (int c = 0; c < ncol; ++c) smooth(s, A, l, c, q == 0 && c == 0);
    launch_restrict(A, C, X, s->ctrl, st);
    vcycle(s, D, l + 1);
    launch_prolong(A, C, X, s->ctrl, st);
    for (int q = 0; q < s->nu2; ++q)
        for (int c = 0; c < ncol; ++c)
            smooth(s, A, l, c, 0, (upd && A.rb && q == s->nu2 - 1 && c == ncol - 1) ? upd : nullptr);
}

// Fine-level residual at phi_in (+ e when given, written to phi_out) and the
// stop decision.
// count_cycle: this residual closes a multigrid cycle (the device counts it).
template <typename T>
void residual(fx_stack *s, const DevSet<T> &D, const double *phi_in, double *phi_out, bool with_e,
              bool count_cycle) {
    const Plan &p = s->plan;
    ResArgs<T> a;
    a.nx = p.nx; a.ny = p.ny; a.nzd = p.nzd; a.kb = p.kb;
    a.v_b = s->d.v_bottom; a.v_t = s->d.v_top;
    a.p_scale = s->d.h / kEps0;
    a.rho_scale = s->scale;
    a.vt_inv = s->VT > 0 ? 1.0 / s->VT : 0.0;
    a.sig_scale = s->VT > 0 ? s->scale / s->VT : 0.0;
    a.dmax = s->dmax;
    a.cxy = s->t_cxy; a.czm = s->t_czm; a.czp = s->t_czp;
    a.wl = s->t_wl; a.wr = s->t_wr; a.p0e = s->t_p0e; a.n0e = s->t_n0e; a.pflags = s->t_flags;
    a.phi_in = phi_in;
    a.phi_out = phi_out;
    a.e = with_e ? D.lv[0].e : nullptr;
    a.P = s->P[s->pcur];
    a.L0 = level_args(s, D, 0);
    a.part = s->part;
    a.ctrl = s->ctrl;
    const int n = launch_residual(a, s->st);
    launch_reduce(s->part, n, s->ctrl, count_cycle ? 1 : 0, s->st);
}

fx_status read_ctrl(fx_stack *s) {
    HIP_OK(hipMemcpyAsync(s->ctrl_host, s->ctrl, sizeof(SolveCtrl), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    return FX_OK;
}

bool holds_history(const fx_stack *s, int b) {
    for (int m = 0; m < s->hist; ++m)
        if (s->prev[m] == b) return true;
    return false;
}

// Lagrange extrapolation to t^{n+1} through t^n, t^{n-1}, ... (equal steps).
const double kExtrap[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};

// Newton-multigrid solve.  The iterate before cycle 0 is phi^n, or (in the
// time loop, with previous levels held) their polynomial extrapolation
// written to buffer other[1].  Cycle c writes other[c % 2] from the previous
// iterate; kernels of cycles after the device has decided to stop return at
// once, so a batch of cycles is enqueued before each host check.
template <typename T>
fx_status solve_impl(fx_stack *s, const DevSet<T> &D, fx_solve_info *info, bool time_step) {
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny, off = (size_t)p.kb * nxy, nd = (size_t)p.nzd * nxy;
    const int entry = s->phicur;
    int other[2], no = 0;
    for (int b = 0; b < fx_stack::kPhiBufs && no < 2; ++b)
        if (b != entry && !holds_history(s, b)) other[no++] = b;
    const int order = time_step ? std::min(s->hist, std::max(0, std::min(s->d.warm_start, fx_stack::kMaxHist))) : 0;
    launch_ctrl_reset(s->ctrl, s->d.max_cycles, s->d.tol_rel * s->d.tol_rel, s->st);
    const int start = order > 0 ? other[1] : entry;   // buffer holding the iterate before cycle 0
    if (order > 0) {
        ExtrapArgs ea;
        ea.nin = order + 1;
        for (int q = 0; q <= order; ++q) {
            ea.c[q] = kExtrap[order][q];
            ea.in[q] = s->phi[q == 0 ? entry : s->prev[q - 1]] + off;
        }
        launch_extrap(s->phi[start] + off, ea, nd, s->st);
    }
    residual<T>(s, D, s->phi[start], nullptr, false, false);
    int enq = 0;                        // cycles enqueued so far
    int batch = s->trace ? 0 : std::max(1, s->k_pred);
    fx_status st;
    for (;;) {
        const bool fold = p.lv[0].rb && p.lc > 0;
        for (int q = 0; q < batch && enq < s->d.max_cycles; ++q, ++enq) {
            const double *src = s->phi[enq == 0 ? start : other[(enq - 1) % 2]];
            double *dst = s->phi[other[enq % 2]];
            if (fold) {
                const UpdArgs u{src + off, dst + off, s->t_flags, s->dmax};
                vcycle<T>(s, D, 0, &u);
                residual<T>(s, D, dst, nullptr, false, true);
            } else {
                vcycle<T>(s, D, 0);
                residual<T>(s, D, src, dst, true, true);
            }
        }
        if ((st = read_ctrl(s))) return st;
        const SolveCtrl &c = *s->ctrl_host;
        if (s->trace)
            fprintf(stderr, "[ferrox] cycle %d |r|/|f| = %.3e\n", c.cycles, c.fn2 > 0 ? std::sqrt(c.rn2 / c.fn2) : 0.0);
        if (c.done || enq >= s->d.max_cycles) break;
        batch = 1;
    }
    const SolveCtrl c = *s->ctrl_host;
    const int ncyc = c.cycles;
    const int final_buf = ncyc == 0 ? start : other[(ncyc - 1) % 2];
    double rn = std::sqrt(c.rn2), fn = std::sqrt(c.fn2);
    fx_status res = FX_OK;
    int newcur = final_buf;
    if (c.done == 2) {
        res = FX_ENONFINITE;
        newcur = entry;                 // the entry iterate is untouched
    } else if (c.done == 1 && fn == 0.0 && rn != 0.0) {
        // f = 0: N(0) = 0 exactly, so phi = 0 is the root
        launch_fill(s->phi[final_buf] + off, nd, 0.0, s->st);
        rn = 0.0;
    } else if (c.done != 1) {
        res = FX_ENOCONV;
    }
    // the entry iterate phi^n becomes the newest stored level
    if (time_step && res == FX_OK && newcur != entry) {
        for (int m = fx_stack::kMaxHist - 1; m > 0; --m) s->prev[m] = s->prev[m - 1];
        s->prev[0] = entry;
        s->hist = std::min(s->hist + 1, fx_stack::kMaxHist);
    } else {
        s->hist = 0;
    }
    s->phicur = newcur;
    if (res != FX_ENONFINITE) s->k_pred = std::max(1, ncyc);
    if (info) { info->cycles = ncyc; info->status = res; info->res_norm = rn; info->rhs_norm = fn; }
    if (res == FX_ENOCONV) return fail(res, "no convergence in %d cycles: |r|/|f| = %.3e", ncyc, rn / fn);
    if (res == FX_ENONFINITE) return fail(res, "non-finite residual");
    return FX_OK;
}

// A solve inside the time loop may start from the extrapolated iterate; the
// history is kept only across consecutive time steps.
fx_status solve(fx_stack *s, fx_solve_info *info, bool time_step = false) {
    return s->d.prec == FX_PREC_MIXED ? solve_impl<float>(s, s->D32, info, time_step)
                                      : solve_impl<double>(s, s->D64, info, time_step);
}

void set_contacts(fx_stack *s) {
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny;
    if (p.kb > 0) launch_fill(s->phi[0], (size_t)p.kb * nxy, s->d.v_bottom, s->st);
    if (p.kt < p.nz) launch_fill(s->phi[0] + (size_t)p.kt * nxy, (size_t)(p.nz - p.kt) * nxy, s->d.v_top, s->st);
}

void tdgl_impl(fx_stack *s, double dt) {
    const Plan &p = s->plan;
    if (p.f0 < 0) return;
    TdglArgs a;
    a.nx = p.nx; a.ny = p.ny; a.f0 = p.f0; a.f1 = p.f1;
    a.h = s->d.h; a.dt = dt;
    a.alpha = s->d.alpha; a.beta = s->d.beta; a.gamma = s->d.gamma;
    a.g11 = s->d.g11; a.g44 = s->d.g44; a.Gamma = s->d.Gamma;
    a.pbc = s->d.pbc; a.lambda = s->d.lambda;
    a.P = s->P[s->pcur]; a.phi = s->phi[s->phicur]; a.Pn = s->P[1 - s->pcur];
    launch_tdgl(a, s->st);
    s->pcur = 1 - s->pcur;
}

// Make the caller's arrays hold the current P and phi.
fx_status sync_to_caller(fx_stack *s) {
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny;
    if (s->pcur != 0) {
        if (p.f0 >= 0)
            HIP_OK(hipMemcpyAsync(s->P[0] + p.f0 * nxy, s->P[1] + p.f0 * nxy, (p.f1 - p.f0) * nxy * sizeof(double),
                                  hipMemcpyDeviceToDevice, s->st));
        s->pcur = 0;
    }
    if (s->phicur != 0) {
        // buffer 0 is the caller's: if it holds a stored level, move that level first
        for (int m = 0; m < s->hist; ++m) {
            if (s->prev[m] != 0) continue;
            int spare = 1;
            while (spare == s->phicur || holds_history(s, spare)) ++spare;
            HIP_OK(hipMemcpyAsync(s->phi[spare] + p.kb * nxy, s->phi[0] + p.kb * nxy,
                                  (size_t)p.nzd * nxy * sizeof(double), hipMemcpyDeviceToDevice, s->st));
            s->prev[m] = spare;
        }
        HIP_OK(hipMemcpyAsync(s->phi[0] + p.kb * nxy, s->phi[s->phicur] + p.kb * nxy,
                              (size_t)p.nzd * nxy * sizeof(double), hipMemcpyDeviceToDevice, s->st));
        s->phicur = 0;
    }
    return FX_OK;
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

}  // namespace

extern "C" {

size_t stack_workspace_bytes(const fx_stack_desc *desc) {
    g_err.clear();
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
    if (((uintptr_t)d_P & 15) != 0 || ((uintptr_t)d_phi & 15) != 0)
        return fail(FX_EINVAL, "d_P and d_phi must be 16-byte aligned");
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
    s->phi[0] = d_phi;
    s->scale = desc->h * desc->h / kEps0;
    s->VT = kKb * desc->T / kQe;
    s->dmax = s->VT > 0 ? 40.0 * s->VT : 0.0;
    s->nu1 = std::max(1, env_int("FERROX_NU1", 2));
    s->nu2 = std::max(1, env_int("FERROX_NU2", 2));
    s->trace = env_int("FERROX_TRACE", 0);
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
#define UP(dst, v, T)                                                                            \
    do {                                                                                         \
        hipError_t e_ = hipMemcpy(dst, (v).data(), nzd * sizeof(T), hipMemcpyHostToDevice);      \
        if (e_ != hipSuccess) { delete s; return fail(FX_EDEVICE, "table upload: %s", hipGetErrorString(e_)); } \
    } while (0)
    UP(s->t_cxy, H0.cxy, double); UP(s->t_czm, H0.czm, double); UP(s->t_czp, H0.czp, double);
    UP(s->t_wl, wl, double); UP(s->t_wr, wr, double); UP(s->t_p0e, p0e, double); UP(s->t_n0e, n0e, double);
    UP(s->t_flags, fl, int);
#undef UP
    for (size_t l = 0; l < p.lv.size(); ++l) {
        st = s->d.prec == FX_PREC_MIXED ? upload_level(p.lv[l], s->D32.lv[l]) : upload_level(p.lv[l], s->D64.lv[l]);
        if (st) { delete s; return st; }
    }
    st = s->d.prec == FX_PREC_MIXED ? upload_coarse(s, s->D32) : upload_coarse(s, s->D64);
    if (st) { delete s; return st; }
    if (hipHostMalloc((void **)&s->ctrl_host, sizeof(SolveCtrl), 0) != hipSuccess) {
        delete s;
        return fail(FX_EDEVICE, "hipHostMalloc failed");
    }
    // P: zero off the ferroelectric in both buffers
    const size_t nfull = (size_t)p.nx * p.ny * p.nz, nxy = (size_t)p.nx * p.ny;
    launch_fill(s->P[1], nfull, 0.0, s->st);
    if (p.f0 >= 0) {
        if (p.f0 > 0) launch_fill(s->P[0], (size_t)p.f0 * nxy, 0.0, s->st);
        if (p.f1 < p.nz) launch_fill(s->P[0] + (size_t)p.f1 * nxy, (size_t)(p.nz - p.f1) * nxy, 0.0, s->st);
    } else {
        launch_fill(s->P[0], nfull, 0.0, s->st);
    }
    // Step 0: phi^{0,(0)} = 0, then solve
    for (int b = 0; b < fx_stack::kPhiBufs; ++b) launch_fill(s->phi[b], nfull, 0.0, s->st);
    set_contacts(s);
    *out = s;
    st = solve(s, nullptr);
    fx_status st2 = sync_to_caller(s);
    return st ? st : st2;
}

fx_status tdgl_step(fx_stack *s, double dt) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (!(dt > 0)) return fail(FX_EINVAL, "dt must be > 0");
    tdgl_impl(s, dt);
    s->hist = 0;
    return sync_to_caller(s);
}

fx_status poisson_solve(fx_stack *s, double v_top, fx_solve_info *info) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (!std::isfinite(v_top)) return fail(FX_EINVAL, "v_top must be finite");
    s->d.v_top = v_top;
    set_contacts(s);
    fx_status st = solve(s, info);
    std::string msg = g_err;
    fx_status st2 = sync_to_caller(s);
    g_err = msg;
    return st ? st : st2;
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
        st = solve(s, &si, true);
        ri.total_cycles += si.cycles;
        if (si.cycles > ri.max_cycles_step) ri.max_cycles_step = si.cycles;
        ri.last_res_rel = si.rhs_norm > 0 ? si.res_norm / si.rhs_norm : 0.0;
        if (st) break;
        ri.steps_done = n + 1;
    }
    std::string msg = g_err;
    fx_status st2 = sync_to_caller(s);
    g_err = msg;
    if (info) *info = ri;
    return st ? st : st2;
}

fx_status get_field(fx_stack *s, int which, double *h_out) {
    g_err.clear();
    if (!s || !h_out) return fail(FX_EINVAL, "NULL argument");
    if (which < FX_FIELD_P || which > FX_FIELD_PHI_PREV3) return fail(FX_EINVAL, "unknown field %d", which);
    fx_status st = sync_to_caller(s);
    if (st) return st;
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny, n = nxy * p.nz;
    if (which >= FX_FIELD_PHI_PREV) {
        const int m = which - FX_FIELD_PHI_PREV;
        if (m >= s->hist) return fail(FX_ESTATE, "time level n-%d is not held", m + 1);
        // device planes from the history buffer, contacts from the caller's array
        HIP_OK(hipMemcpyAsync(h_out, s->phi[0], n * sizeof(double), hipMemcpyDeviceToHost, s->st));
        HIP_OK(hipMemcpyAsync(h_out + p.kb * nxy, s->phi[s->prev[m]] + p.kb * nxy, (size_t)p.nzd * nxy * sizeof(double),
                              hipMemcpyDeviceToHost, s->st));
    } else {
        HIP_OK(hipMemcpyAsync(h_out, which == FX_FIELD_P ? s->P[0] : s->phi[0], n * sizeof(double),
                              hipMemcpyDeviceToHost, s->st));
    }
    HIP_OK(hipStreamSynchronize(s->st));
    return FX_OK;
}

fx_status set_field(fx_stack *s, int which, const double *h_in) {
    g_err.clear();
    if (!s || !h_in) return fail(FX_EINVAL, "NULL argument");
    if (which < FX_FIELD_P || which > FX_FIELD_PHI_PREV3) return fail(FX_EINVAL, "unknown field %d", which);
    fx_status st = sync_to_caller(s);
    if (st) return st;
    const Plan &p = s->plan;
    const size_t nxy = (size_t)p.nx * p.ny, n = nxy * p.nz;
    if (which >= FX_FIELD_PHI_PREV) {
        const int m = which - FX_FIELD_PHI_PREV;
        if (m != s->hist) return fail(FX_ESTATE, "set time level n-%d after n-1 .. n-%d", m + 1, m);
        int b = 1;                      // phicur is 0 after sync_to_caller
        while (holds_history(s, b)) ++b;
        HIP_OK(hipMemcpyAsync(s->phi[b] + p.kb * nxy, h_in + p.kb * nxy, (size_t)p.nzd * nxy * sizeof(double),
                              hipMemcpyHostToDevice, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        s->prev[m] = b;
        s->hist = m + 1;
        return FX_OK;
    }
    s->hist = 0;
    if (which == FX_FIELD_P) {
        HIP_OK(hipMemcpyAsync(s->P[0], h_in, n * sizeof(double), hipMemcpyHostToDevice, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        if (p.f0 >= 0) {
            if (p.f0 > 0) launch_fill(s->P[0], (size_t)p.f0 * nxy, 0.0, s->st);
            if (p.f1 < p.nz) launch_fill(s->P[0] + (size_t)p.f1 * nxy, (size_t)(p.nz - p.f1) * nxy, 0.0, s->st);
        } else {
            launch_fill(s->P[0], n, 0.0, s->st);
        }
    } else {
        HIP_OK(hipMemcpyAsync(s->phi[0], h_in, n * sizeof(double), hipMemcpyHostToDevice, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        set_contacts(s);
    }
    return FX_OK;
}

fx_status stack_probe(fx_stack *s, int kernel, int max_launches) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    if (kernel != FX_PROBE_OFF && kernel != FX_PROBE_SMOOTH_FINE) return fail(FX_EINVAL, "unknown probe %d", kernel);
    if (kernel == FX_PROBE_OFF) { s->probe = 0; return FX_OK; }
    if (max_launches < 1) return fail(FX_EINVAL, "max_launches must be >= 1");
    HIP_OK(hipStreamSynchronize(s->st));
    while ((int)s->ev.size() < 2 * max_launches) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        s->ev.push_back(e);
    }
    s->probe = kernel;
    s->ev_used = 0;
    s->probe_bytes = 0.0;
    return FX_OK;
}

fx_status stack_probe_read(fx_stack *s, double *total_ms, int *launches, double *bytes) {
    g_err.clear();
    if (!s) return fail(FX_EINVAL, "stack is NULL");
    HIP_OK(hipStreamSynchronize(s->st));
    double tot = 0.0;
    for (int q = 0; q + 1 < s->ev_used; q += 2) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, s->ev[q], s->ev[q + 1]));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = s->ev_used / 2;
    if (bytes) *bytes = s->probe_bytes;
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
    if (s->ctrl_host) (void)hipHostFree(s->ctrl_host);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    delete s;
    return FX_OK;
}

const char *last_error(void) { return g_err.c_str(); }

}  // extern "C"
