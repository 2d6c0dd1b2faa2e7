/*
 * ferrox.h -- C ABI of the MI355X TDGL + Poisson time-step library.
 *
 * The library advances the coupled ferroelectric phase-field model of
 * FerroX (arXiv 2210.15668, Methods): the polarisation P (z-component
 * only, as in the Results overview) by the time-dependent Ginzburg-Landau
 * equation, eq. (TDGL2), and the electric potential phi by the Poisson
 * equation with spatially varying permittivity, eq. (Poisson), whose
 * semiconductor charge is eq. (rho) with the Maxwell-Boltzmann carriers of
 * eq. (MaxBolt_ne_np).  The time scheme is the paper's Step 0 / Step 1a /
 * Step 1b (Numerical Approach): P^{n+1} = P^n + dt f(P^n, phi^n), then
 * phi^{n+1} solved for P^{n+1} starting from phi^n.
 *
 * Conventions shared by every entry point
 *  - SI units.  Grid of nx*ny*nz cubic cells of edge h; cell (i,j,k) lives at
 *    index (k*ny + j)*nx + i (z-major, x fastest); k = 0 is the back contact,
 *    k = nz-1 the gate.  Periodic in x and y; Dirichlet in z (section
 *    "Electrical boundary conditions").
 *  - Each z-plane carries one material (fx_material).  Metal planes must form
 *    contiguous runs at the two z-ends; the planes between them are the
 *    device, whose bottom face is held at v_bottom and top face at v_top
 *    (V_app = v_top - v_bottom).  The ferroelectric must be one contiguous run
 *    of at least 3 planes.
 *  - Device pointers ("d_") are HIP device addresses on the current device;
 *    host pointers ("h_") are ordinary process memory.  All work is enqueued
 *    on the stream given to init_stack (a hipStream_t passed as void*;
 *    NULL = the null stream).  Calls return after enqueueing, except where a
 *    host-visible result is needed: init_stack, poisson_solve and run_steps
 *    (and their batch forms) synchronise the stream.  Convergence is decided
 *    on the device; the host reads the solver state back after a few
 *    predicted cycles of a single solve, and every few time steps of a run,
 *    only to learn whether the work it enqueued has finished.
 *  - Errors are reported by fx_status; no exception crosses the ABI.
 *    last_error() returns a message for the most recent failure on the
 *    calling thread.  A stack is not thread-safe: use it from one thread.
 *  - The library allocates no device memory: the caller passes the fields
 *    and one workspace buffer (poisson_solve_static uses the library's own
 *    static device array instead).  init_stack allocates a small pinned host
 *    buffer for reading the solver state back, and host-side tables.
 *  - Batches (init_batch ...) hold many independent stacks of different
 *    sizes that advance together: each launch covers the tiles of all
 *    instances, and every instance stops its own solves.
 */
#ifndef FERROX_H
#define FERROX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FX_OK = 0,
    FX_EINVAL = 1,      /* invalid descriptor or argument                               */
    FX_ENOMEM = 2,      /* workspace too small, or host allocation failed               */
    FX_EDEVICE = 3,     /* a HIP runtime call failed                                    */
    FX_ENOCONV = 4,     /* max_cycles reached before ||r|| <= tol_rel ||f||              */
    FX_ENONFINITE = 5,  /* residual became NaN/Inf                                      */
    FX_ESTATE = 6       /* call not valid in the stack's current state                  */
} fx_status;

typedef enum { FX_MAT_METAL = 0, FX_MAT_FE = 1, FX_MAT_DE = 2, FX_MAT_SC = 3 } fx_material;

/* Carrier statistics of semiconductor planes (eq. rho).  Both measure phi
 * from the neutral bulk of the plane's doping (phi = 0 carries no charge).
 *  BOLTZMANN: eq. (MaxBolt_ne_np) with the intrinsic density ni:
 *      n = n0 e^(phi/VT), p = p0 e^(-phi/VT), p0 n0 = ni^2.
 *  FD: eqs. (FD), (density_state), (ne), (np): n = Nc F(eta_n0 + phi/VT),
 *      p = Nv F(eta_p0 - phi/VT), Nc = 2 (m_e kT/(2 pi hbar^2))^(3/2) (Nv with
 *      m_p), eta_n0 + eta_p0 = -Eg/kT and eta_n0 fixed by neutrality at
 *      phi = 0; F is the Fermi-Dirac integral of order 1/2 (normalised to
 *      e^eta for eta -> -inf) in the closed-form approximation of Bednarczyk
 *      and Bednarczyk (1978), as in the paper's Methods (Poisson solve); ni
 *      is not used. */
typedef enum { FX_CARRIERS_BOLTZMANN = 0, FX_CARRIERS_FD = 1 } fx_carriers;

/* Polarisation surface condition at both ferroelectric faces, eqs. (Pbc),
 * (PbcFree), (PbcDir): lambda dP/dn + P = 0 with outward normal n. */
typedef enum { FX_PBC_FREE = 0, FX_PBC_ZERO = 1, FX_PBC_LAMBDA = 2 } fx_pbc;

/* FP64: every multigrid level in double.  MIXED: the multigrid correction
 * (smoothing, restriction, prolongation, coarse levels) in float inside a
 * double-precision defect-correction loop (residual, carriers, update). */
typedef enum { FX_PREC_FP64 = 0, FX_PREC_MIXED = 1 } fx_precision;

/* FX_FIELD_PHI_PREV + m - 1 (m = 1..3) is phi at time level n - m, kept by
 * run_steps for the extrapolated starting iterate (warm_start); these are
 * part of the state a bitwise-exact checkpoint must carry. */
enum { FX_FIELD_P = 0, FX_FIELD_PHI = 1, FX_FIELD_PHI_PREV = 2, FX_FIELD_PHI_PREV2 = 3, FX_FIELD_PHI_PREV3 = 4 };

typedef struct fx_stack fx_stack;
typedef struct fx_batch fx_batch;

/* Problem statement (Table 1 and Methods of the paper).  Host arrays are
 * read during init_stack only. */
typedef struct {
    int nx, ny, nz;              /* cells                                                   */
    double h;                    /* cell edge [m]                                           */
    const int *plane_mat;        /* nz fx_material codes, k = 0 bottom                      */
    const double *plane_eps_r;   /* nz relative permittivities                              */
    const double *plane_Na;      /* nz acceptor densities [m^-3] (semiconductor planes)     */
    const double *plane_Nd;      /* nz donor densities [m^-3] (semiconductor planes)        */
    double alpha, beta, gamma;   /* Landau f = alpha/2 P^2 + beta/4 P^4 + gamma/6 P^6, eq. (free) */
    double g11, g44;             /* gradient coefficients (z; x and y), eq. (grad)         */
    double Gamma;                /* kinetic coefficient, eq. (TDGL1)                        */
    int pbc;                     /* fx_pbc                                                  */
    double lambda;               /* extrapolation length [m] for FX_PBC_LAMBDA              */
    double ni, T;                /* intrinsic density [m^-3], temperature [K]               */
    double v_bottom, v_top;      /* contact potentials [V]                                  */
    double tol_rel;              /* stop when ||f - N(phi)||_2 <= tol_rel ||f||_2           */
    int max_cycles;              /* multigrid cycles allowed per Poisson solve              */
    int prec;                    /* fx_precision                                            */
    int warm_start;              /* starting iterate of each run_steps solve: the polynomial
                                    extrapolation in time through phi^n and the previous
                                    warm_start levels (0: phi^n itself, as in Step 1b;
                                    1: 2 phi^n - phi^{n-1}; 2: quadratic; 3: cubic)      */
    int time_order;              /* run_steps' time scheme (Numerical Approach): 0 or 1 the
                                    forward-Euler Steps 1a + 1b; 2 the predictor-corrector
                                    Steps 1a, 1b, 2a, 2b (two solves per step; each
                                    predictor solve starts from the extrapolation plus the
                                    last step's phi* - phi^n, each corrector solve from the
                                    extrapolation through phi^n .. phi^{n-3}; this takes two
                                    more full grids of workspace, phi* and phi^{n-3}, which,
                                    unlike the levels n-1 .. n-3, are not part of a field
                                    checkpoint: a restarted run reaches the same roots, not
                                    the same bits)                                        */
    int carriers;                /* fx_carriers: semiconductor carrier statistics           */
    double m_e, m_p;             /* effective masses / free-electron mass (FX_CARRIERS_FD;
                                    Table 1: 1.08 and 0.81)                                 */
    double Eg;                   /* band gap [eV] (FX_CARRIERS_FD)                          */
} fx_stack_desc;

typedef struct {
    int cycles;                  /* V-cycles (= Newton updates) used                        */
    int status;                  /* fx_status of the solve                                  */
    double res_norm;             /* final ||f - N(phi)||_2 (scaled by h^2/eps0)             */
    double rhs_norm;             /* ||f||_2 (same scaling)                                  */
} fx_solve_info;

typedef struct {
    int steps_done;
    int total_cycles;            /* V-cycles summed over the steps                           */
    int max_cycles_step;         /* largest per-step cycle count                             */
    double last_res_rel;         /* final relative residual of the last step                 */
} fx_run_info;

/* Bytes of device workspace init_stack needs for this descriptor (0 if invalid). */
size_t stack_workspace_bytes(const fx_stack_desc *desc);

/*
 * Validate desc, lay out the multigrid hierarchy in d_ws, upload the
 * per-plane tables, and run Step 0: phi := 0 on the device, then solve the
 * Poisson problem for the P held in d_P (Numerical Approach, Step 0).
 *   d_P, d_phi : caller-owned device arrays of nx*ny*nz doubles, 16-byte
 *                aligned.  d_P holds
 *                P^0 (read; entries off ferroelectric planes are ignored and
 *                treated as zero).  d_phi receives phi^0; metal planes hold
 *                their contact potential.  Both must outlive the stack, and
 *                after every call below they hold the stack's current P and
 *                phi.
 *   d_ws       : caller-owned device buffer of at least
 *                stack_workspace_bytes(desc) bytes, 256-byte aligned.
 *   stream     : hipStream_t (as void*) all work is enqueued on.
 *   out        : receives the stack handle (host object owned by the library,
 *                released by destroy_stack).
 * Returns FX_EINVAL for an invalid descriptor (sizes < 1, h/Gamma/T <= 0,
 * gamma <= 0, lambda < 0, metal planes not at the ends, ferroelectric not one
 * run of >= 3 planes), FX_ENOMEM if ws_bytes is too small, FX_ENOCONV /
 * FX_ENONFINITE if Step 0 fails (the stack is still created and returned).
 */
fx_status init_stack(const fx_stack_desc *desc, double *d_P, double *d_phi, void *d_ws,
                     size_t ws_bytes, void *stream, fx_stack **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the Step 0
 * of init_stack -- phi := 0, then the Poisson solve for the P in d_P at
 * desc->v_top to desc->tol_rel -- with no caller workspace and no stack
 * handle.  Its workspace is a static device array of the library, 64 MiB on
 * each GPU it runs on (allocated with the library's code, held until the
 * process ends); no hipMalloc, hipHostMalloc, stream, event or graph is
 * created, and host-side planning uses ordinary heap memory only.
 *   d_P, d_phi : as for init_stack (d_P's entries off ferroelectric planes
 *                are set to zero; d_phi receives phi, metal planes their
 *                contact potential).
 *   stream     : hipStream_t (as void*); the call synchronises it.
 *   info       : NULL or receives the solve's cycles, status and norms.
 * Same kernels and launch sequence as init_stack's Step 0, so phi is the
 * same bit for bit.  Returns FX_EINVAL as init_stack, FX_ENOMEM if
 * stack_workspace_bytes(desc) exceeds 64 MiB (the 128 x 128 x 64 MFIM stack
 * fits), FX_ENOCONV / FX_ENONFINITE as poisson_solve.  Every call on one GPU
 * uses that GPU's one array, and the call initialises all of it that it reads:
 * calls that overlap on one GPU (from several threads or streams) race.
 */
fx_status poisson_solve_static(const fx_stack_desc *desc, double *d_P, double *d_phi, void *stream,
                               fx_solve_info *info);

/*
 * Step 1a of the time scheme: P <- P + dt f(P, phi) with eq. (TDGL2), the
 * current phi held fixed.  phi is not touched.  FX_EINVAL if dt <= 0.
 */
fx_status tdgl_step(fx_stack *s, double dt);

/*
 * Solve the Poisson problem, eq. (Poisson) with eq. (rho), for the current P
 * with gate potential v_top, starting from the current phi (Step 1b warm
 * start).  Stops when ||f - N(phi)||_2 <= tol_rel ||f||_2, f the
 * right-hand side of the discrete system.  info may be NULL.
 * FX_ENOCONV: max_cycles reached, phi holds the last iterate.
 * FX_ENONFINITE: the residual is not finite; phi is restored to its value
 * at entry.
 */
fx_status poisson_solve(fx_stack *s, double v_top, fx_solve_info *info);

/*
 * nsteps steps of Step 1a + Step 1b.  h_v_top_sched: host array of nsteps
 * gate potentials, entry n used for the solve that produces phi^{n+1}; NULL
 * keeps the current v_top.  Stops at the first failing solve and returns its
 * status (info->steps_done counts completed steps).  info may be NULL.
 */
fx_status run_steps(fx_stack *s, int nsteps, double dt, const double *h_v_top_sched,
                    fx_run_info *info);

/*
 * Q-V characteristics (Results, MFIM: the interface charge density Q and the
 * average ferroelectric voltage V_fe^avg of the Q-V_fe and Q-V_app curves).
 * z_int is the face between the ferroelectric and a dielectric plane next to
 * it: below the ferroelectric if that plane is dielectric, else above it.
 * With L the plane below and R the plane above that face, D is the face flux
 * of the Poisson operator, D = -eps0 eps_f (phi_R - phi_L)/h + P_f
 * (eps_f = 2 eps_L eps_R/(eps_L + eps_R), P_f = (eps_R P_L + eps_L P_R)/
 * (eps_L + eps_R)), which in the dielectric half cell is eps0 eps_DE E_z;
 * phi_int is the face value of that half-cell profile.  Then
 *     Q    = -(lateral mean of D)          [C/m^2]
 *     V_fe = v_top - (lateral mean of phi_int)   [V]
 * (z points to the gate, so Q > 0 for a positive gate over a series
 * capacitor, the first quadrant of the paper's Q-V_app loops).
 * stack_qv: of the current state (synchronises the stream).  run_steps_qv:
 * run_steps that also writes Q and V_fe after every completed step n into
 * h_Q[n], h_V_fe[n] (host arrays of nsteps doubles; entries of steps not
 * completed are left as they were); the values are reduced on the device
 * inside the run, two small kernels per step, in a fixed order (repeatable
 * bit for bit).  Both return FX_EINVAL if the ferroelectric has no
 * dielectric neighbour.
 */
fx_status stack_qv(fx_stack *s, double *h_Q, double *h_V_fe);
fx_status run_steps_qv(fx_stack *s, int nsteps, double dt, const double *h_v_top_sched, double *h_Q,
                       double *h_V_fe, fx_run_info *info);

/* Copy the current P, phi or a previous time level of phi (FX_FIELD_*) to /
 * from host memory of nx*ny*nz doubles.  get_field synchronises the stream.
 * set_field of P zeroes entries off ferroelectric planes; set_field of phi
 * rewrites the metal planes with their contact potentials.  Setting P or phi
 * discards the stored time levels (the next run_steps step starts from
 * phi^n); setting FX_FIELD_PHI_PREV, then _PREV2, then _PREV3 afterwards
 * restores them in that order.  get_field of a level that is not held
 * returns FX_ESTATE. */
fx_status get_field(fx_stack *s, int which, double *h_out);
fx_status set_field(fx_stack *s, int which, const double *h_in);

/* Kernel-duration probe (instrumentation for roofline measurement).
 * While FX_PROBE_SMOOTH_FINE is on, every stride-th launch of the
 * finest-level Gauss-Seidel half-sweep (the kernel that moves the most bytes
 * per step) is timestamped by its own dispatch (hipExtLaunchKernelGGL
 * start/stop events, no extra stream work), up to max_launches (<= 4096)
 * timed launches, and the kernel itself adds up the algorithmic bytes of the
 * instances it worked on: one touch each of the other colour's correction,
 * this colour's right-hand side, sigma and correction (FP64: 8 bytes, mixed:
 * 4 bytes per value), plus 16 bytes per cell for the phi pair read and
 * written when the Newton update is folded into the last half-sweep.
 * Launches in which every solve had already stopped do no work and are not
 * counted.  stack_probe resets the counters (and synchronises the stream);
 * stack_probe_read synchronises and returns the summed duration in ms, the
 * number of counted launches and their bytes.  Runs use kernel-by-kernel
 * launches while the probe is on. */
enum { FX_PROBE_OFF = 0, FX_PROBE_SMOOTH_FINE = 1 };
fx_status stack_probe(fx_stack *s, int kernel, int max_launches, int stride);
fx_status stack_probe_read(fx_stack *s, double *total_ms, int *launches, double *bytes);

/* How run_steps / run_batch enqueue their work.  STREAM: kernel by kernel.
 * GRAPH: the repeating unit of a run (one multigrid cycle for every running
 * solve, then the finalization of stopped solves and the start of the next
 * time step where due) is captured once as a HIP graph (1, 2, 4, 8 and 16
 * units) on a private stream and replayed on the caller's stream.  Results
 * are identical.  Defaults: STREAM for stacks, GRAPH for batches (the
 * environment variable FERROX_LAUNCH=0/1 overrides the default).  While a
 * probe is on, runs use STREAM. */
enum { FX_LAUNCH_STREAM = 0, FX_LAUNCH_GRAPH = 1 };
fx_status stack_set_launch(fx_stack *s, int mode);

/* Autotuner.  For every multigrid level with its own smoother launches,
 * times the candidate launch shapes of the Gauss-Seidel half-sweep on the
 * stack's own level arrays -- tiles of 32x8, 64x4 or 128x2 threads, 1, 2, 4
 * or 8 planes per thread (z-march length), and the compiler's register
 * budget or one that keeps 8 waves per SIMD resident -- and keeps the
 * fastest.  Only the division of the work changes, so results are bitwise
 * identical with any choice.  cache_path (NULL: none) names a text file of
 * earlier choices keyed by GPU architecture, precision and the shapes of the
 * level's instances: a level found there is not timed again unless
 * FX_TUNE_FORCE is set; new choices are appended.  Synchronises the stream;
 * call between runs (not while a probe is on).  info may be NULL. */
typedef struct {
    int levels;                  /* levels with their own smoother launches                  */
    int from_cache;              /* of those, shapes taken from the cache file               */
    int configs_timed;           /* candidate shapes timed                                   */
    int cache_written;           /* 1 if new lines were appended to the cache file           */
    double default_us;           /* one half-sweep per searched level, default shapes, summed */
    double tuned_us;             /* the same with the chosen shapes                           */
} fx_tune_info;
enum { FX_TUNE_FORCE = 1 };
fx_status stack_autotune(fx_stack *s, const char *cache_path, int flags, fx_tune_info *info);
/* The shape in use at level l: tile width in threads, planes per thread,
 * 8-wave register budget (0/1). */
fx_status stack_tune_config(const fx_stack *s, int level, int *tile_x, int *zt, int *waves8);

/* Number of multigrid levels and the sizes of level l (for diagnostics). */
int stack_num_levels(const fx_stack *s);
fx_status stack_level_shape(const fx_stack *s, int level, int *nx, int *ny, int *nz);

/* How level l is smoothed (for diagnostics; the arithmetic, and so the result, is the
 * same in every mode): FX_LEVEL_LAUNCHES, a launch per half-sweep and per transfer
 * (some pairs fused); FX_LEVEL_BLOCKED, the pre-smoothing sweeps with the restriction
 * and the prolongation with the post-smoothing sweeps each one launch, over LDS tiles
 * that recompute a ring of neighbour cells; FX_LEVEL_COARSE, inside the one-workgroup
 * coarse kernel.  FX_EINVAL for a bad handle or level. */
enum { FX_LEVEL_LAUNCHES = 0, FX_LEVEL_BLOCKED = 1, FX_LEVEL_COARSE = 2 };
fx_status stack_level_mode(const fx_stack *s, int level, int *mode);

/* Release the stack handle (not the caller's device buffers). */
fx_status destroy_stack(fx_stack *s);

/* ---------------------------------------------------------------- batches
 * n independent stacks (1 <= n <= 4096) of any sizes, one precision.  Each
 * instance behaves as a stack of its own would: same Step 0, same time
 * steps, same results; the instances only share launches.  Workspace:
 * batch_workspace_bytes(descs, n), 256-byte aligned; d_P[i], d_phi[i] are
 * caller-owned device arrays of instance i's nx*ny*nz doubles (16-byte
 * aligned), holding P^0 on entry and the current P and phi after every call,
 * as for init_stack.  init_batch returns the first failing instance's
 * FX_ENOCONV / FX_ENONFINITE if a Step 0 solve fails (the batch is still
 * created). */
typedef struct {
    int status;                  /* fx_status of the instance's last solve in this call     */
    int steps_done;
    int total_cycles;
    int max_cycles_step;
    double last_res_rel;
} fx_batch_info;

size_t batch_workspace_bytes(const fx_stack_desc *descs, int n);
fx_status init_batch(const fx_stack_desc *descs, int n, double *const *d_P, double *const *d_phi, void *d_ws,
                     size_t ws_bytes, void *stream, fx_batch **out);

/* nsteps time steps of every instance.  h_v_top_sched: NULL, or n host
 * arrays of nsteps gate potentials (entry m for the solve producing
 * phi^{n+m+1}).  An instance whose solve fails stops there (its
 * info[i].status says why) while the others go on; the call returns FX_OK
 * when every instance completed, else the status of the first failed one.
 * info: NULL or n entries. */
fx_status run_batch(fx_batch *b, int nsteps, double dt, const double *const *h_v_top_sched,
                    fx_batch_info *info);

/* Q and V_fe as stack_qv / run_steps_qv, per instance: batch_qv fills n
 * entries (NaN for an instance whose ferroelectric has no dielectric
 * neighbour); run_batch_qv records into n host arrays h_Q[i], h_V_fe[i] of
 * nsteps doubles (left as they were for such instances). */
fx_status batch_qv(fx_batch *b, double *h_Q, double *h_V_fe);
fx_status run_batch_qv(fx_batch *b, int nsteps, double dt, const double *const *h_v_top_sched,
                       double *const *h_Q, double *const *h_V_fe, fx_batch_info *info);

/* Copy instance inst's current P, phi or stored level (FX_FIELD_*) to host
 * memory, as get_field. */
fx_status batch_get_field(fx_batch *b, int inst, int which, double *h_out);
fx_status batch_set_launch(fx_batch *b, int mode);
/* How level l is smoothed for the batch's instances that have launches of their own on it
 * (stack_level_mode's FX_LEVEL_*; FX_LEVEL_COARSE once every instance holds it in the
 * coarse kernel).  FX_EINVAL for a bad handle or a negative level. */
fx_status batch_level_mode(const fx_batch *b, int level, int *mode);
fx_status batch_autotune(fx_batch *b, const char *cache_path, int flags, fx_tune_info *info);
fx_status destroy_batch(fx_batch *b);

/* Message of the most recent failing call on this thread ("" if none). */
const char *last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FERROX_H */
