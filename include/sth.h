/*
 * sth.h -- C-ABI of the MI355X (gfx950) library libsth.so: the hybrid
 * micro-macro fine propagator, the drift-diffusion coarse propagator and the
 * multiscale parareal iteration of T. Laidin, "A space-time hybrid parareal
 * method for kinetic equations in the diffusive scaling" (arXiv:2511.13386).
 *
 * Model (1D1V): eps(x) d_t f + v d_x f + E d_v f = (rho M - f)/eps on the torus
 * [0, Lx) x [-vstar, vstar], with f = rho M + eps g (g is the scaled
 * perturbation), Gauss law E_{i+1/2} - E_{i-1/2} = (rho_i - rhobar) dx.
 * The 1D3V problem of the paper (velocity in [-vstar, vstar]^3, field along
 * x) is available for states g(x, vx) M(vy) M(vz) (sth_problem_desc.nv_y,
 * nv_z).
 *
 * Entry points: problem set-up (sth_footprint_bytes, sth_create,
 * sth_destroy), the coarse guess (sth_coarse_sweep[_batched]), the fine
 * propagator over all unconverged slices of a batch (sth_fine_sweep_batched,
 * or in chunks of steps: sth_fine_sweep_chunk), the parareal correction
 * (sth_parareal_correct[_batched]), whole solves recorded as HIP graphs
 * (sth_graph_*), per-class launch configuration (sth_*_fine_config*),
 * diagnostics and results (sth_moments_criteria, sth_get_rho, sth_get_g,
 * sth_get_errors, sth_get_info, sth_fine_run[_masks]).
 * rho lives at cell centres x_i = (i+1/2) dx, g at interfaces x_p = (p+1) dx
 * (interface p separates cells p and p+1; it is "i+1/2" for i = p).
 *
 * Conventions for every entry point:
 *  - Return value: 0 on success, a negative STH_E* code on failure; the
 *    message of the last failure on the calling thread is sth_last_error().
 *  - Host arrays are float64, C order; phase-space arrays are x-major,
 *    g[p*nv + j].  Host pointers are only read during the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously on it unless the entry point says it
 *    synchronises.  Problems are independent; results do not depend on which
 *    other problems share a batched call.
 *  - The library owns all device state of a problem.  It is carved from a
 *    caller-provided device arena (e.g. memory allocated by PyTorch) when one
 *    is given, else allocated with hipMalloc and freed by sth_destroy.
 */
#ifndef STH_H
#define STH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STH_OK          0
#define STH_EINVAL     -1  /* invalid argument or unsupported size            */
#define STH_ENOMEM     -2  /* arena too small or device allocation failed     */
#define STH_EHIP       -3  /* a HIP runtime call failed                       */
#define STH_ENONFINITE -4  /* a non-finite density was detected               */
#define STH_ESTATE     -5  /* call out of order (e.g. correct before sweep)   */

/* flags (sth_problem_desc.flags) */
#define STH_HYBRID     1   /* dynamic domain adaptation (Section 2.2 and the
                              cell rules that follow scheme S^HMM)            */
#define STH_FIELD      2   /* self-consistent field; off means E == 0         */
#define STH_LITERAL_R  4   /* macroscopic criterion on |R| as printed instead
                              of eps^2 |R|                                    */
#define STH_COARSE_EXPLICIT 16 /* coarse propagator G = the explicit limit
                              scheme S^0 (Section 3.3) in ceil(dtG / (0.75
                              cfl_theta dx^2/(2 m2))) steps per interval;
                              default: one backward-Euler drift-diffusion
                              step with the field frozen at the interval
                              start                                         */
#define STH_LITERAL_FLUX 8 /* density update of scheme S^HMM cell by cell as
                              printed (Section 2.3): kinetic cells take the
                              kinetic fluxes of both interfaces, fluid cells
                              the limit fluxes m2 J; not conservative where
                              the two meet.  Default: flux-matched (each
                              interface one flux, kinetic iff the interface is
                              kinetic), which conserves mass exactly.        */

/* precision */
#define STH_FP64       0   /* everything in float64                           */
#define STH_FP32_BULK  1   /* perturbation transport, projection, relaxation
                              and velocity moments in float32; Poisson, flux
                              J, remainder, density update, coarse solve and
                              parareal correction in float64                  */

/* parareal slice-start perturbation (sth_problem_desc.start_mode) */
#define STH_START_LIFT  0  /* lifting L^L of the slice-start density, as in
                              Algorithm 1                                     */
#define STH_START_CARRY 1  /* fine end state of the previous slice from the
                              latest sweep that computed it; lifting of the
                              coarse guess before any exists                  */

typedef struct sth_problem sth_problem;

typedef struct {
    int           nx;          /* cells (= interfaces), 8 <= nx <= 2048        */
    int           nv;          /* velocities, one of 16, 32, 64, 128           */
    double        Lx;          /* torus length (> 0)                           */
    double        vstar;       /* velocity box half-width (> 0)                */
    const double *eps_iface;   /* [nx] Knudsen number at interfaces (> 0)      */
    const double *eps_cell;    /* [nx] Knudsen number at cell centres (> 0)    */
    const double *rho0;        /* [nx] initial density                         */
    const double *g0;          /* [nx*nv] initial g, x-major; NULL means 0     */
    double        T;           /* final time (> 0)                             */
    int           n_slices;    /* parareal time slices N >= 1                  */
    int           k_max;       /* iteration cap K >= 1                         */
    double        tol;         /* stop when the successive error < tol         */
    double        eta0;        /* macroscopic-criterion threshold              */
    double        delta0;      /* perturbation-norm threshold                  */
    int           lift_order;  /* L in {1, 2, 3}                               */
    int           start_mode;  /* STH_START_*                                  */
    double        cfl_theta;   /* fraction of the stable fine step, (0, 1]     */
    int           flags;       /* STH_HYBRID | STH_FIELD | STH_LITERAL_R |
                                  STH_LITERAL_FLUX | STH_COARSE_EXPLICIT      */
    int           precision;   /* STH_FP64 or STH_FP32_BULK                    */
    long long     steps_override; /* > 0 forces the fine steps per slice       */
    int           nv_y, nv_z;  /* 0, 0: 1D1V.  Otherwise the 1D3V problem of
                                  the paper (velocity box [-vstar, vstar]^3,
                                  nv x nv_y x nv_z midpoint nodes, field along
                                  x) for states of the form
                                  g(x, vx) M(vy) M(vz), M the discrete
                                  normalised Maxwellian of each axis: the form
                                  every state keeps when the initial one has
                                  it, since transport, the field and the
                                  relaxation act on vx only and the
                                  projection integrates M(vy) M(vz) to 1.  The
                                  solver carries g(x, vx) (g0 and the outputs
                                  are that factor); the 3D norm of the
                                  perturbation is sqrt(C) times its vx norm,
                                  C = sum M(vy)^2 dvy * sum M(vz)^2 dvz.
                                  Even, 2..512, both set or both 0.            */
} sth_problem_desc;

typedef struct {
    double    dx, dv, dt;      /* grid spacings and the fine step              */
    double    dtG;             /* coarse step T/N                              */
    double    m2;              /* sum_j v_j^2 M_j dv                           */
    double    rhobar;          /* mean initial density                         */
    long long steps_per_slice; /* fine steps in one slice                      */
    int       k_done;          /* parareal iterations completed                */
    int       n_slices;
    double    kinetic_iface_steps; /* kinetic interface-steps of all sweeps so
                                      far (times nv = kinetic cell-updates)    */
    double    last_err;        /* successive error of the last correction      */
    size_t    footprint_bytes; /* device bytes held by the problem             */
    int       fine_resident;   /* 1: the fine sweep keeps the rows of a slice
                                  in registers; 0: streamed every step       */
    int       fine_block;      /* threads per fine-sweep workgroup            */
    long long coarse_steps;    /* steps of the coarse scheme per interval:
                                  1, or that of STH_COARSE_EXPLICIT           */
    double    norm_scale;      /* sqrt(C) of the 1D3V form, 1 in 1D1V         */
} sth_info;

/* Launch configuration of the fine kernel for one kernel class: the class
 * is (precision, nv, nx rounded up to a multiple of 64).  block = threads
 * per workgroup (one workgroup per slice, ceil(nx/block) <= 4 interfaces per
 * thread; at most 512, or 1024 for the streamed form in FP32 bulk and in
 * FP64 with nv = 32); resident = 1 keeps a slice's rows in registers for the
 * whole slice, 0 streams them from device memory every step. */
typedef struct {
    int block;
    int resident;
} sth_fine_config;

/* Every configuration the kernel supports for the class of (precision, nx,
 * nv); writes at most cap of them to out, the total to *count. */
int  sth_fine_config_candidates(int precision, int nx, int nv, sth_fine_config *out, int cap, int *count);
/* Use cfg for the class from now on in this process (all devices, later
 * sweeps and recorded graphs); NULL returns the class to the default rule
 * (512 threads, resident when the rows fit; streamed rows beyond 512
 * interfaces take the 1024-thread workgroup where it exists).  STH_EINVAL when cfg
 * is not supported for every nx of the class.  Results do not depend on the
 * configuration except through the order of the per-step sums. */
int  sth_set_fine_config(int precision, int nx, int nv, const sth_fine_config *cfg);
/* The configuration in force for the class of (precision, nx, nv). */
int  sth_get_fine_config(int precision, int nx, int nv, sth_fine_config *out);

/* Device bytes a problem with this description needs (serving admission).
 * Only sizes are read.  *out receives the byte count. */
int  sth_footprint_bytes(const sth_problem_desc *d, size_t *out);

/* Create a problem (the initial-value problem of Section 3.1: initial data
 * rho_in, g_in, the times T^n = n T / N of the parareal decomposition, and
 * the discretisation of Section 2.3): validate the description, derive the grids, the
 * normalised Maxwellian, the stable fine step, exp(-dt/eps^2) and
 * -expm1(-dt/eps^2) per interface, and upload everything.  `arena` is a
 * 256-byte aligned device pointer of `arena_bytes` >= sth_footprint_bytes
 * (NULL: the library allocates); a host pointer is STH_EINVAL, a short
 * arena STH_ENOMEM.  Synchronises the null stream.  The problem starts at
 * iteration 0 with U^0 = rho0 and no coarse guess. */
int  sth_create(const sth_problem_desc *d, void *arena, size_t arena_bytes, sth_problem **out);

/* Coarse guess (first loop of Algorithm 1): U^n_0 = G(U^{n-1}_0) for
 * n = 1..N with G one backward-Euler drift-diffusion step of length T/N and
 * the field frozen at the slice start (STH_COARSE_EXPLICIT: the explicit
 * limit scheme S^0 of Section 3.3 over T/N); caches G values for the
 * correction. */
int  sth_coarse_sweep(sth_problem *p, void *stream);

/* The same coarse guess for several problems in one launch (one workgroup
 * per problem).  STH_EINVAL if a problem appears twice. */
int  sth_coarse_sweep_batched(sth_problem *const *p, int count, void *stream);

/* Fine propagator F = S^HMM (scheme of Section 2.3 with the cell rules of
 * Section 2.2) over every unconverged slice n > k of every problem in the
 * batch, one workgroup per slice: the parallel loop of Algorithm 1.
 * Slice-start perturbations follow start_mode.  One launch when every slice
 * has the same kernel class (precision, velocity count, interfaces per
 * thread, row form); a batch that mixes classes is one launch per precision
 * and workgroup size, each workgroup running the class of its slice, the
 * longest slices first.  Asynchronous on `stream`: several launches run
 * concurrently on four library streams of the current device (created once
 * per process, each with a CU mask of every CU so that it has a hardware
 * queue of its own; as streams created with a mask they are blocking
 * streams), which wait for `stream` and which `stream` then waits for.
 * STH_EINVAL if a problem appears twice, STH_ESTATE if one has no coarse
 * guess or a chunked sweep in progress. */
int  sth_fine_sweep_batched(sth_problem *const *p, int count, void *stream);

/* The same fine sweep advanced in chunks of at most max_steps fine steps per
 * slice, so that a caller can interleave other work between chunks (the
 * serving loop batches solves per chunk).  A call starts the sweep of every
 * problem that has none in progress (slice starts as above), then runs the
 * next chunk of steps of every slice of every problem, launched as
 * sth_fine_sweep_batched launches; a suspended slice keeps its state in
 * the problem's memory (its rows, lazy projection and halos in the slice's
 * slot, its macroscopic state in a checkpoint).  done_out[count] (optional)
 * receives 1 for each problem whose sweep has ended (in this call or an
 * earlier one) and awaits its correction; such problems are not swept
 * again.  The results equal those of sth_fine_sweep_batched bit for bit,
 * whatever the chunk lengths.  sth_fine_sweep_batched refuses a problem
 * with a chunked sweep in progress (STH_ESTATE). */
int  sth_fine_sweep_chunk(sth_problem *const *p, int count, long long max_steps, int *done_out, void *stream);

/* Sequential correction of Algorithm 1 with the new coarse value:
 * U^{k+1}_{k+1} = F^{k+1}, U^n_{k+1} = G(U^{n-1}_{k+1}) + F^n - G(U^{n-1}_k)
 * for n > k+1, then k := k+1.  When err_out is non-NULL the call
 * synchronises and stores max_{n,i} |U^n_{k+1} - U^n_k|; k_out (optional)
 * receives the new k.  Returns STH_ESTATE if no fine sweep preceded it,
 * STH_ENONFINITE (after the correction, with *err_out set) when the error
 * is not finite, i.e. a slice density holds a NaN or an infinity. */
int  sth_parareal_correct(sth_problem *p, double *err_out, int *k_out, void *stream);

/* The same correction for several problems in one launch (one workgroup per
 * problem), each problem at its own k.  When errs_out is non-NULL the call
 * synchronises once and stores each problem's error in errs_out[count];
 * STH_ENONFINITE (all corrections done, errs_out filled) when any of them is
 * not finite.  Every problem must have had a fine sweep since its last
 * correction, and none may appear twice (STH_ESTATE / STH_EINVAL otherwise). */
int  sth_parareal_correct_batched(sth_problem *const *p, int count, double *errs_out, void *stream);

/* Successive errors err_0 .. err_{k-1} of the iterations done so far
 * (Algorithm 1) to host_out[k].  Synchronises. */
int  sth_get_errors(const sth_problem *p, double *host_out);

/* A whole multiscale parareal solve of several problems recorded once as a
 * HIP graph (stream capture) and replayed by one launch: the coarse guess,
 * then for k = 0, 1, ... the fine sweep of every problem (all kernel classes
 * concurrent, as sth_fine_sweep_batched) and their corrections in one
 * launch (as sth_parareal_correct_batched).  Each problem stops on the
 * device when err_k < tol or after min(k_max, N) iterations: its later
 * kernels find its stop flag set and return at once, so no host round trip
 * decides convergence.  A launch restarts every problem from U^0 = rho0
 * (iteration count and kinetic counters cleared), so replays repeat the
 * same solve.  The graph reads the problems' device memory and its own
 * tables: the problems must outlive it and must not be used by other calls
 * while a launch is in flight.  Recording runs no kernel; creation copies
 * the tables to the device and synchronises. */
typedef struct sth_graph sth_graph;
int  sth_graph_create(sth_problem *const *p, int count, sth_graph **out);
/* Enqueue one replay on `stream`.  The problems' host-side state is
 * undefined until sth_graph_wait. */
int  sth_graph_launch(sth_graph *g, void *stream);
/* Synchronise `stream`, then settle each problem's state from the device:
 * iterations done (iters_out[count], optional) and last error
 * (last_err_out[count], optional); STH_ENONFINITE (outputs filled) when a
 * problem's last error is not finite.  Afterwards the problems continue with
 * the ordinary calls. */
int  sth_graph_wait(sth_graph *g, void *stream, int *iters_out, double *last_err_out);
void sth_graph_destroy(sth_graph *g);

/* Diagnostics of slice end n (0..N): the density U^n and, for n >= 1, the
 * perturbation the last fine sweep of slice n ended with (0 before any):
 * E, J at interfaces, Phi = -<v g>, N = eps ||g||_2 at interfaces, the
 * remainder R at cells and the kinetic-rule cell status (1 = kinetic).
 * Each output is a host array of nx entries; NULL skips it.  Synchronises. */
int  sth_moments_criteria(const sth_problem *p, int slice, double *E, double *J, double *Phi,
                          double *N, double *R, int *cell_mask, void *stream);

/* Copy the parareal iterate of Algorithm 1, the slice-end densities U^n_k
 * for n = 0..N at the current iteration k, to host_out[(N+1)*nx].
 * Synchronises. */
int  sth_get_rho(const sth_problem *p, double *host_out);

/* Copy the end-of-slice perturbation g of slice n (1..N) from the last fine
 * sweep that computed it (the fine propagator F of Algorithm 1 returns the
 * state (rho, g) of scheme S^HMM, Section 2.3; the iterate keeps only rho),
 * x-major, to host_out[nx*nv].  Synchronises. */
int  sth_get_g(const sth_problem *p, int slice, double *host_out);

/* Scalars of the problem (grids, steps, counters).  Synchronises. */
int  sth_get_info(const sth_problem *p, sth_info *out);

/* Run nsteps fine steps of one slice from a host state (rho_in, g_in, g_in
 * NULL = 0) outside the parareal bookkeeping, with the problem's grids,
 * step and flags; results to host arrays (any may be NULL): rho_out[nx],
 * g_out[nx*nv] x-major, cell_mask_out[nx], kinetic interface-steps.
 * nsteps = 0 returns the start state after the first status rule (g zero
 * on fluid interfaces).  Uses the same kernel as the batched sweep.
 * Synchronises. */
int  sth_fine_run(sth_problem *p, const double *rho_in, const double *g_in, long long nsteps,
                  double *rho_out, double *g_out, int *cell_mask_out, double *kin_out,
                  void *stream);

/* sth_fine_run with the cell status of every step exposed (the kinetic
 * region of Section 2.2, decided by the rule of that section on the data of
 * step n - 1 and applied at step n).  Row n (n = 0..nsteps) is the status
 * applied at step n, row nsteps the status after the last step; a row is
 * (nx + 63) / 64 words, bit (i mod 64) of word i / 64 set for a kinetic cell
 * i.  mask_hist (device memory, or NULL) receives the rows; mask_replay
 * (device memory, or NULL) imposes them instead of the rule, so that runs
 * in two precisions can share one sequence of kinetic regions and their
 * difference is then precision alone.  Both need STH_HYBRID (else
 * STH_EINVAL); host pointers there are STH_EINVAL.  mask_words is the
 * number of 64-bit words each given array holds; it must be at least
 * (nsteps + 1) * ((nx + 63) / 64), else STH_EINVAL (nothing is launched).
 * The caller owns both arrays.  Synchronises. */
int  sth_fine_run_masks(sth_problem *p, const double *rho_in, const double *g_in, long long nsteps,
                        const uint64_t *mask_replay, uint64_t *mask_hist, long long mask_words,
                        double *rho_out, double *g_out, int *cell_mask_out, double *kin_out,
                        void *stream);

/* sth_fine_run for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid allocation): the same arguments, kernel
 * and results, bit for bit, but the run's unit table, slice slot, densities,
 * status, counter and the staging of the perturbation live in a static
 * device workspace of 2 MiB per device (held until the process ends)
 * instead of the problem's arena; the call allocates no device memory and,
 * on success, no host memory.  STH_EINVAL (nothing launched) when the run
 * needs more than the workspace: nx * nv * (realsz + 8) bytes and about
 * 2 * nx * realsz more when g_in or g_out is given, else the slot alone
 * (512 x 64 FP64 uses 0.55 MiB; 1024 x 128 FP64 with g is refused).  Every
 * call on a device shares that device's workspace: calls that overlap on
 * one device race (the call synchronises the device first and its stream
 * before returning, so sequential calls are safe).  The device current at
 * the call must be the problem's.  Synchronises. */
int sth_fine_run_noalloc(const sth_problem *p, const double *rho_in, const double *g_in, long long nsteps,
                         double *rho_out, double *g_out, int *cell_mask_out, double *kin_out,
                         void *stream);

/* Release the problem (and its device memory if the library allocated it). */
void sth_destroy(sth_problem *p);

/* Message of the last failure on the calling thread ("" if none). */
const char *sth_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
