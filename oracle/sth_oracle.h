/*
 * sth_oracle.h -- plain, slow, FP64 CPU oracle for the hybrid micro-macro
 * fine propagator, the drift-diffusion coarse propagator and the multiscale
 * parareal iteration of
 *   T. Laidin, "A space-time hybrid parareal method for kinetic equations in
 *   the diffusive scaling" (arXiv:2511.13386).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * Model: 1D1V, x in [0, Lx) periodic, v in [-vstar, vstar] (Section 5 truncates
 * velocity to a box).  Unknowns: rho at cell centres x_i = (i+1/2)dx and the
 * scaled perturbation g' = (f - rho M)/eps at interfaces x_p = (p+1)dx
 * (interface p lies between cells p and p+1, i.e. p is "i+1/2").
 *
 * All arrays are caller-owned.  Phase-space arrays are x-major: g[p*nv + j].
 *
 * Parity unpinned (no value independent of this oracle exists): the hybrid
 * mask dynamics over long runs and full parareal results at large sizes.
 * Everything else is pinned by tests/test_oracle_pins.py and, for the
 * lifting at orders 2 and 3, by tests/test_lift_recursion.py (the
 * identification recursion carried out symbolically).
 */
#ifndef STH_ORACLE_H
#define STH_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* flag bits */
#define ORC_HYBRID   1  /* dynamic domain adaptation on (Section 2.2/2.3)      */
#define ORC_FIELD    2  /* self-consistent field on; off means E == 0          */
#define ORC_LITERAL_R 4 /* criterion on |R| as printed instead of eps^2 |R|    */
#define ORC_COARSE_EXPLICIT 16 /* coarse propagator G = the explicit limit
                              scheme S^0 (Section 3.3) in coarse_steps steps
                              per coarse interval; default: one backward-Euler
                              drift-diffusion step                           */
#define ORC_LITERAL_FLUX 8 /* cell-wise density update of scheme S^HMM as
                              printed: a kinetic cell takes the kinetic fluxes
                              of its two interfaces, a fluid cell the limit
                              fluxes m2 J (not conservative where the two kinds
                              of cells meet); default: flux-matched            */
#define ORC_STORE_F32 32 /* the perturbation g' is stored in IEEE binary32:
                              rounded to the nearest float after every fine
                              step (and at the start), all arithmetic still in
                              FP64.  Measures the floor that storing the state
                              of the FP32-bulk form in 24 bits puts under its
                              error, whatever its arithmetic; not a scheme of
                              the paper                                       */

/* slice-start perturbation of the parareal fine sweeps */
#define ORC_START_LIFT  0 /* lifting L^L of the slice-start density (Algorithm 1) */
#define ORC_START_CARRY 1 /* fine end state of the previous slice, carried       */

typedef struct {
    int    nx, nv;
    double Lx;          /* torus length                                       */
    double vstar;       /* velocity box half-width                            */
    double rhobar;      /* mean of the initial density (Poisson background)   */
    double dt;          /* fine time step                                     */
    double eta0;        /* macroscopic-criterion threshold                    */
    double delta0;      /* perturbation-norm threshold                        */
    int    flags;       /* ORC_* bits                                         */
    int    lift_order;  /* L in {1,2,3} for the lifting operator              */
    int    start_mode;  /* ORC_START_* for the parareal slice starts          */
    long   coarse_steps; /* steps of S^0 per coarse interval (ORC_COARSE_EXPLICIT) */
    double norm_scale;  /* 1D3V states g(x,vx) M(vy) M(vz): the 3D norm of the
                           perturbation over its vx norm (<= 0 means 1, 1D1V) */
} orc_params;

typedef struct {
    double kinetic_iface_steps; /* sum over steps of #kinetic interfaces      */
    double mask_flips;          /* interface status changes over the run      */
    double final_kinetic;       /* #kinetic interfaces after the last step    */
} orc_stats;

/* velocity grid: midpoint nodes, normalised Maxwellian, m2 = <v^2 M> */
void   orc_velocity_grid(int nv, double vstar, double *v, double *M, double *m2);
/* raw Maxwellian exp(-v^2/2)/sqrt(2 pi) at the same nodes (no renormalisation) */
void   orc_maxwellian_raw(int nv, double vstar, double *Mraw);

/* Table 1 coefficient of derivative order d (1..4) at offset k (-3..3) */
double orc_fd_coef(int d, int k);

/* discrete Gauss law, zero-mean gauge; E at interfaces */
void   orc_poisson(int nx, double dx, const double *rho, double rhobar, double *E);
/* macroscopic flux of the limit scheme at interfaces */
void   orc_flux_J(int nx, double dx, const double *rho, const double *E, double *J);
/* cell-centred remainder R (eq. RemainderBis) with Table 1 stencils */
void   orc_remainder(int nx, double dx, const double *rho, const double *E,
                     double rhobar, int field, double *R);

/* stable fine step bound and the per-slice step count */
double orc_dt_max(const orc_params *p, const double *eps_iface, double Emax, double theta);
long   orc_steps_per_slice(double slice_len, double dt_max, double *dt_out);

/* upwind transport (v d_x + E d_v) g' at every interface, before projection */
void   orc_transport(int nx, int nv, double Lx, double vstar, const double *g,
                      const double *E, double *A);

/* lifting operator L^L of Definition 1, evaluated at interfaces: g[p*nv+j] */
void   orc_lift(const orc_params *p, const double *eps_iface, const double *rho, double *g);

/* criteria diagnostics for a state (rho, g'): E, J, Phi=-<v g'>, N, R, mask */
void   orc_diagnostics(const orc_params *p, const double *eps_iface, const double *eps_cell,
                       const double *rho, const double *g, double *E, double *J,
                       double *Phi, double *N, double *R, int *cell_mask);

/* one slice of the hybrid fine propagator: nsteps steps of S^HMM from (rho, g) */
void   orc_fine_propagate(const orc_params *p, const double *eps_iface, const double *eps_cell,
                          const double *rho_in, const double *g_in, long nsteps,
                          double *rho_out, double *g_out, int *cell_mask_out, orc_stats *st);

/* the same with the per-step cell status recorded (hist) or imposed
 * (replay), each [(nsteps+1)][nx] bytes or NULL; hybrid runs only */
void   orc_fine_propagate_masks(const orc_params *p, const double *eps_iface, const double *eps_cell,
                                const double *rho_in, const double *g_in, long nsteps,
                                const unsigned char *replay, unsigned char *hist,
                                double *rho_out, double *g_out, int *cell_mask_out, orc_stats *st);

/* coarse G over one interval dtG: one backward-Euler drift-diffusion step
 * with frozen field, or (ORC_COARSE_EXPLICIT) coarse_steps steps of the
 * explicit limit scheme S^0 */
void   orc_coarse_step(const orc_params *p, double dtG, const double *rho_in, double *rho_out);

/* cyclic tridiagonal solve: a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i (mod n) */
int    orc_cyclic_tridiag(int n, const double *a, const double *b, const double *c,
                          const double *d, double *x);

/* multiscale parareal (Algorithm 1).  U[(N+1)*nx], err[K].  Returns iterations. */
int    orc_parareal(const orc_params *p, const double *eps_iface, const double *eps_cell,
                    int N, long steps_per_slice, double dtG, int K, double tol,
                    const double *rho_in, const double *g_in, double *U, double *err,
                    double *kinetic_iface_steps);

/* serial fine sweep with the same slice-start rule: S^n = F(S^{n-1}, g^{n-1}) */
void   orc_serial_fine(const orc_params *p, const double *eps_iface, const double *eps_cell,
                       int N, long steps_per_slice, const double *rho_in, const double *g_in,
                       double *S);

/* independent fine propagations of several slices, OpenMP over slices */
void   orc_fine_batch(const orc_params *p, const double *eps_iface, const double *eps_cell,
                      int nunits, long nsteps, const double *rho_in, const double *g_in,
                      double *rho_out, double *kinetic_iface_steps);

int    orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
