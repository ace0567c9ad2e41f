/*
 * sth_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Written from arXiv:2511.13386 (T. Laidin).  Every routine follows the
 * definition in the paper in the order the paper gives it, with plain loops
 * and sequential sums, so that it can be checked against the text by eye.
 * Nothing here is blocked, fused or reordered for speed.  Where the paper is
 * silent or garbled the reading used is stated in the comment of the routine.
 *
 * Only the tests, the smoke check and the benchmark's CPU baseline use this
 * file.  It shares no code with the GPU library.
 */
#include "sth_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

/* ---------------------------------------------------------------------------
 * Table 1 ("Central finite differences coefficients"), rows = derivative order
 * 1..4, columns = stencil offsets -3..3.  Copied from the table as printed.
 * ------------------------------------------------------------------------- */
static const double FD[4][7] = {
    {-1.0 / 60.0, 3.0 / 20.0, -3.0 / 4.0, 0.0, 3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0},
    {1.0 / 90.0, -3.0 / 20.0, 3.0 / 2.0, -49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0},
    {1.0 / 8.0, -1.0, 13.0 / 8.0, 0.0, -13.0 / 8.0, 1.0, -1.0 / 8.0},
    {-1.0 / 6.0, 2.0, -13.0 / 2.0, 28.0 / 3.0, -13.0 / 2.0, 2.0, -1.0 / 6.0},
};

double orc_fd_coef(int d, int k)
{
    if (d < 1 || d > 4 || k < -3 || k > 3) return 0.0;
    return FD[d - 1][k + 3];
}

/* d-th derivative of a periodic array f at index i with Table 1, scaled by h^d */
static double fd(int d, const double *f, int n, int i, double h)
{
    double s = 0.0;
    for (int k = -3; k <= 3; ++k) s += FD[d - 1][k + 3] * f[wrap(i + k, n)];
    return s / pow(h, (double)d);
}

/* ---------------------------------------------------------------------------
 * Velocity grid (Section 2.3, "Mesh and discretization"; Section 5 velocity
 * box).  Midpoint nodes v_j = -v* + (j+1/2) dv, first-order quadrature
 * <h> = sum_j h_j dv.  The Maxwellian is exp(-v^2/2)/sqrt(2 pi) in one
 * velocity dimension (the printed exponent has the sign garbled); it is
 * renormalised discretely so that <M> = 1 under the quadrature.
 * m2 = sum_j v_j^2 M_j dv is the coefficient of the limit scheme S^0.
 * ------------------------------------------------------------------------- */
void orc_velocity_grid(int nv, double vstar, double *v, double *M, double *m2)
{
    double dv = 2.0 * vstar / nv;
    double Z = 0.0;
    for (int j = 0; j < nv; ++j) {
        v[j] = -vstar + (j + 0.5) * dv;
        M[j] = exp(-0.5 * v[j] * v[j]);
        Z += M[j] * dv;
    }
    double s = 0.0;
    for (int j = 0; j < nv; ++j) {
        M[j] /= Z;
        s += v[j] * v[j] * M[j] * dv;
    }
    *m2 = s;
}

void orc_maxwellian_raw(int nv, double vstar, double *Mraw)
{
    double dv = 2.0 * vstar / nv;
    for (int j = 0; j < nv; ++j) {
        double v = -vstar + (j + 0.5) * dv;
        Mraw[j] = exp(-0.5 * v * v) / sqrt(2.0 * M_PI);
    }
}

/* ---------------------------------------------------------------------------
 * Discrete Gauss law of S^MM / S^0 / S^HMM:
 *     E_{i+1/2} - E_{i-1/2} = (rho_i - rhobar) dx,
 * closed on the torus by the zero-mean gauge sum_p E_p = 0.  Interface p is
 * i+1/2 with i = p, so E_p - E_{p-1} = (rho_p - rhobar) dx.
 * ------------------------------------------------------------------------- */
void orc_poisson(int nx, double dx, const double *rho, double rhobar, double *E)
{
    double s = 0.0;
    for (int p = 0; p < nx; ++p) {
        s += (rho[p] - rhobar) * dx;
        E[p] = s;
    }
    double mean = 0.0;
    for (int p = 0; p < nx; ++p) mean += E[p];
    mean /= nx;
    for (int p = 0; p < nx; ++p) E[p] -= mean;
}

/* J_{i+1/2} = (rho_{i+1} - rho_i)/dx - E_{i+1/2} rho_{i+1/2}  (limit scheme S^0),
 * with rho_{i+1/2} the average of the two neighbouring cells. */
void orc_flux_J(int nx, double dx, const double *rho, const double *E, double *J)
{
    for (int p = 0; p < nx; ++p) {
        int q = wrap(p + 1, nx);
        J[p] = (rho[q] - rho[p]) / dx - E[p] * 0.5 * (rho[p] + rho[q]);
    }
}

/* ---------------------------------------------------------------------------
 * Remainder R of the higher-order macroscopic model (eq. Remainder /
 * RemainderBis), at cell centres, with the Table 1 stencils:
 *     R = -d3 J + E d2 J + (2 rho - 3 rhobar) d1 J + 2 J d1 rho - d1 rho dt E.
 * Cell-centred quantities: E_i = (E_{i-1/2} + E_{i+1/2})/2,
 * J_i = d1 rho_i - E_i rho_i, and dt E = J - mean(J), which is the time
 * derivative of the Gauss law with the zero-mean gauge.  With the field off
 * (E == 0, no Poisson coupling) the field terms vanish and R = -d3 J.
 * ------------------------------------------------------------------------- */
void orc_remainder(int nx, double dx, const double *rho, const double *E,
                   double rhobar, int field, double *R)
{
    double *Ec = malloc(sizeof(double) * nx);
    double *Jc = malloc(sizeof(double) * nx);
    double *d1r = malloc(sizeof(double) * nx);
    double meanJ = 0.0;
    for (int i = 0; i < nx; ++i) {
        Ec[i] = field ? 0.5 * (E[wrap(i - 1, nx)] + E[i]) : 0.0;
        d1r[i] = fd(1, rho, nx, i, dx);
        Jc[i] = d1r[i] - Ec[i] * rho[i];
        meanJ += Jc[i];
    }
    meanJ /= nx;
    for (int i = 0; i < nx; ++i) {
        double d1J = fd(1, Jc, nx, i, dx);
        double d2J = fd(2, Jc, nx, i, dx);
        double d3J = fd(3, Jc, nx, i, dx);
        if (field) {
            double dtE = Jc[i] - meanJ;
            R[i] = -d3J + Ec[i] * d2J + (2.0 * rho[i] - 3.0 * rhobar) * d1J
                   + 2.0 * Jc[i] * d1r[i] - d1r[i] * dtE;
        } else {
            R[i] = -d3J;
        }
    }
    free(Ec);
    free(Jc);
    free(d1r);
}

/* ---------------------------------------------------------------------------
 * Stable fine step.  The paper gives no CFL rule; the bound used is that of
 * the exponential-relaxation/upwind micro step: for an interface with
 * c = 2 eps (vmax/dx + Emax/dv) > 1 the amplification of the stiffest upwind
 * mode stays in [-1, 1] iff dt <= eps^2 ln((c+1)/(c-1)); otherwise the
 * coupled diffusive limit dt <= dx^2/(2 m2) applies.  A 0.75 margin covers the
 * c -> 1 transition; theta is the user CFL fraction.
 * ------------------------------------------------------------------------- */
double orc_dt_max(const orc_params *p, const double *eps_iface, double Emax, double theta)
{
    int nx = p->nx, nv = p->nv;
    double dx = p->Lx / nx, dv = 2.0 * p->vstar / nv;
    double vmax = p->vstar - 0.5 * dv;
    double *v = malloc(sizeof(double) * nv), *M = malloc(sizeof(double) * nv), m2;
    orc_velocity_grid(nv, p->vstar, v, M, &m2);
    double sdiff = dx * dx / (2.0 * m2);
    double smin = sdiff;
    for (int q = 0; q < nx; ++q) {
        double eps = eps_iface[q];
        double c = 2.0 * eps * (vmax / dx + Emax / dv);
        double s = sdiff;
        if (c > 1.0) {
            double s2 = eps * eps * log((c + 1.0) / (c - 1.0));
            if (s2 < s) s = s2;
        }
        if (s < smin) smin = s;
    }
    free(v);
    free(M);
    return theta * 0.75 * smin;
}

long orc_steps_per_slice(double slice_len, double dt_max, double *dt_out)
{
    long n = (long)ceil(slice_len / dt_max);
    if (n < 1) n = 1;
    *dt_out = slice_len / (double)n;
    return n;
}

/* ---------------------------------------------------------------------------
 * Lifting L^L (Definition 1, Section 3.2/3.3): g = sum_{l=1..L} eps^l h^(l)
 * from the Chapman-Enskog recursion (eq. Identification) with the transport
 * operator T = v d_x + E d_v, dv M = -v M, the closures dt rho = d_x J and
 * dt E = J - mean J, evaluated at interfaces from the averaged density
 * rho~_p = (rho_p + rho_{p+1})/2 with Table 1 derivatives of interface
 * arrays.  In g' = g/eps units:
 *     h1 = -v M J
 *     h2 = (v^2 - m2) M K,                 K = d1 J - E J
 *     h3 = v M [dtJ - (v^2 - m2) d1 K - (2 + m2 - v^2) E K],
 *          dtJ = d2 J - (J - mean J) rho~ - E d1 J
 *     g'  = h1 + eps h2 + eps^2 h3, truncated at order L.
 * The continuous constant 1 = <v^2 M> is replaced by the discrete m2 so that
 * <h2> = 0 holds under the quadrature; h1 and h3 are odd in v.
 * ------------------------------------------------------------------------- */
void orc_lift(const orc_params *p, const double *eps_iface, const double *rho, double *g)
{
    int nx = p->nx, nv = p->nv, field = (p->flags & ORC_FIELD) != 0;
    double dx = p->Lx / nx;
    double *v = malloc(sizeof(double) * nv), *M = malloc(sizeof(double) * nv), m2;
    orc_velocity_grid(nv, p->vstar, v, M, &m2);
    double *E = calloc(nx, sizeof(double));
    double *J = malloc(sizeof(double) * nx), *K = malloc(sizeof(double) * nx);
    double *rt = malloc(sizeof(double) * nx);
    if (field) orc_poisson(nx, dx, rho, p->rhobar, E);
    orc_flux_J(nx, dx, rho, E, J);
    double meanJ = 0.0;
    for (int q = 0; q < nx; ++q) {
        rt[q] = 0.5 * (rho[q] + rho[wrap(q + 1, nx)]);
        meanJ += J[q];
    }
    meanJ /= nx;
    for (int q = 0; q < nx; ++q) K[q] = fd(1, J, nx, q, dx) - E[q] * J[q];
    for (int q = 0; q < nx; ++q) {
        double d1J = fd(1, J, nx, q, dx);
        double d2J = fd(2, J, nx, q, dx);
        double d1K = fd(1, K, nx, q, dx);
        double dtJ = d2J - E[q] * d1J - (field ? (J[q] - meanJ) * rt[q] : 0.0);
        double eps = eps_iface[q];
        for (int j = 0; j < nv; ++j) {
            double vj = v[j], w = vj * vj - m2;
            double h1 = -vj * M[j] * J[q];
            double h2 = w * M[j] * K[q];
            double h3 = vj * M[j] * (dtJ - w * d1K - (2.0 + m2 - vj * vj) * E[q] * K[q]);
            double val = h1;
            if (p->lift_order >= 2) val += eps * h2;
            if (p->lift_order >= 3) val += eps * eps * h3;
            g[q * nv + j] = val;
        }
    }
    free(v); free(M); free(E); free(J); free(K); free(rt);
}

/* ---------------------------------------------------------------------------
 * Criteria (Section 2.2 and the cell rules after S^HMM).
 *   N_p   = || g_p ||_2 = eps_p sqrt(sum_j g'_{p,j}^2 dv)   (g = eps g')
 *   crit  = eps_i^2 |R_i|  (the deviation of the higher-order model from the
 *           limit is eps^2 R); ORC_LITERAL_R compares |R_i| as printed.
 * Fluid cell:   kinetic at n+1 iff crit > eta0.
 * Kinetic cell: kinetic at n+1 iff max(N_{i-1/2}, N_{i+1/2}) > delta0 or
 *               crit > eta0 ("at least one condition" keeps it kinetic).
 * Interface p is kinetic iff one of its two cells is.
 * ------------------------------------------------------------------------- */
static double crit_R(const orc_params *p, double eps_c, double R)
{
    return (p->flags & ORC_LITERAL_R) ? fabs(R) : eps_c * eps_c * fabs(R);
}

/* N_p = eps_p ||g'_p||_2 over the velocity space; for 1D3V states of the
 * form g(x, vx) M(vy) M(vz) the 3D norm is norm_scale times the vx norm. */
static void gnorms(const orc_params *p, const double *eps_iface, const double *g, double *N)
{
    double dv = 2.0 * p->vstar / p->nv;
    double ns = p->norm_scale > 0.0 ? p->norm_scale : 1.0;
    for (int q = 0; q < p->nx; ++q) {
        double s = 0.0;
        for (int j = 0; j < p->nv; ++j) s += g[q * p->nv + j] * g[q * p->nv + j] * dv;
        N[q] = (eps_iface[q] * ns) * sqrt(s);
    }
}

void orc_diagnostics(const orc_params *p, const double *eps_iface, const double *eps_cell,
                     const double *rho, const double *g, double *E, double *J,
                     double *Phi, double *N, double *R, int *cell_mask)
{
    int nx = p->nx, nv = p->nv, field = (p->flags & ORC_FIELD) != 0;
    double dx = p->Lx / nx, dv = 2.0 * p->vstar / nv;
    double *v = malloc(sizeof(double) * nv), *M = malloc(sizeof(double) * nv), m2;
    orc_velocity_grid(nv, p->vstar, v, M, &m2);
    if (field) orc_poisson(nx, dx, rho, p->rhobar, E);
    else memset(E, 0, sizeof(double) * nx);
    orc_flux_J(nx, dx, rho, E, J);
    orc_remainder(nx, dx, rho, E, p->rhobar, field, R);
    gnorms(p, eps_iface, g, N);
    for (int q = 0; q < nx; ++q) {
        double s = 0.0;
        for (int j = 0; j < nv; ++j) s += v[j] * g[q * nv + j] * dv;
        Phi[q] = -s;
    }
    for (int i = 0; i < nx; ++i) {
        double nl = N[wrap(i - 1, nx)], nr = N[i];
        double nmax = nl > nr ? nl : nr;
        cell_mask[i] = (nmax > p->delta0) || (crit_R(p, eps_cell[i], R[i]) > p->eta0);
    }
    free(v);
    free(M);
}

/* ---------------------------------------------------------------------------
 * Upwind transport of the perturbation at interface q (the operator inside
 * T^n of S^MM, before the projection):
 *   A_j = [v+ (g_{q,j} - g_{q-1,j}) + v- (g_{q+1,j} - g_{q,j})]/dx
 *       + (G_{j+1/2} - G_{j-1/2})/dv,
 *   G_{j+1/2} = E+ g_{q,j} + E- g_{q,j+1},  G_{-1/2} = G_{nv-1/2} = 0,
 * with r+ = max(r, 0), r- = min(r, 0): the upwind value is taken on the side
 * the characteristic comes from (the printed r^- = (|r| - r)/2 has its sign
 * garbled: it would make the flux downwind for negative speeds).
 * ------------------------------------------------------------------------- */
static void transport_at(int nx, int nv, double dx, double dv, const double *v,
                         const double *g, double Eq, int q, double *A)
{
    int qm = wrap(q - 1, nx), qp = wrap(q + 1, nx);
    double Ep = Eq > 0.0 ? Eq : 0.0, Em = Eq < 0.0 ? Eq : 0.0;
    for (int j = 0; j < nv; ++j) {
        double vp = v[j] > 0.0 ? v[j] : 0.0, vm = v[j] < 0.0 ? v[j] : 0.0;
        double ax = vp * (g[q * nv + j] - g[qm * nv + j]) / dx
                  + vm * (g[qp * nv + j] - g[q * nv + j]) / dx;
        double Ghi = (j < nv - 1) ? Ep * g[q * nv + j] + Em * g[q * nv + j + 1] : 0.0;
        double Glo = (j > 0) ? Ep * g[q * nv + j - 1] + Em * g[q * nv + j] : 0.0;
        A[j] = ax + (Ghi - Glo) / dv;
    }
}

void orc_transport(int nx, int nv, double Lx, double vstar, const double *g,
                   const double *E, double *A)
{
    double dx = Lx / nx, dv = 2.0 * vstar / nv;
    double *v = malloc(sizeof(double) * nv), *M = malloc(sizeof(double) * nv), m2;
    orc_velocity_grid(nv, vstar, v, M, &m2);
    for (int q = 0; q < nx; ++q) transport_at(nx, nv, dx, dv, v, g, E[q], q, A + (size_t)q * nv);
    free(v);
    free(M);
}

/* ---------------------------------------------------------------------------
 * Hybrid fine propagator F = S^HMM over nsteps steps (Section 2.3).
 *
 * Per step n -> n+1, with g' = g/eps stored at interfaces:
 *  1. E^n from rho^n (Gauss law), J^n_p (limit-scheme flux).
 *  2. Criteria on (rho^n, g'^n) give the status at n+1.
 *  3. Kinetic interfaces of step n (S^MM in g' form):
 *       A_{p,j} = upwind (v d_x + E d_v) g'   with
 *         x: v+ (g'_{p,j} - g'_{p-1,j})/dx + v- (g'_{p+1,j} - g'_{p,j})/dx,
 *            r+ = max(r,0), r- = min(r,0) (the printed r^-- sign is garbled)
 *         v: (G_{j+1/2} - G_{j-1/2})/dv, G_{j+1/2} = E+ g'_j + E- g'_{j+1},
 *            zero flux through +-v*
 *       T_{p,j} = A_{p,j} - M_j <A_p>             ((I - Pi) projection)
 *       g'^{n+1} = e_p g'^n - a_p (eps_p T + v_j M_j J_p),
 *            e_p = exp(-dt/eps_p^2), a_p = 1 - e_p
 *       Phi_p = -<v g'^{n+1}_p>
 *     Fluid interfaces: g' = 0, Phi_p = m2 J_p (limit-scheme flux).
 *     Each interface carries one flux, so the density update telescopes
 *     (flux-matched coupling, the conservative form named in the Remark after
 *     Lemma 1).
 *  4. rho^{n+1}_i = rho^n_i + dt/dx (Phi_{i+1/2} - Phi_{i-1/2}).
 *  5. Interfaces fluid at n+1 get g' = 0; the stored 0 is the start value of
 *     an interface that turns kinetic.
 * The status at the first step is the kinetic-cell rule applied to every cell
 * with the given g'.
 * ------------------------------------------------------------------------- */
void orc_fine_propagate(const orc_params *p, const double *eps_iface, const double *eps_cell,
                        const double *rho_in, const double *g_in, long nsteps,
                        double *rho_out, double *g_out, int *cell_mask_out, orc_stats *st)
{
    orc_fine_propagate_masks(p, eps_iface, eps_cell, rho_in, g_in, nsteps, NULL, NULL,
                             rho_out, g_out, cell_mask_out, st);
}

/* The same propagator with the cell status of every step exposed: hist
 * (if not NULL) receives the status applied at step n in row n, n = 0..nsteps
 * (row nsteps: the status after the last step); replay (if not NULL) supplies
 * those rows instead of the rule of Section 2.2, so that two runs can share
 * one sequence of kinetic regions.  Rows are nx bytes (1 = kinetic cell);
 * both need the hybrid flag. */
void orc_fine_propagate_masks(const orc_params *p, const double *eps_iface, const double *eps_cell,
                              const double *rho_in, const double *g_in, long nsteps,
                              const unsigned char *replay, unsigned char *hist,
                              double *rho_out, double *g_out, int *cell_mask_out, orc_stats *st)
{
    int nx = p->nx, nv = p->nv;
    int hybrid = (p->flags & ORC_HYBRID) != 0, field = (p->flags & ORC_FIELD) != 0;
    double dx = p->Lx / nx, dv = 2.0 * p->vstar / nv, dt = p->dt;
    double *v = malloc(sizeof(double) * nv), *M = malloc(sizeof(double) * nv), m2;
    orc_velocity_grid(nv, p->vstar, v, M, &m2);

    double *rho = malloc(sizeof(double) * nx);
    double *g = malloc(sizeof(double) * nx * nv), *gn = malloc(sizeof(double) * nx * nv);
    double *E = calloc(nx, sizeof(double)), *J = malloc(sizeof(double) * nx);
    double *R = malloc(sizeof(double) * nx), *N = malloc(sizeof(double) * nx);
    double *Phi = malloc(sizeof(double) * nx), *A = malloc(sizeof(double) * nv);
    double *e = malloc(sizeof(double) * nx), *a = malloc(sizeof(double) * nx);
    int *cell = malloc(sizeof(int) * nx), *ncell = malloc(sizeof(int) * nx);
    int *ifc = malloc(sizeof(int) * nx), *nifc = malloc(sizeof(int) * nx);

    memcpy(rho, rho_in, sizeof(double) * nx);
    if (g_in) memcpy(g, g_in, sizeof(double) * nx * nv);
    else memset(g, 0, sizeof(double) * nx * nv);
    const int store_f32 = (p->flags & ORC_STORE_F32) != 0;
    if (store_f32)
        for (size_t u = 0; u < (size_t)nx * nv; ++u) g[u] = (double)(float)g[u];
    for (int q = 0; q < nx; ++q) {
        double r = dt / (eps_iface[q] * eps_iface[q]);
        e[q] = exp(-r);
        a[q] = -expm1(-r);
    }
    double kin_steps = 0.0, flips = 0.0;

    /* status at the first step */
    if (hybrid) {
        if (field) orc_poisson(nx, dx, rho, p->rhobar, E);
        orc_remainder(nx, dx, rho, E, p->rhobar, field, R);
        gnorms(p, eps_iface, g, N);
        for (int i = 0; i < nx; ++i) {
            double nl = N[wrap(i - 1, nx)], nr = N[i];
            double nmax = nl > nr ? nl : nr;
            cell[i] = (nmax > p->delta0) || (crit_R(p, eps_cell[i], R[i]) > p->eta0);
            if (replay) cell[i] = replay[i] != 0;
            if (hist) hist[i] = (unsigned char)cell[i];
        }
        for (int q = 0; q < nx; ++q) {
            ifc[q] = cell[q] || cell[wrap(q + 1, nx)];
            if (!ifc[q])
                for (int j = 0; j < nv; ++j) g[q * nv + j] = 0.0;
        }
    } else {
        for (int q = 0; q < nx; ++q) cell[q] = ifc[q] = 1;
    }

    for (long n = 0; n < nsteps; ++n) {
        /* 1. field and macroscopic flux at time n */
        if (field) orc_poisson(nx, dx, rho, p->rhobar, E);
        orc_flux_J(nx, dx, rho, E, J);

        /* 2. status at n+1 from data at n */
        if (hybrid) {
            orc_remainder(nx, dx, rho, E, p->rhobar, field, R);
            gnorms(p, eps_iface, g, N);
            for (int i = 0; i < nx; ++i) {
                double c = crit_R(p, eps_cell[i], R[i]);
                if (cell[i]) {
                    double nl = N[wrap(i - 1, nx)], nr = N[i];
                    double nmax = nl > nr ? nl : nr;
                    ncell[i] = (nmax > p->delta0) || (c > p->eta0);
                } else {
                    ncell[i] = c > p->eta0;
                }
                if (replay) ncell[i] = replay[(size_t)(n + 1) * nx + i] != 0;
                if (hist) hist[(size_t)(n + 1) * nx + i] = (unsigned char)ncell[i];
            }
            for (int q = 0; q < nx; ++q) nifc[q] = ncell[q] || ncell[wrap(q + 1, nx)];
        }

        /* 3. perturbation update and interface fluxes */
        for (int q = 0; q < nx; ++q) {
            if (ifc[q]) kin_steps += 1.0;
            if (!ifc[q]) {
                for (int j = 0; j < nv; ++j) gn[q * nv + j] = 0.0;
                Phi[q] = m2 * J[q];
                continue;
            }
            transport_at(nx, nv, dx, dv, v, g, E[q], q, A);
            double sA = 0.0;
            for (int j = 0; j < nv; ++j) sA += A[j] * dv;
            double flux = 0.0;
            for (int j = 0; j < nv; ++j) {
                double T = A[j] - M[j] * sA;
                double val = e[q] * g[q * nv + j] - a[q] * (eps_iface[q] * T + v[j] * M[j] * J[q]);
                gn[q * nv + j] = val;
                flux += v[j] * val * dv;
            }
            Phi[q] = -flux;
        }

        /* 4. density update: flux-matched (conservative), or cell-wise as
         *    printed in scheme S^HMM (kinetic cells: kinetic fluxes; fluid
         *    cells: limit fluxes m2 J), with the cell status of time n */
        if (hybrid && (p->flags & ORC_LITERAL_FLUX)) {
            for (int i = 0; i < nx; ++i) {
                int im = wrap(i - 1, nx);
                double fr = cell[i] ? Phi[i] : m2 * J[i];
                double fl = cell[i] ? Phi[im] : m2 * J[im];
                rho[i] = rho[i] + dt / dx * (fr - fl);
            }
        } else {
            for (int i = 0; i < nx; ++i) rho[i] = rho[i] + dt / dx * (Phi[i] - Phi[wrap(i - 1, nx)]);
        }

        if (store_f32)
            for (size_t u = 0; u < (size_t)nx * nv; ++u) gn[u] = (double)(float)gn[u];

        /* 5. new status; fluid interfaces hold g' = 0 */
        if (hybrid) {
            for (int q = 0; q < nx; ++q) {
                if (nifc[q] != ifc[q]) flips += 1.0;
                if (!nifc[q])
                    for (int j = 0; j < nv; ++j) gn[q * nv + j] = 0.0;
                ifc[q] = nifc[q];
                cell[q] = ncell[q];
            }
        }
        double *t = g; g = gn; gn = t;
    }

    memcpy(rho_out, rho, sizeof(double) * nx);
    if (g_out) memcpy(g_out, g, sizeof(double) * nx * nv);
    if (cell_mask_out) memcpy(cell_mask_out, cell, sizeof(int) * nx);
    if (st) {
        double fk = 0.0;
        for (int q = 0; q < nx; ++q) fk += ifc[q];
        st->kinetic_iface_steps = kin_steps;
        st->mask_flips = flips;
        st->final_kinetic = fk;
    }
    free(v); free(M); free(rho); free(g); free(gn); free(E); free(J); free(R); free(N);
    free(Phi); free(A); free(e); free(a); free(cell); free(ncell); free(ifc); free(nifc);
}

/* ---------------------------------------------------------------------------
 * Cyclic tridiagonal solve by the Sherman-Morrison correction of the Thomas
 * algorithm (textbook).  Row i: a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i with
 * indices mod n; a_0 multiplies x_{n-1} and c_{n-1} multiplies x_0.
 * ------------------------------------------------------------------------- */
static void thomas(int n, const double *a, const double *b, const double *c,
                   const double *d, double *x, double *cp, double *dp)
{
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double m = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / m;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

int orc_cyclic_tridiag(int n, const double *a, const double *b, const double *c,
                       const double *d, double *x)
{
    if (n < 3) return -1;
    double *bb = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n);
    double *z = malloc(sizeof(double) * n), *cp = malloc(sizeof(double) * n);
    double *dp = malloc(sizeof(double) * n);
    double gamma = -b[0];
    memcpy(bb, b, sizeof(double) * n);
    bb[0] = b[0] - gamma;
    bb[n - 1] = b[n - 1] - a[0] * c[n - 1] / gamma;
    thomas(n, a, bb, c, d, x, cp, dp);
    for (int i = 0; i < n; ++i) u[i] = 0.0;
    u[0] = gamma;
    u[n - 1] = c[n - 1];
    thomas(n, a, bb, c, u, z, cp, dp);
    double fact = (x[0] + a[0] * x[n - 1] / gamma) / (1.0 + z[0] + a[0] * z[n - 1] / gamma);
    for (int i = 0; i < n; ++i) x[i] -= fact * z[i];
    free(bb); free(u); free(z); free(cp); free(dp);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Coarse propagator G: one backward-Euler step of the drift-diffusion limit
 * (eq. DD) in the discrete form of S^0, with the field frozen at the slice
 * start (the field is explicit in time, Section 3.3):
 *     (I - dtG L_E) rho~ = rho^n,
 *     (L_E r)_i = m2 (J_{i+1/2}[r] - J_{i-1/2}[r]) / dx,
 *     J_{i+1/2}[r] = (r_{i+1} - r_i)/dx - E_{i+1/2} (r_i + r_{i+1})/2,
 * followed by the conservative form rho^{n+1} = rho^n + dtG L_E rho~, which
 * equals rho~ in exact arithmetic and telescopes in floating point.
 * ------------------------------------------------------------------------- */
/* explicit limit scheme S^0 (Section 2.3): nsteps steps of
 *   rho_i <- rho_i + dt/dx (m2 J_{i+1/2} - m2 J_{i-1/2}),
 * J from the current rho and its Gauss-law field (the fluid fluxes of the
 * fine scheme, in the same order of operations) */
static void limit_scheme(const orc_params *p, double dt, long nsteps, const double *rho_in, double *rho_out)
{
    int nx = p->nx, field = (p->flags & ORC_FIELD) != 0;
    double dx = p->Lx / nx;
    double *v = malloc(sizeof(double) * p->nv), *M = malloc(sizeof(double) * p->nv), m2;
    orc_velocity_grid(p->nv, p->vstar, v, M, &m2);
    double *E = calloc(nx, sizeof(double)), *J = malloc(sizeof(double) * nx);
    double *Phi = malloc(sizeof(double) * nx);
    memcpy(rho_out, rho_in, sizeof(double) * nx);
    for (long n = 0; n < nsteps; ++n) {
        if (field) orc_poisson(nx, dx, rho_out, p->rhobar, E);
        orc_flux_J(nx, dx, rho_out, E, J);
        for (int q = 0; q < nx; ++q) Phi[q] = m2 * J[q];
        for (int i = 0; i < nx; ++i) rho_out[i] = rho_out[i] + dt / dx * (Phi[i] - Phi[wrap(i - 1, nx)]);
    }
    free(v); free(M); free(E); free(J); free(Phi);
}

void orc_coarse_step(const orc_params *p, double dtG, const double *rho_in, double *rho_out)
{
    if (p->flags & ORC_COARSE_EXPLICIT) {
        long ns = p->coarse_steps > 0 ? p->coarse_steps : 1;
        limit_scheme(p, dtG / (double)ns, ns, rho_in, rho_out);
        return;
    }
    int nx = p->nx, field = (p->flags & ORC_FIELD) != 0;
    double dx = p->Lx / nx;
    double *v = malloc(sizeof(double) * p->nv), *M = malloc(sizeof(double) * p->nv), m2;
    orc_velocity_grid(p->nv, p->vstar, v, M, &m2);
    double *E = calloc(nx, sizeof(double));
    double *a = malloc(sizeof(double) * nx), *b = malloc(sizeof(double) * nx);
    double *c = malloc(sizeof(double) * nx), *x = malloc(sizeof(double) * nx);
    double *Jt = malloc(sizeof(double) * nx);
    if (field) orc_poisson(nx, dx, rho_in, p->rhobar, E);
    double alpha = m2 * dtG / (dx * dx), beta = m2 * dtG / (2.0 * dx);
    for (int i = 0; i < nx; ++i) {
        double Ew = E[wrap(i - 1, nx)], Ee = E[i];
        a[i] = -alpha - beta * Ew;
        b[i] = 1.0 + 2.0 * alpha + beta * (Ee - Ew);
        c[i] = -alpha + beta * Ee;
    }
    orc_cyclic_tridiag(nx, a, b, c, rho_in, x);
    orc_flux_J(nx, dx, x, E, Jt);
    for (int i = 0; i < nx; ++i)
        rho_out[i] = rho_in[i] + dtG * m2 * (Jt[i] - Jt[wrap(i - 1, nx)]) / dx;
    free(v); free(M); free(E); free(a); free(b); free(c); free(x); free(Jt);
}

/* ---------------------------------------------------------------------------
 * Multiscale parareal (Section 3.1 and Algorithm 1), standard form:
 *   U^0 = rho_in;  coarse guess U^n_0 = G(U^{n-1}_0), Gc^n = U^n_0.
 *   iteration k = 0, 1, ...:
 *     jumps (independent per slice, the paper's parallel loop), n > k:
 *        Fv^n = F(U^{n-1}_k, g^{n-1})
 *     sequential correction with the new coarse value:
 *        U^{k+1}_{k+1} = Fv^{k+1}
 *        U^n_{k+1} = G(U^{n-1}_{k+1}) + (Fv^n - Gc^n), Gc^n = G(U^{n-1}_{k+1})
 *        converged slices n <= k keep their value
 *     err_k = max_{n,i} |U^n_{k+1} - U^n_k|; stop when err_k < tol or k+1 = K.
 * The field is never corrected: each propagator recomputes it from rho.
 * Slice-start perturbation g^{n-1} (g_in for n = 1):
 *   ORC_START_LIFT  the lifting L^L(U^{n-1}_k), as in Algorithm 1;
 *   ORC_START_CARRY the end state of slice n-1 from the most recent fine
 *                   sweep that computed it, the lifting of the slice-start
 *                   density before any exists.  At K = N this reproduces the
 *                   serial fine run whose perturbation is carried across
 *                   slice ends.
 * ------------------------------------------------------------------------- */
static void slice_start(const orc_params *p, const double *eps_iface, int n, const double *g_in,
                        const double *Uprev, const double *gend_prev, int have_prev, double *gs)
{
    size_t sz = (size_t)p->nx * p->nv;
    if (n == 1) {
        if (g_in) memcpy(gs, g_in, sizeof(double) * sz);
        else memset(gs, 0, sizeof(double) * sz);
    } else if (p->start_mode == ORC_START_CARRY && have_prev) {
        memcpy(gs, gend_prev, sizeof(double) * sz);
    } else {
        orc_lift(p, eps_iface, Uprev, gs);
    }
}

int orc_parareal(const orc_params *p, const double *eps_iface, const double *eps_cell,
                 int N, long steps_per_slice, double dtG, int K, double tol,
                 const double *rho_in, const double *g_in, double *U, double *err,
                 double *kinetic_iface_steps)
{
    int nx = p->nx;
    size_t slab = (size_t)nx, gsz = (size_t)nx * p->nv;
    double *Gc = calloc((size_t)(N + 1) * slab, sizeof(double));
    double *Fv = calloc((size_t)(N + 1) * slab, sizeof(double));
    double *Un = malloc(sizeof(double) * (size_t)(N + 1) * slab);
    double *gend = calloc((size_t)(N + 1) * gsz, sizeof(double));
    double *gst = calloc((size_t)(N + 1) * gsz, sizeof(double));
    int *have = calloc((size_t)(N + 1), sizeof(int));
    double kin = 0.0;

    memcpy(U, rho_in, sizeof(double) * nx);
    for (int n = 1; n <= N; ++n) {
        orc_coarse_step(p, dtG, U + (n - 1) * slab, U + n * slab);
        memcpy(Gc + n * slab, U + n * slab, sizeof(double) * nx);
    }
    int iters = 0;
    for (int k = 0; k < K && k < N; ++k) {
        for (int n = k + 1; n <= N; ++n)
            slice_start(p, eps_iface, n, g_in, U + (n - 1) * slab, gend + (n - 1) * gsz,
                        have[n - 1], gst + n * gsz);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : kin)
        for (int n = k + 1; n <= N; ++n) {
            orc_stats st;
            orc_fine_propagate(p, eps_iface, eps_cell, U + (n - 1) * slab, gst + n * gsz,
                               steps_per_slice, Fv + n * slab, gend + n * gsz, NULL, &st);
            kin += st.kinetic_iface_steps;
        }
        for (int n = k + 1; n <= N; ++n) have[n] = 1;
        memcpy(Un, U, sizeof(double) * (size_t)(N + 1) * slab);
        memcpy(Un + (k + 1) * slab, Fv + (k + 1) * slab, sizeof(double) * nx);
        double *Gn = malloc(sizeof(double) * nx);
        for (int n = k + 2; n <= N; ++n) {
            orc_coarse_step(p, dtG, Un + (n - 1) * slab, Gn);
            for (int i = 0; i < nx; ++i)
                Un[n * slab + i] = Gn[i] + (Fv[n * slab + i] - Gc[n * slab + i]);
            memcpy(Gc + n * slab, Gn, sizeof(double) * nx);
        }
        free(Gn);
        double e = 0.0;
        for (size_t t = 0; t < (size_t)(N + 1) * slab; ++t) {
            double d = fabs(Un[t] - U[t]);
            if (!(d <= e)) e = d; /* a NaN difference propagates into the error */
        }
        memcpy(U, Un, sizeof(double) * (size_t)(N + 1) * slab);
        err[k] = e;
        iters = k + 1;
        if (e < tol) break;
    }
    if (kinetic_iface_steps) *kinetic_iface_steps = kin;
    free(Gc); free(Fv); free(Un); free(gend); free(gst); free(have);
    return iters;
}

/* serial fine sweep with the parareal slice-start rule, which parareal
 * reproduces at K = N: S^n = F(S^{n-1}, g^{n-1}) */
void orc_serial_fine(const orc_params *p, const double *eps_iface, const double *eps_cell,
                     int N, long steps_per_slice, const double *rho_in, const double *g_in,
                     double *S)
{
    int nx = p->nx;
    size_t gsz = (size_t)nx * p->nv;
    double *gs = malloc(sizeof(double) * gsz), *ge = calloc(gsz, sizeof(double));
    memcpy(S, rho_in, sizeof(double) * nx);
    for (int n = 1; n <= N; ++n) {
        slice_start(p, eps_iface, n, g_in, S + (size_t)(n - 1) * nx, ge, n > 1, gs);
        orc_fine_propagate(p, eps_iface, eps_cell, S + (size_t)(n - 1) * nx, gs, steps_per_slice,
                           S + (size_t)n * nx, ge, NULL, NULL);
    }
    free(gs);
    free(ge);
}

void orc_fine_batch(const orc_params *p, const double *eps_iface, const double *eps_cell,
                    int nunits, long nsteps, const double *rho_in, const double *g_in,
                    double *rho_out, double *kinetic_iface_steps)
{
    int nx = p->nx, nv = p->nv;
    double kin = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : kin)
    for (int u = 0; u < nunits; ++u) {
        orc_stats st;
        orc_fine_propagate(p, eps_iface, eps_cell, rho_in + (size_t)u * nx,
                           g_in ? g_in + (size_t)u * nx * nv : NULL, nsteps,
                           rho_out + (size_t)u * nx, NULL, NULL, &st);
        kin += st.kinetic_iface_steps;
    }
    if (kinetic_iface_steps) *kinetic_iface_steps = kin;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
