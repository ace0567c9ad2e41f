// sth_kernels.hip -- gfx950 kernels of the hybrid micro-macro parareal solver.
//
// Method: T. Laidin, arXiv:2511.13386.  Fine propagator = scheme S^HMM of
// Section 2.3 (micro-macro scheme S^MM on kinetic interfaces, limit scheme S^0
// fluxes on fluid ones) with the cell rules of Section 2.2; coarse propagator
// = backward Euler of the drift-diffusion limit; parareal of Section 3 /
// Algorithm 1.
//
// Fine-sweep design (MI355X): one workgroup owns one parareal slice of one
// problem for the whole slice (all its fine steps in one persistent launch).
// Thread t owns interfaces/cells p = k*B + t (slab k), one lane per
// interface, so every velocity moment of an interface is an in-register sum
// and the x-upwind neighbour is one lane away (cross-lane shift; the two wave
// edges read a double-buffered LDS halo).  The perturbation of the slice
// stays in VGPRs for the whole slice when it fits ("resident"), otherwise it
// is streamed from a v-major global buffer each step (coalesced: lanes are
// consecutive interfaces).  Per fine step the workgroup needs three barriers:
//   P1  density update from the previous fluxes, interface status, wave
//       prefix sums of (rho - rhobar) dx                       | B1
//   P2  field E (Gauss law, zero-mean gauge), flux J, cell-centred J  | B2
//   P3  transport + projection + relaxation of kinetic interfaces, flux
//       Phi, norms; remainder R and the cell rule                  | B3
#include "sth_internal.h"
#include "sth.h"

#include <cmath>

namespace sth {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// Central 7-point stencils of Table 1 (derivative orders 1..3), offsets -3..3.
__device__ __forceinline__ double fd1(const double *f, int i, int n)
{
    return (-1.0 / 60.0) * f[wrapi(i - 3, n)] + (3.0 / 20.0) * f[wrapi(i - 2, n)]
           + (-3.0 / 4.0) * f[wrapi(i - 1, n)] + (3.0 / 4.0) * f[wrapi(i + 1, n)]
           + (-3.0 / 20.0) * f[wrapi(i + 2, n)] + (1.0 / 60.0) * f[wrapi(i + 3, n)];
}
__device__ __forceinline__ double fd2(const double *f, int i, int n)
{
    return (1.0 / 90.0) * f[wrapi(i - 3, n)] + (-3.0 / 20.0) * f[wrapi(i - 2, n)]
           + (3.0 / 2.0) * f[wrapi(i - 1, n)] + (-49.0 / 18.0) * f[i]
           + (3.0 / 2.0) * f[wrapi(i + 1, n)] + (-3.0 / 20.0) * f[wrapi(i + 2, n)]
           + (1.0 / 90.0) * f[wrapi(i + 3, n)];
}
__device__ __forceinline__ double fd3(const double *f, int i, int n)
{
    return (1.0 / 8.0) * f[wrapi(i - 3, n)] + (-1.0) * f[wrapi(i - 2, n)]
           + (13.0 / 8.0) * f[wrapi(i - 1, n)] + (-13.0 / 8.0) * f[wrapi(i + 1, n)]
           + (1.0) * f[wrapi(i + 2, n)] + (-1.0 / 8.0) * f[wrapi(i + 3, n)];
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS layout of the fine kernel.  Same function on host (sizing) and device.
struct FineLds {
    size_t rho, jc, phi, E, nrm, cm, tot, wtot, jtot, halo, total;
};
__host__ __device__ inline FineLds fine_lds(int nx, int nv, int realsz, int nslot)
{
    FineLds L;
    size_t o = 0;
    L.rho = o;  o = align16(o + sizeof(double) * nx);
    L.jc = o;   o = align16(o + sizeof(double) * nx);
    L.phi = o;  o = align16(o + sizeof(double) * nx);
    L.E = o;    o = align16(o + sizeof(double) * nx);
    L.nrm = o;  o = align16(o + (size_t)realsz * 2 * nx);
    L.cm = o;   o = align16(o + sizeof(unsigned char) * nx);
    L.tot = o;  o = align16(o + sizeof(double) * nslot);
    L.wtot = o; o = align16(o + sizeof(double) * nslot);
    L.jtot = o; o = align16(o + sizeof(double) * nslot);
    L.halo = o; o = align16(o + (size_t)realsz * 2 * 2 * ((nx + kWave - 1) / kWave) * (nv / 2));
    L.total = o;
    return L;
}


// ------------------------------------------------------------ fine sweep
// Row state.  A unit's perturbation lives in a v-major global buffer
// W[j][p] (lanes = consecutive interfaces, so every row access is coalesced)
// followed by C1[2][p].  The projection of the micro-macro step is applied
// lazily: the stored row is w = g - M c1 with c1 = a eps <A> from the step that
// produced it, and every read reconstructs g = w + M c1.  One step therefore
// reads and writes each cell once:
//   g_j  = w_j + M_j c1
//   A_j  = |v_j|/dx (g_j - g_up,j) + (G_{j+1/2} - G_{j-1/2})/dv
//   w'_j = e g_j - a eps A_j - a J v_j M_j          (= g'_j - M_j a eps <A>)
//   c1'  = a eps <A> = a eps dv sum_j |v_j|/dx (g_j - g_up,j)
// (the velocity part of <A> telescopes to zero with zero-flux ends), and the
// moments of g' follow from running sums of w':
//   Phi = -dv sum v_j w'_j                         (sum_j v_j M_j = 0)
//   |g'|^2 = dv (sum w'^2 + 2 c1' sum w' M + c1'^2 sum M^2).
constexpr int kChunk = 8;  // velocities per software-pipelined chunk
constexpr int kFineBlock = 512;  // threads per fine-sweep workgroup at most

// Uniform per-velocity constants are read through the constant address space
// so that they are scalar loads into SGPRs, not vector registers.
template <typename Real>
using ConstPtr = const __attribute__((address_space(4))) Real *;

template <typename Real>
struct RowCoef {
    Real Ep, Em, e, aeps, aJ;  // E+/dv, E-/dv, exp(-dt/eps^2), a eps, a J
    Real c1, c1n, c1p;         // lazy projection of this row and its neighbours
};

template <typename Real>
struct RowOut {
    Real Sx, phi, ww, wm;      // sum |v|/dx (g - g_up), sum v w', sum w'^2, sum w' M
};

// One kinetic-interface row.  lastlane: last valid lane of the segment; the
// wave-edge upwind neighbours come from the halo rows hnext (v<0 half of row
// p+1) and hprev (v>0 half of row p-1), stored raw (w form).
template <typename Real, int NV>
__device__ __forceinline__ RowOut<Real> row_pass(Real *__restrict__ Wp, int nx, bool valid, bool kin,
                                                 const RowCoef<Real> &c, int lane, int lastlane,
                                                 ConstPtr<Real> vt, const Real *hnext, const Real *hprev,
                                                 Real *hfirst_out, Real *hlast_out)
{
    constexpr int HV = NV / 2;
    RowOut<Real> o{0, 0, 0, 0};
    Real Glo = 0;
    Real cur[kChunk + 1];
#pragma unroll
    for (int t = 0; t <= kChunk; ++t)
        cur[t] = (valid && t < NV) ? Wp[(size_t)t * nx] : Real(0);
#pragma unroll 1
    for (int j0 = 0; j0 < NV; j0 += kChunk) {
        Real nxt[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            const int jj = j0 + kChunk + 1 + t;
            nxt[t] = (valid && jj < NV) ? Wp[(size_t)jj * nx] : Real(0);
        }
        Real gnext = cur[0] + vt[4 * j0 + 1] * c.c1;
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            const int j = j0 + t;
            const Real cx = vt[4 * j], M = vt[4 * j + 1], vM = vt[4 * j + 2], v = vt[4 * j + 3];
            const Real gj = gnext;
            gnext = (j + 1 < NV) ? cur[t + 1] + vt[4 * (j + 1) + 1] * c.c1 : Real(0);
            Real gx;
            if (j < HV) {      // v_j < 0: upwind neighbour is p+1
                const Real h = hnext[j] + M * c.c1n;
                gx = __shfl_down(gj, 1, kWave);
                gx = lane == lastlane ? h : gx;
            } else {           // v_j > 0: upwind neighbour is p-1
                const Real h = hprev[j - HV] + M * c.c1p;
                gx = __shfl_up(gj, 1, kWave);
                gx = lane == 0 ? h : gx;
            }
            const Real ghi = (j < NV - 1) ? c.Ep * gj + c.Em * gnext : Real(0);
            const Real dg = gj - gx;
            const Real gv = ghi - Glo;
            Glo = ghi;
            o.Sx += cx * dg;
            const Real A = cx * dg + gv;
            Real w = c.e * gj - c.aeps * A - c.aJ * vM;
            w = kin ? w : Real(0);
            if (valid && kin) Wp[(size_t)j * nx] = w;
            if (lane == 0 && j < HV) hfirst_out[j] = w;
            if (lane == lastlane && j >= HV) hlast_out[j - HV] = w;
            o.phi += v * w;
            o.ww += w * w;
            o.wm += w * M;
        }
        cur[0] = cur[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) cur[t + 1] = nxt[t];
    }
    return o;
}

// Fine sweep: one workgroup per unit (slice), all fine steps of the slice in
// one launch.  Threads own interfaces/cells p = k*B + t (slab k).
template <typename Real, int NV, int IPTM>
__global__ void __launch_bounds__(kFineBlock) k_fine(const FineUnit *__restrict__ units)
{
    constexpr int HV = NV / 2;
    extern __shared__ __align__(16) unsigned char smem[];

    const FineUnit &U = units[blockIdx.x];
    const FineConst *__restrict__ C = &U.c;
    const int nx = C->nx;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int BS = blockDim.x, NW = BS / kWave;
    const int ipt = (nx + BS - 1) / BS;
    const int nseg = (nx + kWave - 1) / kWave;
    const int nslot = ipt * NW;
    const int flags = C->flags;
    const bool hybrid = flags & STH_HYBRID, field = flags & STH_FIELD, literal = flags & STH_LITERAL_R;
    const long long nsteps = U.nsteps > 0 ? U.nsteps : C->nsteps;
    const double *__restrict__ g_e = C->e_p;
    const double *__restrict__ g_a = C->a_p;
    const double *__restrict__ g_eps = C->eps_p;
    const double *__restrict__ g_epsc = C->eps_c;

    const FineLds L = fine_lds(nx, NV, (int)sizeof(Real), nslot);
    double *s_rho = (double *)(smem + L.rho);
    double *s_jc = (double *)(smem + L.jc);
    double *s_phi = (double *)(smem + L.phi);
    Real *s_nrm = (Real *)(smem + L.nrm);      // [2][nx]
    unsigned char *s_cm = (unsigned char *)(smem + L.cm);
    double *s_tot = (double *)(smem + L.tot);
    double *s_wtot = (double *)(smem + L.wtot);
    double *s_jtot = (double *)(smem + L.jtot);
    double *s_E = (double *)(smem + L.E);

    Real *W = (Real *)U.g_out;                 // [NV][nx] rows
    Real *C1 = W + (size_t)NV * nx;            // [2][nx] lazy projection
    Real *s_halo = (Real *)(smem + L.halo);    // [2 parity][2 side][nseg][HV] halo rows
    // side 0: first row of a segment, v<0 half; side 1: last row, v>0 half
#define HALO(par, side, seg) (s_halo + ((size_t)((par) * 2 + (side)) * nseg + (seg)) * HV)

    Real msq = 0;  // sum_j M_j^2
    for (int j = 0; j < NV; ++j) {
        const Real M = (Real)C->vtab[NV + j];
        msq += M * M;
    }
    // [NV][4] table in the working precision for the row passes
    const ConstPtr<Real> vtr = (ConstPtr<Real>)(sizeof(Real) == 8 ? (const void *)C->vrow64
                                                                 : (const void *)C->vrow32);

    const Real *gin = (const Real *)U.g_in;
    const Real dvR = (Real)C->dv;

    unsigned kinbits = 0, cmbits = 0;          // status of the thread's slabs
    unsigned long long kcount = 0;
    double comp[IPTM];                         // compensation of the density sums

    // ---------------------------------------------------------- prologue
#pragma unroll
    for (int k = 0; k < IPTM; ++k) {
        const int i = k * BS + tid;
        const bool valid = (k < ipt) && (i < nx);
        comp[k] = 0.0;
        if (valid) s_rho[i] = U.rho_in[i];
        kinbits |= 1u << k;
        cmbits |= 1u << k;
        if (valid) {
            Real q = 0;
            const int seg = i / kWave, last = min(kWave - 1, nx - 1 - seg * kWave);
            for (int j = 0; j < NV; ++j) {
                const Real v = gin ? gin[(size_t)j * nx + i] : Real(0);
                W[(size_t)j * nx + i] = v;
                q += v * v;
                if (lane == 0 && j < HV) HALO(0, 0, seg)[j] = v;
                if (lane == last && j >= HV) HALO(0, 1, seg)[j - HV] = v;
            }
            C1[i] = Real(0);
            C1[nx + i] = Real(0);
            s_nrm[i] = (Real)g_eps[i] * (Real)sqrt((double)(q * dvR));
        }
    }
    __syncthreads();

    double incl[IPTM];

    // Wave prefix sums of d_i = (rho_i - rhobar) dx and of d_i (nx - i), whose
    // total is sum_p s_p (for the zero-mean gauge).
    auto macro_scan = [&]() {
        const double rhobar = C->rhobar, dx = C->dx;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            if (k < ipt) {
                const int i = k * BS + tid;
                const bool valid = i < nx;
                const double d = valid ? (s_rho[i] - rhobar) * dx : 0.0;
                incl[k] = wave_incl_scan(d, lane);
                const double tot = __shfl(incl[k], kWave - 1, kWave);
                const double w = wave_sum(valid ? d * (double)(nx - i) : 0.0);
                if (lane == 0) {
                    s_tot[k * NW + wid] = tot;
                    s_wtot[k * NW + wid] = w;
                }
            }
        }
    };
    // Field E_p (Gauss law, zero-mean gauge), flux J_p, and (hybrid) the
    // cell-centred J_i = d1 rho_i - E_i rho_i with E_i = E_p - d_p/2.
    auto macro_field = [&]() {
        const double rhobar = C->rhobar, dx = C->dx, inv_dx = 1.0 / dx;
        const double t = lane < nslot ? s_tot[lane] : 0.0;
        const double ex = wave_incl_scan(t, lane) - t;
        const double Wsum = wave_sum(lane < nslot ? s_wtot[lane] : 0.0);
        const double mean_s = Wsum / (double)nx;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            if (k < ipt) {
                const int i = k * BS + tid;
                const bool valid = i < nx;
                const double pre = __shfl(ex, k * NW + wid, kWave);
                const double E = field ? (pre + incl[k]) - mean_s : 0.0;
                double jsum = 0.0;
                if (valid) {
                    const double r = s_rho[i];
                    s_E[i] = E;
                    if (hybrid) {
                        const double Ec = field ? E - 0.5 * (r - rhobar) * dx : 0.0;
                        const double jc = fd1(s_rho, i, nx) * inv_dx - Ec * r;
                        s_jc[i] = jc;
                        jsum = jc;
                    }
                }
                if (hybrid) {
                    jsum = wave_sum(jsum);
                    if (lane == 0) s_jtot[k * NW + wid] = jsum;
                }
            }
        }
    };
    // Remainder R_i (eq. RemainderBis, Table 1 stencils) and the cell rule;
    // initial = true applies the kinetic-cell rule to every cell.
    auto macro_rule = [&](int par, bool initial) {
        const double rhobar = C->rhobar, dx = C->dx, inv_dx = 1.0 / dx;
        const double inv_dx2 = inv_dx * inv_dx, inv_dx3 = inv_dx2 * inv_dx;
        const double eta0 = C->eta0, delta0 = C->delta0;
        const double mJ = wave_sum(lane < nslot ? s_jtot[lane] : 0.0) / (double)nx;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) {
                const double r = s_rho[i];
                const double jc = s_jc[i];
                const double d1J = fd1(s_jc, i, nx) * inv_dx;
                const double d3J = fd3(s_jc, i, nx) * inv_dx3;
                double R;
                if (field) {
                    const double Ec = s_E[i] - 0.5 * (r - rhobar) * dx;
                    const double d1r = fd1(s_rho, i, nx) * inv_dx;
                    const double d2J = fd2(s_jc, i, nx) * inv_dx2;
                    R = -d3J + Ec * d2J + (2.0 * r - 3.0 * rhobar) * d1J + 2.0 * jc * d1r
                        - d1r * (jc - mJ);
                } else {
                    R = -d3J;
                }
                const double ec = g_epsc[i];
                const double crit = literal ? fabs(R) : ec * ec * fabs(R);
                const double nl = (double)s_nrm[par * nx + wrapi(i - 1, nx)];
                const double nr = (double)s_nrm[par * nx + i];
                const double nmax = nl > nr ? nl : nr;
                int c;
                if (initial || ((cmbits >> k) & 1u)) c = (nmax > delta0) || (crit > eta0);
                else c = crit > eta0;
                cmbits = (cmbits & ~(1u << k)) | ((unsigned)c << k);
                s_cm[i] = (unsigned char)c;
            }
        }
    };
    // Interface status of step n from s_cm; interfaces turning fluid get
    // g' = 0 (row, lazy projection, norm, both halo parities).
    auto apply_status = [&](int par) {
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) {
                const int kn = s_cm[i] | s_cm[wrapi(i + 1, nx)];
                if (((kinbits >> k) & 1u) && !kn) {
                    const int seg = i / kWave, last = min(kWave - 1, nx - 1 - seg * kWave);
                    for (int j = 0; j < NV; ++j) W[(size_t)j * nx + i] = Real(0);
                    C1[i] = Real(0);
                    C1[nx + i] = Real(0);
                    s_nrm[par * nx + i] = Real(0);
                    for (int pp = 0; pp < 2; ++pp) {
                        if (lane == 0)
                            for (int j = 0; j < HV; ++j) HALO(pp, 0, seg)[j] = Real(0);
                        if (lane == last)
                            for (int j = 0; j < HV; ++j) HALO(pp, 1, seg)[j] = Real(0);
                    }
                }
                kinbits = (kinbits & ~(1u << k)) | ((unsigned)kn << k);
            }
        }
    };
    // Conservative density update with the fluxes of the previous step,
    // compensated (Kahan) so that long slices keep the mass to round-off.
    auto density_update = [&]() {
        const double dtdx = C->dt / C->dx;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) {
                const double r = s_rho[i];
                const double y = dtdx * (s_phi[i] - s_phi[wrapi(i - 1, nx)]) - comp[k];
                const double t = r + y;
                comp[k] = (t - r) - y;
                s_rho[i] = t;
            }
        }
    };

    if (hybrid) {
        macro_scan();
        __syncthreads();
        macro_field();
        __syncthreads();
        macro_rule(0, true);
    } else {
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) s_cm[i] = 1;
        }
    }
    __syncthreads();

    // ---------------------------------------------------------- step loop
    for (long long n = 0; n < nsteps; ++n) {
        const int par = (int)(n & 1), npar = par ^ 1;
        // P1: density update with the previous fluxes, interface status.
        if (n > 0) density_update();
        if (hybrid) apply_status(par);
        macro_scan();
        __syncthreads();  // B1
        // P2: field and fluxes.
        macro_field();
        __syncthreads();  // B2
        // P3: phase-space pass of kinetic interfaces, then the cell rule.
        {
            const double dv = C->dv, m2 = C->m2, inv_dx = 1.0 / C->dx;
#pragma unroll 1
            for (int k = 0; k < ipt; ++k) {
                const int i = k * BS + tid;
                const bool valid = i < nx;
                const bool kv = valid && ((kinbits >> k) & 1u);
                kcount += kv ? 1ull : 0ull;
                const int seg = k * NW + wid;
                double E = 0.0, J = 0.0;
                if (valid) {
                    const double r = s_rho[i], rn = s_rho[wrapi(i + 1, nx)];
                    E = s_E[i];
                    J = (rn - r) * inv_dx - E * 0.5 * (r + rn);
                }
                const unsigned long long any = __ballot(kv);
                double Phi = m2 * J;
                Real Nn = 0;
                if (any && seg < nseg) {
                    const int last = min(kWave - 1, nx - 1 - seg * kWave);
                    const int segn = seg + 1 == nseg ? 0 : seg + 1;
                    const int segp = seg == 0 ? nseg - 1 : seg - 1;
                    const Real er = valid ? (Real)g_e[i] : Real(0);
                    const Real ar = valid ? (Real)g_a[i] : Real(0);
                    const Real epsr = valid ? (Real)g_eps[i] : Real(1);
                    RowCoef<Real> c;
                    c.Ep = (Real)(E > 0.0 ? E / dv : 0.0);
                    c.Em = (Real)(E < 0.0 ? E / dv : 0.0);
                    c.e = er;
                    c.aeps = ar * epsr;
                    c.aJ = (Real)((double)ar * J);
                    const Real *C1p = C1 + (size_t)par * nx;
                    c.c1 = valid ? C1p[i] : Real(0);
                    c.c1n = valid ? C1p[wrapi(i + 1, nx)] : Real(0);
                    c.c1p = valid ? C1p[wrapi(i - 1, nx)] : Real(0);
                    const RowOut<Real> o =
                        row_pass<Real, NV>(W + i, nx, valid, kv, c, lane, last, vtr,
                                           HALO(par, 0, segn), HALO(par, 1, segp),
                                           HALO(npar, 0, seg), HALO(npar, 1, seg));
                    if (kv) {
                        const Real c1n = c.aeps * (o.Sx * dvR);
                        C1[(size_t)npar * nx + i] = c1n;
                        Phi = -(double)o.phi * dv;
                        const Real q = o.ww + Real(2) * c1n * o.wm + c1n * c1n * msq;
                        Nn = epsr * (Real)sqrt((double)(q > Real(0) ? q * dvR : Real(0)));
                    } else if (valid) {
                        C1[(size_t)npar * nx + i] = Real(0);
                    }
                } else if (valid) {
                    C1[(size_t)npar * nx + i] = Real(0);
                }
                if (valid) {
                    s_phi[i] = Phi;
                    s_nrm[npar * nx + i] = Nn;
                }
            }
        }
        if (hybrid) macro_rule(par, false);
        __syncthreads();  // B3
    }

    // ---------------------------------------------------------- epilogue
    if (nsteps > 0) density_update();
    const int fpar = (int)(nsteps & 1);
    if (hybrid) apply_status(fpar);
#pragma unroll
    for (int k = 0; k < IPTM; ++k) {
        const int i = k * BS + tid;
        if (k < ipt && i < nx) {
            U.rho_out[i] = s_rho[i];
            if (U.mask_out) U.mask_out[i] = hybrid ? (int)((cmbits >> k) & 1u) : 1;
            const Real c1 = C1[(size_t)fpar * nx + i];
            if (c1 != Real(0))
                for (int j = 0; j < NV; ++j) W[(size_t)j * nx + i] += vtr[4 * j + 1] * c1;
            C1[i] = Real(0);
            C1[nx + i] = Real(0);
        }
    }
    if (U.kin) {
        const unsigned long long tot = wave_sum(kcount);
        if (lane == 0) atomicAdd(U.kin, tot);
    }
#undef HALO
}

// Launch shape of a fine-sweep class: one workgroup per unit, up to 1024
// threads, interfaces distributed over at most kMaxSlabs slabs.
FineShape fine_shape(int prec, int nx, int nv, int force_stream, int force_block)
{
    (void)force_stream;
    FineShape s{};
    s.prec = prec;
    s.nv = nv;
    s.stream = 1;
    const int realsz = prec == 0 ? 8 : 4;
    int nxr = ((nx + kWave - 1) / kWave) * kWave;
    int b = force_block > 0 ? force_block : kFineBlock;
    if (b > kFineBlock) b = kFineBlock;
    if (b > nxr) b = nxr;
    s.block = b;
    s.ipt = (nx + b - 1) / b;
    const int nslot = s.ipt * (s.block / kWave);
    s.lds = fine_lds(nx, nv, realsz, nslot).total;
    return s;
}

template <typename Real, int NV, int IPT>
static hipError_t launch_one(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    auto kern = k_fine<Real, NV, IPT>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)s.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n), dim3(s.block), s.lds, st, d);
    return hipGetLastError();
}

template <typename Real, int NV>
static hipError_t launch_nv(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    switch (s.ipt) {
        case 1: return launch_one<Real, NV, 1>(s, d, n, st);
        case 2: return launch_one<Real, NV, 2>(s, d, n, st);
        case 3:
        case 4: return launch_one<Real, NV, 4>(s, d, n, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fine(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (s.ipt > kMaxSlabs || s.block % kWave != 0) return hipErrorInvalidValue;
    if (s.prec == 0) {
        switch (s.nv) {
            case 16: return launch_nv<double, 16>(s, d, n, st);
            case 32: return launch_nv<double, 32>(s, d, n, st);
            case 64: return launch_nv<double, 64>(s, d, n, st);
            case 128: return launch_nv<double, 128>(s, d, n, st);
        }
    } else {
        switch (s.nv) {
            case 16: return launch_nv<float, 16>(s, d, n, st);
            case 32: return launch_nv<float, 32>(s, d, n, st);
            case 64: return launch_nv<float, 64>(s, d, n, st);
            case 128: return launch_nv<float, 128>(s, d, n, st);
        }
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------ block helpers
// Poisson on one workgroup: E[p] from rho (global or LDS), zero-mean gauge.
// Sequential prefix sum by thread 0 (the macro quantities of the non-hot
// kernels are O(nx)).
__device__ void block_poisson(const double *rho, double *E, int nx, double dx, double rhobar,
                              bool field)
{
    if (!field) {
        for (int p = threadIdx.x; p < nx; p += blockDim.x) E[p] = 0.0;
        __syncthreads();
        return;
    }
    __shared__ double s_mean;
    if (threadIdx.x == 0) {
        double s = 0.0, m = 0.0;
        for (int p = 0; p < nx; ++p) {
            s += (rho[p] - rhobar) * dx;
            E[p] = s;
            m += s;
        }
        s_mean = m / (double)nx;
    }
    __syncthreads();
    const double m = s_mean;
    for (int p = threadIdx.x; p < nx; p += blockDim.x) E[p] -= m;
    __syncthreads();
}

__device__ double block_sum(double x)
{
    __shared__ double s_part[16];
    x = wave_sum(x);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) s_part[wid] = x;
    __syncthreads();
    const int nw = (blockDim.x + kWave - 1) / kWave;
    double t = lane < nw ? s_part[lane] : 0.0;
    t = wave_sum(t);
    return t;
}

__device__ double block_max(double x)
{
    __shared__ double s_part[16];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double y = __shfl_xor(x, off, kWave);
        x = (y > x || y != y) ? y : x;
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) s_part[wid] = x;
    __syncthreads();
    const int nw = (blockDim.x + kWave - 1) / kWave;
    double t = lane < nw ? s_part[lane] : 0.0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double y = __shfl_xor(t, off, kWave);
        t = (y > t || y != y) ? y : t;
    }
    return t;
}

// ------------------------------------------------------------ lifting
// Lifting L^L (Definition 1) at interfaces from the averaged density, with
// the Chapman-Enskog terms (g' units, K = d1 J - E J):
//   h1 = -v M J, h2 = (v^2 - m2) M K,
//   h3 = v M [dtJ - (v^2 - m2) d1 K - (2 + m2 - v^2) E K],
//   dtJ = d2 J - (J - mean J) rho~ - E d1 J  (field terms vanish without field).
// Workspace: 4*nx doubles of dynamic LDS.
template <typename Real>
__global__ void __launch_bounds__(1024) k_lift(const LiftJob *__restrict__ jobs)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const LiftJob J = jobs[blockIdx.x];
    const FineConst *C = J.pc;
    const int nx = C->nx, nv = C->nv;
    const bool field = C->flags & STH_FIELD;
    const double dx = C->dx, inv_dx = 1.0 / dx;
    double *s_rho = (double *)smem;
    double *s_E = s_rho + nx;
    double *s_J = s_E + nx;
    double *s_K = s_J + nx;
    for (int p = threadIdx.x; p < nx; p += blockDim.x) s_rho[p] = J.rho[p];
    __syncthreads();
    block_poisson(s_rho, s_E, nx, dx, C->rhobar, field);
    double part = 0.0;
    for (int p = threadIdx.x; p < nx; p += blockDim.x) {
        const double rn = s_rho[wrapi(p + 1, nx)];
        s_J[p] = (rn - s_rho[p]) * inv_dx - s_E[p] * 0.5 * (s_rho[p] + rn);
        part += s_J[p];
    }
    const double meanJ = block_sum(part) / (double)nx;
    __syncthreads();
    for (int p = threadIdx.x; p < nx; p += blockDim.x) s_K[p] = fd1(s_J, p, nx) * inv_dx - s_E[p] * s_J[p];
    __syncthreads();
    const double m2 = C->m2;
    const double *vt = C->vtab;
    Real *g = (Real *)J.g;
    for (int p = threadIdx.x; p < nx; p += blockDim.x) {
        const double Jp = s_J[p], Kp = s_K[p], Ep = s_E[p];
        const double d1J = fd1(s_J, p, nx) * inv_dx;
        const double d2J = fd2(s_J, p, nx) * inv_dx * inv_dx;
        const double d1K = fd1(s_K, p, nx) * inv_dx;
        const double rt = 0.5 * (s_rho[p] + s_rho[wrapi(p + 1, nx)]);
        const double dtJ = d2J - Ep * d1J - (field ? (Jp - meanJ) * rt : 0.0);
        const double eps = C->eps_p[p];
        for (int j = 0; j < nv; ++j) {
            const double v = vt[3 * nv + j], M = vt[nv + j], w = v * v - m2;
            double val = -v * M * Jp;
            if (J.lift_order >= 2) val += eps * (w * M * Kp);
            if (J.lift_order >= 3) val += eps * eps * (v * M * (dtJ - w * d1K - (2.0 + m2 - v * v) * Ep * Kp));
            g[(size_t)j * nx + p] = (Real)val;
        }
    }
}

hipError_t launch_lift(int prec, const LiftJob *d_jobs, int njobs, int nx, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * 4 * nx;
    int b = ((nx + kWave - 1) / kWave) * kWave;
    if (b > 1024) b = 1024;
    if (prec == 0) {
        hipError_t e = hipFuncSetAttribute((const void *)k_lift<double>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lift<double>, dim3(njobs), dim3(b), lds, st, d_jobs);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)k_lift<float>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lift<float>, dim3(njobs), dim3(b), lds, st, d_jobs);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ coarse propagator
// One backward-Euler step of the drift-diffusion limit with the field frozen
// at the slice start, cyclic tridiagonal solve (Thomas with the
// Sherman-Morrison correction for the periodic corner), then the
// conservative form rho_in + dtG L_E(solution).  Workspace in LDS: 8*nx.
__device__ void coarse_step_block(const FineConst *C, const double *rin, double *rout, double dtG,
                                  double *w)
{
    const int nx = C->nx;
    const double dx = C->dx, m2 = C->m2;
    const bool field = C->flags & STH_FIELD;
    double *E = w, *a = w + nx, *b = w + 2 * nx, *c = w + 3 * nx, *x = w + 4 * nx;
    double *z = w + 5 * nx, *cp = w + 6 * nx, *dp = w + 7 * nx;
    block_poisson(rin, E, nx, dx, C->rhobar, field);
    const double alpha = m2 * dtG / (dx * dx), beta = m2 * dtG / (2.0 * dx);
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double Ew = E[wrapi(i - 1, nx)], Ee = E[i];
        a[i] = -alpha - beta * Ew;
        b[i] = 1.0 + 2.0 * alpha + beta * (Ee - Ew);
        c[i] = -alpha + beta * Ee;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double gamma = -b[0];
        const double b0 = b[0] - gamma;
        const double bl = b[nx - 1] - a[0] * c[nx - 1] / gamma;
        // Thomas on the modified matrix for two right-hand sides (rho, u)
        double m = b0;
        cp[0] = c[0] / m;
        dp[0] = rin[0] / m;
        z[0] = gamma / m;  // forward sweep of u = (gamma, 0, ..., 0, c_{n-1})
        for (int i = 1; i < nx; ++i) {
            const double bi = (i == nx - 1) ? bl : b[i];
            m = bi - a[i] * cp[i - 1];
            cp[i] = c[i] / m;
            dp[i] = (rin[i] - a[i] * dp[i - 1]) / m;
            const double ui = (i == nx - 1) ? c[nx - 1] : 0.0;
            z[i] = (ui - a[i] * z[i - 1]) / m;
        }
        x[nx - 1] = dp[nx - 1];
        for (int i = nx - 2; i >= 0; --i) {
            x[i] = dp[i] - cp[i] * x[i + 1];
            z[i] = z[i] - cp[i] * z[i + 1];
        }
        const double fact = (x[0] + a[0] * x[nx - 1] / gamma) / (1.0 + z[0] + a[0] * z[nx - 1] / gamma);
        for (int i = 0; i < nx; ++i) x[i] -= fact * z[i];
    }
    __syncthreads();
    // conservative form: flux of the solution, then rho_in + dtG m2 dJ/dx
    for (int p = threadIdx.x; p < nx; p += blockDim.x) {
        const int q = wrapi(p + 1, nx);
        cp[p] = (x[q] - x[p]) / dx - E[p] * 0.5 * (x[p] + x[q]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nx; i += blockDim.x)
        rout[i] = rin[i] + dtG * m2 * (cp[i] - cp[wrapi(i - 1, nx)]) / dx;
    __syncthreads();
}

__global__ void __launch_bounds__(1024) k_coarse(CoarseJob J)
{
    double *work = J.work;
    const int nx = J.pc->nx;
    const size_t slab = (size_t)nx;
    double *gn = work + 8 * slab;
    if (J.mode == 0) {
        for (int n = 1; n <= J.N; ++n) {
            coarse_step_block(J.pc, J.U + (n - 1) * slab, J.U + n * slab, J.dtG, work);
            for (int i = threadIdx.x; i < nx; i += blockDim.x) J.Gc[n * slab + i] = J.U[n * slab + i];
            __syncthreads();
        }
        return;
    }
    const int k = J.k;
    double e = 0.0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double nv = J.Fv[(k + 1) * slab + i];
        const double d = fabs(nv - J.U[(k + 1) * slab + i]);
        e = (d > e || d != d) ? d : e;
        J.U[(k + 1) * slab + i] = nv;
    }
    __syncthreads();
    for (int n = k + 2; n <= J.N; ++n) {
        coarse_step_block(J.pc, J.U + (n - 1) * slab, gn, J.dtG, work);
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            const double g = gn[i];
            const double nv = g + (J.Fv[n * slab + i] - J.Gc[n * slab + i]);
            const double d = fabs(nv - J.U[n * slab + i]);
            e = (d > e || d != d) ? d : e;
            J.U[n * slab + i] = nv;
            J.Gc[n * slab + i] = g;
        }
        __syncthreads();
    }
    e = block_max(e);
    if (threadIdx.x == 0) J.err[0] = e;
}

hipError_t launch_coarse(const CoarseJob &job, int nx, hipStream_t st)
{
    int b = ((nx + kWave - 1) / kWave) * kWave;
    if (b > 1024) b = 1024;
    hipLaunchKernelGGL(k_coarse, dim3(1), dim3(b), 0, st, job);
    return hipGetLastError();
}

// ------------------------------------------------------------ diagnostics
// E, J at interfaces, Phi = -<v g>, N = eps ||g||_2, remainder R at cells and
// the kinetic-cell rule, for one state (rho, g).  LDS: 3*nx doubles.
template <typename Real>
__global__ void __launch_bounds__(1024) k_diag(DiagJob J)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const FineConst *C = J.pc;
    const int nx = C->nx, nv = C->nv;
    const bool field = C->flags & STH_FIELD, literal = C->flags & STH_LITERAL_R;
    const double dx = C->dx, dv = C->dv, inv_dx = 1.0 / dx, rhobar = C->rhobar;
    double *s_rho = (double *)smem, *s_E = s_rho + nx, *s_jc = s_E + nx;
    double *oE = J.out, *oJ = J.out + nx, *oPhi = J.out + 2 * nx, *oN = J.out + 3 * nx, *oR = J.out + 4 * nx;
    const Real *g = (const Real *)J.g;
    const double *vt = C->vtab;
    for (int p = threadIdx.x; p < nx; p += blockDim.x) s_rho[p] = J.rho[p];
    __syncthreads();
    block_poisson(s_rho, s_E, nx, dx, rhobar, field);
    double part = 0.0;
    for (int p = threadIdx.x; p < nx; p += blockDim.x) {
        const double rn = s_rho[wrapi(p + 1, nx)];
        oE[p] = s_E[p];
        oJ[p] = (rn - s_rho[p]) * inv_dx - s_E[p] * 0.5 * (s_rho[p] + rn);
        double ph = 0.0, q = 0.0;
        if (g) {
            for (int j = 0; j < nv; ++j) {
                const double gv = (double)g[(size_t)j * nx + p];
                ph += vt[3 * nv + j] * gv * dv;
                q += gv * gv * dv;
            }
        }
        oPhi[p] = -ph;
        oN[p] = C->eps_p[p] * sqrt(q);
        const double ec = field ? 0.5 * (s_E[wrapi(p - 1, nx)] + s_E[p]) : 0.0;
        s_jc[p] = fd1(s_rho, p, nx) * inv_dx - ec * s_rho[p];
        part += s_jc[p];
    }
    const double meanJ = block_sum(part) / (double)nx;
    __syncthreads();
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double d1r = fd1(s_rho, i, nx) * inv_dx;
        const double d1J = fd1(s_jc, i, nx) * inv_dx;
        const double d3J = fd3(s_jc, i, nx) * inv_dx * inv_dx * inv_dx;
        double R;
        if (field) {
            const double ec = 0.5 * (s_E[wrapi(i - 1, nx)] + s_E[i]);
            const double d2J = fd2(s_jc, i, nx) * inv_dx * inv_dx;
            R = -d3J + ec * d2J + (2.0 * s_rho[i] - 3.0 * rhobar) * d1J + 2.0 * s_jc[i] * d1r
                - d1r * (s_jc[i] - meanJ);
        } else {
            R = -d3J;
        }
        oR[i] = R;
        const double eps = C->eps_c[i];
        const double crit = literal ? fabs(R) : eps * eps * fabs(R);
        const double nl = oN[wrapi(i - 1, nx)], nr = oN[i];
        J.mask[i] = ((nl > nr ? nl : nr) > C->delta0) || (crit > C->eta0);
    }
}

hipError_t launch_diag(int prec, const DiagJob &job, int nx, hipStream_t st)
{
    const size_t lds = sizeof(double) * 3 * nx;
    int b = ((nx + kWave - 1) / kWave) * kWave;
    if (b > 1024) b = 1024;
    if (prec == 0) {
        hipError_t e = hipFuncSetAttribute((const void *)k_diag<double>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_diag<double>, dim3(1), dim3(b), lds, st, job);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)k_diag<float>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_diag<float>, dim3(1), dim3(b), lds, st, job);
    }
    return hipGetLastError();
}

}  // namespace sth
