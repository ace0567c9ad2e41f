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
// and the x-upwind neighbour is one lane away (DPP shift of the wavefront;
// the two wave edges read a double-buffered LDS halo).  The perturbation is
// streamed each step from a v-major global buffer that stays resident in the
// XCD's L2 (coalesced: lanes are consecutive interfaces), read and written
// once per cell and step.  The macroscopic quantities (rho, E, J, Phi,
// norms, status) live in LDS.  Three barriers per fine step (see k_fine).
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

// DPP move of a double (both halves with the same control); lanes without a
// source or outside row_mask read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Inclusive prefix sum over the 64 lanes with DPP: row_shr 1, 2, 4, 8 inside
// each row of 16 lanes, then row_bcast:15 and row_bcast:31 across rows.
__device__ __forceinline__ double wave_scan_f64(double x)
{
    x += dpp_f64<0x111, 0xf>(x);
    x += dpp_f64<0x112, 0xf>(x);
    x += dpp_f64<0x114, 0xf>(x);
    x += dpp_f64<0x118, 0xf>(x);
    x += dpp_f64<0x142, 0xa>(x);
    x += dpp_f64<0x143, 0xc>(x);
    return x;
}

// Value of lane l (wavefront-uniform l) in every lane.
__device__ __forceinline__ double lane_value(double x, int l)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// DPP move of a double whose lanes outside row_mask are left undefined (no
// initialisation of the destination): for reductions that read one lane.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64_u(double x)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)b, CTRL, ROWMASK, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64_z(double x);

// Sum over the 64 lanes, in every lane: zero-filling row shifts give each
// row's sum in its lane 15, the row broadcasts add the rows below into lane
// 63 (the other lanes end undefined), which is read back.
__device__ __forceinline__ double wave_total_f64(double x)
{
    x += dpp_f64_z<0x111>(x);
    x += dpp_f64_z<0x112>(x);
    x += dpp_f64_z<0x114>(x);
    x += dpp_f64_z<0x118>(x);
    x += dpp_f64_u<0x142, 0xa>(x);
    x += dpp_f64_u<0x143, 0xc>(x);
    return lane_value(x, kWave - 1);
}

// Two inclusive prefix sums at once (independent chains interleave and fill
// each other's DPP wait states); the row shifts zero-fill (bound_ctrl).
template <int CTRL>
__device__ __forceinline__ double dpp_f64_z(double x)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ void wave_scan2_f64(double &a, double &b)
{
    a += dpp_f64_z<0x111>(a);
    b += dpp_f64_z<0x111>(b);
    a += dpp_f64_z<0x112>(a);
    b += dpp_f64_z<0x112>(b);
    a += dpp_f64_z<0x114>(a);
    b += dpp_f64_z<0x114>(b);
    a += dpp_f64_z<0x118>(a);
    b += dpp_f64_z<0x118>(b);
    a += dpp_f64<0x142, 0xa>(a);
    b += dpp_f64<0x142, 0xa>(b);
    a += dpp_f64<0x143, 0xc>(a);
    b += dpp_f64<0x143, 0xc>(b);
}

// Returns x unchanged but hides its value from the optimiser: values derived
// from it inside a loop are recomputed there instead of being hoisted into
// registers held across the loop.
__device__ __forceinline__ int opaque_v(int x)
{
    asm volatile("" : "+v"(x));
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

// The same stencils on an array with periodic ghost cells: f points at the
// centre, f[-3..3] are valid.
__device__ __forceinline__ double fd1g(const double *f)
{
    return (-1.0 / 60.0) * f[-3] + (3.0 / 20.0) * f[-2] + (-3.0 / 4.0) * f[-1] + (3.0 / 4.0) * f[1]
           + (-3.0 / 20.0) * f[2] + (1.0 / 60.0) * f[3];
}
__device__ __forceinline__ double fd2g(const double *f)
{
    return (1.0 / 90.0) * f[-3] + (-3.0 / 20.0) * f[-2] + (3.0 / 2.0) * f[-1] + (-49.0 / 18.0) * f[0]
           + (3.0 / 2.0) * f[1] + (-3.0 / 20.0) * f[2] + (1.0 / 90.0) * f[3];
}
__device__ __forceinline__ double fd3g(const double *f)
{
    return (1.0 / 8.0) * f[-3] + (-1.0) * f[-2] + (13.0 / 8.0) * f[-1] + (-13.0 / 8.0) * f[1] + (1.0) * f[2]
           + (-1.0 / 8.0) * f[3];
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS layout of the fine kernel.  Same function on host (sizing) and device.
struct FineLds {
    size_t rho, jc, phi, phiJ, E, nrm, cm, crit, tot, wtot, jtot, dummy, c1, halo, total;
};
// res: the resident kernel, which also keeps the lazy projection c1[2][nx]
// and the halo rows [2 parity][2 side][nseg][nv/2] in LDS.
__host__ __device__ inline FineLds fine_lds(int nx, int nv, int realsz, int nslot, bool res)
{
    FineLds L;
    size_t o = 0;
    // periodic ghost cells: rho, jc [-3, nx+3); phi [-1, nx); nrm [-1, nx];
    // cm (per parity) and crit [0, nx]
    L.rho = o;  o = align16(o + sizeof(double) * (nx + 6));
    L.jc = o;   o = align16(o + sizeof(double) * (nx + 6));
    L.phi = o;  o = align16(o + sizeof(double) * (nx + 1));
    L.phiJ = o; o = align16(o + sizeof(double) * (nx + 1));
    L.E = o;    o = align16(o + sizeof(double) * nx);
    L.nrm = o;  o = align16(o + (size_t)realsz * (nx + 2));
    L.cm = o;   o = align16(o + sizeof(unsigned char) * 2 * (nx + 1));
    L.crit = o; o = align16(o + sizeof(unsigned char) * (nx + 1));
    L.tot = o;  o = align16(o + sizeof(double) * nslot);
    L.wtot = o; o = align16(o + sizeof(double) * nslot);
    L.jtot = o; o = align16(o + sizeof(double) * nslot);
    L.dummy = o; o = align16(o + (sizeof(double) + 1) * kWave);  // per-lane sink of ghost writes
    L.c1 = o;   if (res) o = align16(o + (size_t)realsz * 2 * nx);
    L.halo = o; if (res) o = align16(o + (size_t)realsz * 2 * 2 * ((nx + kWave - 1) / kWave) * (nv / 2));
    L.total = o;
    return L;
}


// ------------------------------------------------------------ fine sweep
// Row state.  A unit's perturbation lives in a v-major global buffer
// W[j][p] with rows padded to a multiple of the wavefront (lanes =
// consecutive interfaces, so every row access is one coalesced, unmasked
// load or store), followed by C1[2][p] and the halo rows.  The projection of
// the micro-macro step is applied lazily: the stored row is w = g - M c1 with
// c1 = a eps <A> from the step that produced it, and every read reconstructs
// g = w + M c1.  One step therefore reads and writes each cell once:
//   g_j  = w_j + M_j c1
//   A_j  = |v_j|/dx (g_j - g_up,j) + (G_{j+1/2} - G_{j-1/2})/dv
//   w'_j = e g_j - a eps A_j - a J v_j M_j          (= g'_j - M_j a eps <A>)
//   c1'  = a eps <A> = a eps dv sum_j A_j
// (the velocity part of <A> telescopes to zero with zero-flux ends).  The
// same pass yields the flux of g' and the norm of g:
//   Phi = -dv sum v_j w'_j   (sum_j v_j M_j = 0),   |g|^2 = dv sum g_j^2.
// Interfaces that are not kinetic run the same pass with e = a = 0, which
// keeps their rows at zero without a branch.  The upwind neighbour in x is
// one lane away; the wavefront's edge lanes read it from the halo rows
// H[parity][side][segment][HV] (side 0: v<0 half of a segment's first
// interface, side 1: v>0 half of its last), double-buffered by step parity
// and kept in global memory, so that the velocity loop touches no LDS.

// Uniform per-velocity constants are read through the constant address space
// so that they are scalar loads into SGPRs, not vector registers.
template <typename Real>
using ConstPtr = const __attribute__((address_space(4))) Real *;
// Global memory pointer (global, not flat, loads and stores).
template <typename Real>
using GlobPtr = __attribute__((address_space(1))) Real *;

// Whole-wavefront shifts by one lane (DPP wave_shl:1 / wave_shr:1): lane l
// gets x of lane l+1 (from_next_or) or l-1 (from_prev_or); the lane without
// a source keeps old.
__device__ __forceinline__ int dpp_next_or(int old, int x) { return __builtin_amdgcn_update_dpp(old, x, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_prev_or(int old, int x) { return __builtin_amdgcn_update_dpp(old, x, 0x138, 0xf, 0xf, false); }

__device__ __forceinline__ float from_next_or(float old, float x)
{
    return __int_as_float(dpp_next_or(__float_as_int(old), __float_as_int(x)));
}
__device__ __forceinline__ float from_prev_or(float old, float x)
{
    return __int_as_float(dpp_prev_or(__float_as_int(old), __float_as_int(x)));
}
__device__ __forceinline__ double from_next_or(double old, double x)
{
    const long long b = __double_as_longlong(x), a = __double_as_longlong(old);
    const unsigned lo = (unsigned)dpp_next_or((int)a, (int)b);
    const unsigned hi = (unsigned)dpp_next_or((int)(a >> 32), (int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double from_prev_or(double old, double x)
{
    const long long b = __double_as_longlong(x), a = __double_as_longlong(old);
    const unsigned lo = (unsigned)dpp_prev_or((int)a, (int)b);
    const unsigned hi = (unsigned)dpp_prev_or((int)(a >> 32), (int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Unit slot storage is addressed through a buffer resource: wavefront-
// uniform base and row offset (scalar registers) plus a per-lane byte offset
// that stays fixed over a row pass, so a row access costs no vector address
// arithmetic.
constexpr int kBufferFlags = 0x00020000;  // raw buffer, gfx9 family descriptor word 3

template <typename Real>
__device__ __forceinline__ Real buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(double x, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(float x, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, 0);
}

// Returns p unchanged but hides its value from the optimiser, so that loads
// through it stay inside the step loop instead of being hoisted (the hoisted
// per-velocity constants would not fit in scalar registers).
template <typename T>
__device__ __forceinline__ T opaque(T p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// Pins a running sum in its register at this point of the program: the
// compiler may otherwise sink a whole chain of accumulations to the point
// where the sum is used, keeping every term alive until then.
__device__ __forceinline__ void keep(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void keep(float &x) { asm volatile("" : "+v"(x)); }

template <typename Real>
struct RowCoef {
    Real Ep, Em, e, a, aeps, aJ;  // E+/dv, E-/dv, exp(-dt/eps^2), a = -expm1(-dt/eps^2), a eps,
                                  // a J (all but E+-/dv zero if not kinetic)
    Real c1, c1n, c1p;            // lazy projection of this interface and of p+1, p-1
};

// Running sums of a row pass.  They are kept in FP64 in both precisions:
// in FP64 each velocity pair is added to them; in FP32 bulk the pairs of a
// group of at most four are summed in FP32 and the group sums accumulate in
// FP64 (this bounds the rounding of the flux, the projection and the norm
// over long slices, at one conversion per sum and group).
template <typename Real>
struct RowOut {
    double Sx, phi, gg;        // sum A, sum sign(v)|v|/dx w', sum g^2
};

// FP32-bulk sums of the current group of pairs.
template <typename Real>
struct PairAcc {
    Real sx, ph, gg;
};

template <typename Real>
__device__ __forceinline__ void acc_pair(RowOut<Real> &o, PairAcc<Real> &a, Real Aj, Real Am, Real cx, Real wj,
                                         Real wm, Real gj, Real gm)
{
    if constexpr (sizeof(Real) == 8) {
        o.Sx += (double)(Aj + Am);
        o.phi += (double)(cx * (wm - wj));
        o.gg += (double)(gj * gj + gm * gm);
        keep(o.Sx);
        keep(o.phi);
        keep(o.gg);
    } else {
        a.sx += Aj + Am;
        a.ph += cx * (wm - wj);
        a.gg = __builtin_fmaf(gm, gm, __builtin_fmaf(gj, gj, a.gg));
        keep(a.sx);
        keep(a.ph);
        keep(a.gg);
    }
}

// Relaxation with the source for a mirror pair, w' = e g - a eps A - a J v M
// (v M of the pair's v<0 member; its mirror has the opposite sign).  FP32
// bulk computes it as an increment, w' = g + d with d = -(a g + a eps A +
// a J v M) formed first: where dt/eps^2 is below the FP32 resolution, e
// rounds to 1 or to 1 - 2^-24 and e g would relax g at a wrong rate or not at
// all, while a keeps its 24 bits and the one rounding of g + d is unbiased.
// FP64 keeps the printed form (e exact to 1e-16).
template <typename Real>
__device__ __forceinline__ void relax_pair(const RowCoef<Real> &c, Real gj, Real gm, Real Aj, Real Am, Real vM,
                                           Real &wj, Real &wm)
{
    if constexpr (sizeof(Real) == 4) {
        const Real sJ = c.aJ * vM;
        const Real dj = __builtin_fmaf(-c.a, gj, __builtin_fmaf(-c.aeps, Aj, -sJ));
        const Real dm = __builtin_fmaf(-c.a, gm, __builtin_fmaf(-c.aeps, Am, sJ));
        wj = gj + dj;
        wm = gm + dm;
    } else {
        wj = c.e * gj - c.aeps * Aj - c.aJ * vM;
        wm = c.e * gm - c.aeps * Am + c.aJ * vM;
    }
}

// Lazy-projection read g = w + M c1: one fused multiply-add per value in FP32
// bulk (the compiler would otherwise share M c1 between the two members of a
// pair and round it); FP64 keeps the compiler's form.
template <typename Real>
__device__ __forceinline__ Real recon(Real w, Real M, Real c1)
{
    if constexpr (sizeof(Real) == 4) return __builtin_fmaf(M, c1, w);
    else return w + M * c1;
}

// End of a group of pairs (FP32 bulk): its sums join the FP64 ones.
template <typename Real>
__device__ __forceinline__ void acc_flush(RowOut<Real> &o, PairAcc<Real> &a)
{
    if constexpr (sizeof(Real) == 4) {
        o.Sx += (double)a.sx;
        o.phi += (double)a.ph;
        o.gg += (double)a.gg;
        a.sx = a.ph = a.gg = Real(0);
        keep(o.Sx);
        keep(o.phi);
        keep(o.gg);
    }
}

// Byte offsets of one row pass in the unit slot (wavefront-uniform except vo).
struct RowIO {
    __amdgpu_buffer_rsrc_t rs;  // the unit slot
    unsigned vo;                // lane: byte offset of its interface in a row
    unsigned rowb;              // bytes per row
    unsigned hn, hp;            // halos read: v<0 half of interface p+1 (next segment's first),
                                // v>0 half of interface p-1 (previous segment's last)
    unsigned hno, hpo;          // halos written: this segment's first (v<0) and last (v>0) interface
};

// Software-pipelined chunk of velocity pairs (j, NV-1-j): rows and halo
// values of CH pairs.  Chunk length per velocity grid: an even number of
// chunks per half, and a rolled chunk loop wherever the grid has more than
// two chunks (a straight run of chunks lets the compiler stretch live
// ranges across them).
// FP32 rows take half the registers, so their chunks are twice as long
// (twice the loads in flight) on the wider grids, except in workgroups of
// kWideBlock threads, whose lanes have 128 registers at most.
template <typename Real, int NV, int BLK>
constexpr int pair_chunk_len()
{
    return NV == 32 ? 2 : (NV >= 64 && sizeof(Real) == 4 && BLK <= kFineBlock ? 8 : 4);
}
template <typename Real, int CH>
struct PairBuf {
    Real wn[CH], wp[CH], hn[CH], hp[CH];
};

// One chunk of velocity pairs t0.. of a row.  A pair couples v_j < 0 (j = t,
// upwind neighbour p+1) with its mirror v_m = -v_j (m = NV-1-t, upwind
// neighbour p-1); both share |v|/dx, M and |v M|, so one row of the table
// serves two velocities.  The v<0 half runs up from j = 0 carrying the
// G flux of its lower face, the v>0 half runs down from m = NV-1 carrying
// that of its upper face; they meet at the middle pair (LAST).  On entry
// cur holds the stored rows and halos of this chunk and gj, gm the
// reconstructed g of its first pair; the chunk loads the next chunk into nxt
// (ping-pong, no register copies).  The wavefront's edge lanes keep the halo
// value in the DPP shift (no source lane); in a ragged segment (RAGGED) the
// last valid lane is not a wavefront edge and selects its halo explicitly.
template <typename Real, int NV, bool LAST, bool RAGGED, int CH>
__device__ __forceinline__ void pair_chunk(int t0, const RowIO &io, const RowCoef<Real> &c, bool first, bool last,
                                           ConstPtr<Real> vt, const PairBuf<Real, CH> &cur, PairBuf<Real, CH> &nxt,
                                           Real &gj, Real &gm, Real &Glo, Real &Ghi, RowOut<Real> &o)
{
    constexpr int HV = NV / 2;
    constexpr unsigned R = sizeof(Real);
    // keep the scheduler from hoisting later chunks' loads into this one
    __builtin_amdgcn_sched_barrier(0);
    PairAcc<Real> a{0, 0, 0};
    if (!LAST) {
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int t = t0 + CH + u;
            nxt.wn[u] = buf_load<Real>(io.rs, io.vo, (unsigned)t * io.rowb);
            nxt.wp[u] = buf_load<Real>(io.rs, io.vo, (unsigned)(NV - 1 - t) * io.rowb);
            nxt.hn[u] = buf_load<Real>(io.rs, 0u, io.hn + (unsigned)t * R);
            nxt.hp[u] = buf_load<Real>(io.rs, 0u, io.hp + (unsigned)(HV - 1 - t) * R);
        }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int t = t0 + u, j = t, m = NV - 1 - t;
        const Real cx = vt[4 * t], M = vt[4 * t + 1], vM = vt[4 * t + 2], Mn = vt[4 * t + 3];
        Real gjn, gmn;  // g_{j+1}, g_{m-1}
        if (u + 1 < CH) {
            gjn = recon(cur.wn[u + 1], Mn, c.c1);
            gmn = recon(cur.wp[u + 1], Mn, c.c1);
        } else if (!LAST) {
            gjn = recon(nxt.wn[0], Mn, c.c1);
            gmn = recon(nxt.wp[0], Mn, c.c1);
        } else {  // middle pair: rows HV-1 and HV are each other's neighbours
            gjn = gm;
            gmn = gj;
        }
        // upwind neighbours in x
        const Real hj = cur.hn[u] + M * c.c1n;
        Real gxj = from_next_or(hj, gj);
        if (RAGGED) gxj = last ? hj : gxj;
        const Real hm = cur.hp[u] + M * c.c1p;
        const Real gxm = from_prev_or(hm, gm);
        // G fluxes in v: G_{j+1/2} and G_{m-1/2} (the same face at the middle)
        const Real Gj = c.Ep * gj + c.Em * gjn;
        const Real Gm = (LAST && u == CH - 1) ? Gj : c.Ep * gmn + c.Em * gm;
        const Real gvj = Gj - Glo, gvm = Ghi - Gm;
        Glo = Gj;
        Ghi = Gm;
        const Real dgj = gj - gxj, dgm = gm - gxm;
        const Real Aj = cx * dgj + gvj, Am = cx * dgm + gvm;
        Real wj, wm;
        relax_pair(c, gj, gm, Aj, Am, vM, wj, wm);
        buf_store(wj, io.rs, io.vo, (unsigned)j * io.rowb);
        buf_store(wm, io.rs, io.vo, (unsigned)m * io.rowb);
        if (first) buf_store(wj, io.rs, 0u, io.hno + (unsigned)j * R);
        if (last) buf_store(wm, io.rs, 0u, io.hpo + (unsigned)(m - HV) * R);
        acc_pair(o, a, Aj, Am, cx, wj, wm, gj, gm);
        if ((u & 3) == 3 || u == CH - 1) acc_flush(o, a);
        gj = gjn;
        gm = gmn;
    }
}

// One row (interface) of a wavefront segment: every velocity pair, chunk by
// chunk.  first/last: the lane is the first / last valid interface of its
// segment (it writes the halos of its segment).
template <typename Real, int NV, bool RAGGED, int CH>
__device__ __forceinline__ RowOut<Real> row_pass(const RowIO &io, const RowCoef<Real> &c, bool first, bool last,
                                                 ConstPtr<Real> vt)
{
    constexpr int HV = NV / 2;
    constexpr unsigned R = sizeof(Real);
    RowOut<Real> o{0, 0, 0};
    PairBuf<Real, CH> A, B;
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        A.wn[u] = buf_load<Real>(io.rs, io.vo, (unsigned)u * io.rowb);
        A.wp[u] = buf_load<Real>(io.rs, io.vo, (unsigned)(NV - 1 - u) * io.rowb);
        A.hn[u] = buf_load<Real>(io.rs, 0u, io.hn + (unsigned)u * R);
        A.hp[u] = buf_load<Real>(io.rs, 0u, io.hp + (unsigned)(HV - 1 - u) * R);
    }
    Real Glo = 0, Ghi = 0;  // zero-flux velocity ends
    Real gj = recon(A.wn[0], vt[1], c.c1), gm = recon(A.wp[0], vt[1], c.c1);
#pragma unroll 1
    for (int t0 = 0; t0 < HV - 2 * CH; t0 += 2 * CH) {
        pair_chunk<Real, NV, false, RAGGED, CH>(t0, io, c, first, last, vt, A, B, gj, gm, Glo, Ghi, o);
        pair_chunk<Real, NV, false, RAGGED, CH>(t0 + CH, io, c, first, last, vt, B, A, gj, gm, Glo, Ghi, o);
    }
    pair_chunk<Real, NV, false, RAGGED, CH>(HV - 2 * CH, io, c, first, last, vt, A, B, gj, gm, Glo, Ghi, o);
    pair_chunk<Real, NV, true, RAGGED, CH>(HV - CH, io, c, first, last, vt, B, A, gj, gm, Glo, Ghi, o);
    return o;
}

// Resident form of a row pass: the rows of the interface live in registers
// (Wr[j], w form) for the whole slice, the halo rows in LDS (hn/hp read,
// hno/hpo written, all indexed by pair).  Same arithmetic as pair_chunk.
// The scalar table row and the two halo values of pair t+1 are requested
// right after the first use of those of pair t, so that the single wait on
// the LDS/scalar counter at the top of each pair finds them complete.  In a
// ragged segment the lane after the last valid one holds a copy of the v<0
// half of interface 0 (its periodic neighbour), so the DPP shift needs no
// per-lane select.
template <typename Real, int NV>
__device__ __forceinline__ RowOut<Real> row_pass_res(Real (&Wr)[NV], const RowCoef<Real> &c, bool first, bool last,
                                                     ConstPtr<Real> vt, const Real *hn, const Real *hp, Real *hno,
                                                     Real *hpo)
{
    constexpr int HV = NV / 2;
    RowOut<Real> o{0, 0, 0};
    PairAcc<Real> a{0, 0, 0};
    Real Glo = 0, Ghi = 0;  // zero-flux velocity ends
    Real cx = vt[0], M = vt[1], vM = vt[2], Mn = vt[3];
    Real hjv = hn[0], hmv = hp[HV - 1];
    Real gj = recon(Wr[0], M, c.c1), gm = recon(Wr[NV - 1], M, c.c1);
#pragma unroll
    for (int t = 0; t < HV; ++t) {
        const int j = t, m = NV - 1 - t;
        Real gjn, gmn;  // g_{j+1}, g_{m-1}
        if (t + 1 < HV) {
            gjn = recon(Wr[j + 1], Mn, c.c1);
            gmn = recon(Wr[m - 1], Mn, c.c1);
        } else {  // middle pair
            gjn = gm;
            gmn = gj;
        }
        const Real hj = hjv + M * c.c1n, hm = hmv + M * c.c1p;
        const Real cxc = cx, vMc = vM;
        __builtin_amdgcn_sched_barrier(0);
        if (t + 1 < HV) {
            cx = vt[4 * (t + 1)];
            M = vt[4 * (t + 1) + 1];
            vM = vt[4 * (t + 1) + 2];
            Mn = vt[4 * (t + 1) + 3];
            hjv = hn[t + 1];
            hmv = hp[HV - 2 - t];
        }
        __builtin_amdgcn_sched_barrier(0);
        const Real gxj = from_next_or(hj, gj);
        const Real gxm = from_prev_or(hm, gm);
        const Real Gj = c.Ep * gj + c.Em * gjn;
        const Real Gm = (t + 1 == HV) ? Gj : c.Ep * gmn + c.Em * gm;
        const Real gvj = Gj - Glo, gvm = Ghi - Gm;
        Glo = Gj;
        Ghi = Gm;
        const Real dgj = gj - gxj, dgm = gm - gxm;
        const Real Aj = cxc * dgj + gvj, Am = cxc * dgm + gvm;
        Real wj, wm;
        relax_pair(c, gj, gm, Aj, Am, vMc, wj, wm);
        Wr[j] = wj;
        Wr[m] = wm;
        // the stored rows that pair t+1 reads stay live until the new values
        // of pair t exist, so that each new value takes the register of the
        // value it replaces (else the allocation rotates by one row per pass
        // and every step pays a register copy per row)
        if (t + 1 < HV) {
            asm volatile("" ::"v"(Wr[j + 1]));
            asm volatile("" ::"v"(Wr[m - 1]));
        }
        if (first) hno[t] = wj;
        if (last) hpo[HV - 1 - t] = wm;
        acc_pair(o, a, Aj, Am, cxc, wj, wm, gj, gm);
        if ((t & 3) == 3 || t + 1 == HV) acc_flush(o, a);
        gj = gjn;
        gm = gmn;
    }
    return o;
}

// Fine sweep: one workgroup per unit (slice), all fine steps of the slice in
// one launch.  Threads own interfaces/cells p = k*B + t (slab k).
//
// Per step n the workgroup needs three barriers:
//   P1  cell status of step n from the criteria of step n-1 (interfaces
//       turning fluid drop their perturbation), density update with the
//       fluxes of step n-1, wave prefix sums of (rho - rhobar) dx     | B1
//   P2  field E (Gauss law, zero-mean gauge), cell-centred flux J      | B2
//   P3  phase-space pass of every segment with a kinetic interface:
//       transport, projection, relaxation, flux Phi and the norm of g;
//       remainder criterion of every cell (after the pass, by the first
//       half of the wavefronts, which the SIMDs serve first)            | B3
// RES: resident form (rows in registers, halos and c1 in LDS), for units
// whose rows fit in the registers of their lanes; otherwise the rows stream
// from the unit slot every step.
template <typename Real, int NV, int IPTM, bool RES, int BLK>
__device__ __forceinline__ void fine_body(const FineUnit *__restrict__ units)
{
    constexpr int CH = pair_chunk_len<Real, NV, BLK>();
    constexpr int HV = NV / 2;
    // Where the mean of the cell-centred J is reduced: in FP32 bulk the row
    // pass leaves the criterion phase little slack, so the field phase does
    // it; in FP64 the criterion phase does.
    constexpr bool kJtotInField = sizeof(Real) == 4;
    extern __shared__ __align__(16) unsigned char smem[];

    const FineUnit &U = units[blockIdx.x];
    if (U.stop && *U.stop) return;  // the problem has converged: uniform exit
    const FineConst *__restrict__ C = &U.c;
    const int nx = C->nx;
    const int ld = fine_ld(nx);
    // tid and lane are re-laundered at every step (see opaque_v)
    int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int BS = blockDim.x, NW = BS / kWave;
    const int ipt = (nx + BS - 1) / BS;
    const int nseg = (nx + kWave - 1) / kWave;
    const int nslot = ipt * NW;
    const int flags = C->flags;
    const bool hybrid = flags & STH_HYBRID, field = flags & STH_FIELD, literal = flags & STH_LITERAL_R;
    const bool cellwise = hybrid && (flags & STH_LITERAL_FLUX);
    // cell status history / replay (diagnostic runs only), read once
    const unsigned long long *const mrep = U.mask_replay;
    unsigned long long *const mhist = U.mask_hist;
    const bool mdbg = hybrid && (mrep != nullptr || mhist != nullptr);
    const long long nsteps = U.nsteps >= 0 ? U.nsteps : C->nsteps;
    const long long step0 = U.step0 > 0 ? U.step0 : 0;
    const long long step1 = (U.step1 > 0 && U.step1 < nsteps) ? U.step1 : nsteps;
    const bool resume = step0 > 0, suspend = step1 < nsteps;
    const double *__restrict__ g_e = C->e_p;
    const double *__restrict__ g_a = C->a_p;
    const double *__restrict__ g_eps = C->eps_p;
    const double *__restrict__ g_epsn = C->eps_n;  // norms: eps times the velocity-space scale
    const double *__restrict__ g_epsc = C->eps_c;

    const FineLds L = fine_lds(nx, NV, (int)sizeof(Real), nslot, RES);
    // macroscopic arrays with periodic ghost cells (see fine_lds); the owner
    // of a cell also writes its ghost copies
    double *s_rho = (double *)(smem + L.rho) + 3;
    double *s_jc = (double *)(smem + L.jc) + 3;
    double *s_phi = (double *)(smem + L.phi) + 1;
    double *s_phiJ = (double *)(smem + L.phiJ) + 1;  // m2 J per interface (cell-wise update)
    double *s_E = (double *)(smem + L.E);
    Real *s_nrm = (Real *)(smem + L.nrm) + 1;  // eps ||g|| of the last pass
    unsigned char *s_cm = (unsigned char *)(smem + L.cm);      // [2][nx+1] cell status by step parity
    unsigned char *s_crit = (unsigned char *)(smem + L.crit);  // [nx+1] remainder criterion
    const int ncm = nx + 1;
    // Ghost copies are written without branches: a lane whose cell has no
    // ghost writes its second copy to its own slot of a sink array.
    double *s_sink = (double *)(smem + L.dummy);
    unsigned char *s_sink8 = (unsigned char *)(s_sink + kWave);
    auto put_rho = [&](int i, double v) {
        s_rho[i] = v;
        double *g = i < 3 ? s_rho + nx + i : (i >= nx - 3 ? s_rho + (i - nx) : s_sink + lane);
        *g = v;
    };
    auto put_jc = [&](int i, double v) {
        s_jc[i] = v;
        double *g = i < 3 ? s_jc + nx + i : (i >= nx - 3 ? s_jc + (i - nx) : s_sink + lane);
        *g = v;
    };
    auto put_nrm = [&](int i, Real v) {
        s_nrm[i] = v;
        Real *g = i == 0 ? s_nrm + nx : (i == nx - 1 ? s_nrm - 1 : (Real *)(s_sink + lane));
        *g = v;
    };
    double *s_tot = (double *)(smem + L.tot);
    double *s_jtot = (double *)(smem + L.jtot);
    double *s_wtot = (double *)(smem + L.wtot);

    GlobPtr<Real> W = (GlobPtr<Real>)U.g_out;        // [NV][ld] rows
    GlobPtr<Real> C1 = W + (size_t)NV * ld;          // [2][ld] lazy projection
    const size_t hoff = fine_halo_off(nx, NV);       // H[2 parity][2 side][nseg][HV]
    GlobPtr<Real> H = W + hoff;
    const __amdgpu_buffer_rsrc_t slot =
        __builtin_amdgcn_make_buffer_rsrc(U.g_out, 0, (int)(sizeof(Real) * fine_slot_elems(nx, NV)), kBufferFlags);
    // element offset of a halo row: side 0 = v<0 half of a segment's first
    // interface, side 1 = v>0 half of its last
#define HALO(par, side, seg) ((size_t)(((par) * 2 + (side)) * nseg + (seg)) * HV)
    // resident form: rows in registers, c1 and halos in LDS
    Real Wr[RES ? IPTM : 1][RES ? NV : 1];
    Real *s_c1 = (Real *)(smem + L.c1);              // [2][nx]
    Real *s_halo = (Real *)(smem + L.halo);          // [2][2][nseg][HV]

    // [NV][4] table in the working precision for the row passes
    const ConstPtr<Real> vtr = (ConstPtr<Real>)(sizeof(Real) == 8 ? (const void *)C->vrow64
                                                                 : (const void *)C->vrow32);

    const Real *gin = (const Real *)U.g_in;
    const Real dvR = (Real)C->dv;
    const double rhobar = C->rhobar, dx = C->dx, dv = C->dv, m2 = C->m2;
    const double inv_dx = 1.0 / dx, dtdx = C->dt / dx, inv_nx = 1.0 / (double)nx;

    unsigned kinbits = 0, cmbits = 0;          // status of the thread's slabs
    unsigned long long kcount = 0;
    double comp[IPTM];                         // compensation of the density sums

    // ---------------------------------------------------------- prologue
    // Rows from g_in (padding lanes hold zero), halos of both parities,
    // norms of g_in, status "kinetic" before the first rule.
#pragma unroll
    for (int k = 0; k < IPTM; ++k) {
        const int i = k * BS + tid;
        comp[k] = 0.0;
        kinbits |= 1u << k;
        cmbits |= 1u << k;
        if constexpr (RES) {
#pragma unroll
            for (int j = 0; j < NV; ++j) Wr[k][j] = Real(0);
        }
        if (resume) continue;
        if (k < ipt && i < nseg * kWave) {
            const bool valid = i < nx;
            const int seg = i / kWave, last = min(kWave - 1, nx - 1 - seg * kWave);
            Real q = 0;
            if constexpr (RES) {
#pragma unroll
                for (int j = 0; j < NV; ++j) {
                    const Real v = (gin && valid) ? gin[(size_t)j * ld + i] : Real(0);
                    Wr[k][j] = v;
                    q += v * v;
                    if (lane == 0 && j < HV) {
                        s_halo[HALO(0, 0, seg) + j] = v;
                        s_halo[HALO(1, 0, seg) + j] = Real(0);
                    }
                    if (lane == last && j >= HV) {
                        s_halo[HALO(0, 1, seg) + j - HV] = v;
                        s_halo[HALO(1, 1, seg) + j - HV] = Real(0);
                    }
                }
                if (valid) {
                    s_c1[i] = Real(0);
                    s_c1[nx + i] = Real(0);
                }
            } else {
                for (int j = 0; j < NV; ++j) {
                    const Real v = (gin && valid) ? gin[(size_t)j * ld + i] : Real(0);
                    W[(size_t)j * ld + i] = v;
                    q += v * v;
                    if (lane == 0 && j < HV) {
                        H[HALO(0, 0, seg) + j] = v;
                        H[HALO(1, 0, seg) + j] = Real(0);
                    }
                    if (lane == last && j >= HV) {
                        H[HALO(0, 1, seg) + j - HV] = v;
                        H[HALO(1, 1, seg) + j - HV] = Real(0);
                    }
                }
                C1[i] = Real(0);
                C1[ld + i] = Real(0);
            }
            if (valid) {
                put_rho(i, U.rho_in[i]);
                put_nrm(i, (Real)g_epsn[i] * (Real)sqrt((double)(q * dvR)));
                s_cm[ncm + i] = 1;
                if (i == 0) s_cm[ncm + nx] = 1;
            }
        }
    }
    // Resumed slice: the macroscopic state from the checkpoint, the rows,
    // lazy projection and halos of this step's parity from the slot (the
    // resident form reloads them into registers and LDS).
    const int par0 = (int)(step0 & 1);
    if (resume) {
        const double *ck = U.ckpt;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k >= ipt) continue;
            if (i < nx) {
                comp[k] = ck[(size_t)nx + i];
                put_rho(i, ck[i]);
                const double ph = ck[2 * (size_t)nx + i], pj = ck[3 * (size_t)nx + i];
                s_phi[i] = ph;
                *(i == nx - 1 ? s_phi - 1 : s_sink + lane) = ph;
                s_phiJ[i] = pj;
                *(i == nx - 1 ? s_phiJ - 1 : s_sink + lane) = pj;
                put_nrm(i, (Real)ck[4 * (size_t)nx + i]);
                const unsigned char cmo = (unsigned char)(ck[5 * (size_t)nx + i] != 0.0);
                const unsigned char cr = (unsigned char)(ck[6 * (size_t)nx + i] != 0.0);
                s_cm[(par0 ^ 1) * ncm + i] = cmo;
                if (i == 0) s_cm[(par0 ^ 1) * ncm + nx] = cmo;
                s_crit[i] = cr;
                if (i == 0) s_crit[nx] = cr;
            }
            if constexpr (RES) {
                if (i < nseg * kWave) {
                    const bool valid = i < nx;
                    const int seg = i / kWave, last = min(kWave - 1, nx - 1 - seg * kWave);
#pragma unroll
                    for (int j = 0; j < NV; ++j) Wr[k][j] = valid ? W[(size_t)j * ld + i] : Real(0);
                    // both parities: a segment without kinetic interfaces
                    // skips its pass and keeps the other parity's values
                    if (valid) {
                        s_c1[i] = C1[i];
                        s_c1[nx + i] = C1[(size_t)ld + i];
                    }
#pragma unroll 1
                    for (int pp = 0; pp < 2; ++pp) {
                        if (lane == 0) {
#pragma unroll 1
                            for (int j = 0; j < HV; ++j) s_halo[HALO(pp, 0, seg) + j] = H[HALO(pp, 0, seg) + j];
                        }
                        if (lane == last) {
#pragma unroll 1
                            for (int j = 0; j < HV; ++j) s_halo[HALO(pp, 1, seg) + j] = H[HALO(pp, 1, seg) + j];
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    if (resume && hybrid) {
        // status of the last step run: cells from the checkpoint, interface
        // i kinetic iff one of its cells is
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) {
                const unsigned ci = s_cm[(par0 ^ 1) * ncm + i], cn = s_cm[(par0 ^ 1) * ncm + i + 1];
                cmbits = (cmbits & ~(1u << k)) | (ci << k);
                kinbits = (kinbits & ~(1u << k)) | ((ci | cn) << k);
            }
        }
    }

    double incl[IPTM];

    // Wave prefix sums of d_i = (rho_i - rhobar) dx and of d_i (nx - i), whose
    // total is sum_p s_p (for the zero-mean gauge).
    auto macro_scan = [&]() {
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            if (k < ipt) {
                const int i = k * BS + tid;
                const bool valid = i < nx;
                const double d = valid ? (s_rho[i] - rhobar) * dx : 0.0;
                double a = d, b = valid ? d * (double)(nx - i) : 0.0;
                wave_scan2_f64(a, b);
                incl[k] = a;
                const double tot = lane_value(a, kWave - 1);
                const double w = lane_value(b, kWave - 1);
                if (lane == 0) {
                    s_tot[k * NW + wid] = tot;
                    s_wtot[k * NW + wid] = w;
                }
            }
        }
    };
    // Field E_p (Gauss law, zero-mean gauge), and (hybrid) the cell-centred
    // J_i = d1 rho_i - E_i rho_i with E_i = E_p - d_p/2.
    auto macro_field = [&]() {
        const double t = lane < nslot ? s_tot[lane] : 0.0;
        double a = t, b = lane < nslot ? s_wtot[lane] : 0.0;
        wave_scan2_f64(a, b);
        const double ex = a - t;
        const double mean_s = lane_value(b, kWave - 1) * inv_nx;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            if (k < ipt) {
                const int i = k * BS + tid;
                const bool valid = i < nx;
                const double pre = lane_value(ex, k * NW + wid);
                const double E = field ? (pre + incl[k]) - mean_s : 0.0;
                double jsum = 0.0;
                if (valid) {
                    const double r = s_rho[i];
                    s_E[i] = E;
                    if (hybrid) {
                        const double Ec = field ? E - 0.5 * (r - rhobar) * dx : 0.0;
                        const double jc = fd1g(s_rho + i) * inv_dx - Ec * r;
                        put_jc(i, jc);
                        jsum = jc;
                    }
                }
                if (hybrid && kJtotInField) {
                    jsum = wave_total_f64(jsum);
                    if (lane == 0) s_jtot[k * NW + wid] = jsum;
                }
            }
        }
    };
    // Remainder R_i (eq. RemainderBis, Table 1 stencils) of the current
    // density and its criterion bit.
    auto crit_cell = [&](int i, double mJ) {
        const double inv_dx2 = inv_dx * inv_dx, inv_dx3 = inv_dx2 * inv_dx;
        const double r = s_rho[i];
        const double jc = s_jc[i];
        const double d1J = fd1g(s_jc + i) * inv_dx;
        const double d3J = fd3g(s_jc + i) * inv_dx3;
        double R;
        if (field) {
            const double Ec = s_E[i] - 0.5 * (r - rhobar) * dx;
            const double d1r = fd1g(s_rho + i) * inv_dx;
            const double d2J = fd2g(s_jc + i) * inv_dx2;
            R = -d3J + Ec * d2J + (2.0 * r - 3.0 * rhobar) * d1J + 2.0 * jc * d1r - d1r * (jc - mJ);
        } else {
            R = -d3J;
        }
        const double ec = g_epsc[i];
        const double crit = literal ? fabs(R) : ec * ec * fabs(R);
        s_crit[i] = (unsigned char)(crit > C->eta0);
        *(i == 0 ? s_crit + nx : s_sink8 + lane) = (unsigned char)(crit > C->eta0);
    };
    // Mean of the cell-centred J over all cells: from the wavefront totals
    // of the field phase, or (FP64) summed by each wavefront that needs it,
    // in the same order in every one, which keeps that reduction out of the
    // field phase and in the criterion phase's slack.
    auto mean_jc = [&]() {
        if constexpr (kJtotInField) {
            return wave_total_f64(lane < nslot ? s_jtot[lane] : 0.0) * inv_nx;
        } else {
            double acc = 0.0;
#pragma unroll 1
            for (int q = lane; q < nx; q += kWave) acc += s_jc[q];
            return wave_total_f64(acc) * inv_nx;
        }
    };
    auto macro_crit = [&]() {
        const double mJ = mean_jc();
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) crit_cell(i, mJ);
        }
    };
    // The same for every cell, by the first half of the wavefronts (each
    // lane takes its own cells and those of the lane BS/2 further): called
    // after the row pass, where the SIMDs' first wavefronts would otherwise
    // wait at the barrier for the second ones, which the scheduler serves
    // later.
    auto macro_crit_half = [&]() {
        const double mJ = mean_jc();
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = k * BS + tid + h * (BS / 2);
                if (k < ipt && i < nx) crit_cell(i, mJ);
            }
        }
    };
    // Cell status of step n (parity par) from the criterion bits, the norms
    // and the status of step n-1: a kinetic cell stays kinetic while a norm
    // of its interfaces or its criterion exceeds the threshold, a fluid cell
    // turns kinetic on the criterion.  Each thread evaluates its cell i and
    // cell i+1, which fixes the status of interface i; interfaces turning
    // fluid get g' = 0 (row, lazy projection, halos of both parities).
    auto status = [&](int par, long long n) {
        const double delta0 = C->delta0;
        const unsigned char *cm_old = s_cm + (par ^ 1) * ncm;
        const int mw = (nx + kWave - 1) / kWave;
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) {
                // every input read up front, combined without short-circuits
                const double Nm = (double)s_nrm[i - 1], N0 = (double)s_nrm[i], Np = (double)s_nrm[i + 1];
                const unsigned cr0 = s_crit[i], cr1 = s_crit[i + 1], co0 = cm_old[i], co1 = cm_old[i + 1];
                const double n0 = Nm > N0 ? Nm : N0, n1 = N0 > Np ? N0 : Np;
                int ci = (int)(cr0 | (co0 & (n0 > delta0 ? 1u : 0u)));
                int cn = (int)(cr1 | (co1 & (n1 > delta0 ? 1u : 0u)));
                if (mdbg) {
                    const size_t row = (size_t)n * mw;
                    if (mrep) {
                        const int i1 = i + 1 == nx ? 0 : i + 1;
                        ci = (int)((mrep[row + (i >> 6)] >> (i & 63)) & 1ull);
                        cn = (int)((mrep[row + (i1 >> 6)] >> (i1 & 63)) & 1ull);
                    }
                    // the cells of a wavefront are 64 consecutive ones from a
                    // multiple of 64: one word per wavefront
                    const unsigned long long b = __ballot(ci != 0);
                    if (mhist && lane == 0) mhist[row + (i >> 6)] = b;
                }
                s_cm[par * ncm + i] = (unsigned char)ci;
                *(i == 0 ? s_cm + par * ncm + nx : s_sink8 + lane) = (unsigned char)ci;
                cmbits = (cmbits & ~(1u << k)) | ((unsigned)ci << k);
                const int kn = ci | cn;
                if (((kinbits >> k) & 1u) && !kn) {
                    // rare; rolled loops keep their addresses out of the step loop's registers
                    const int seg = i / kWave, last = min(kWave - 1, nx - 1 - seg * kWave);
                    if constexpr (RES) {
#pragma unroll
                        for (int j = 0; j < NV; ++j) Wr[k][j] = Real(0);
                        s_c1[i] = Real(0);
                        s_c1[nx + i] = Real(0);
#pragma unroll 1
                        for (int pp = 0; pp < 2; ++pp) {
                            if (lane == 0) {
#pragma unroll 1
                                for (int j = 0; j < HV; ++j) s_halo[HALO(pp, 0, seg) + j] = Real(0);
                            }
                            if (lane == last) {
#pragma unroll 1
                                for (int j = 0; j < HV; ++j) s_halo[HALO(pp, 1, seg) + j] = Real(0);
                            }
                        }
                    } else {
#pragma unroll 1
                    for (int j = 0; j < NV; ++j) W[(size_t)j * ld + i] = Real(0);
                    C1[i] = Real(0);
                    C1[ld + i] = Real(0);
#pragma unroll 1
                    for (int pp = 0; pp < 2; ++pp) {
                        if (lane == 0) {
#pragma unroll 1
                            for (int j = 0; j < HV; ++j) H[HALO(pp, 0, seg) + j] = Real(0);
                        }
                        if (lane == last) {
#pragma unroll 1
                            for (int j = 0; j < HV; ++j) H[HALO(pp, 1, seg) + j] = Real(0);
                        }
                    }
                    }
                }
                kinbits = (kinbits & ~(1u << k)) | ((unsigned)kn << k);
            }
        }
    };
    // Density update with the fluxes of the previous step, compensated
    // (Kahan) so that long slices keep the mass to round-off: flux-matched
    // (conservative), or cell-wise as printed in scheme S^HMM with the cell
    // status cm of the previous step (kinetic cell: kinetic fluxes, fluid
    // cell: m2 J).
    auto density_update = [&](unsigned cm) {
#pragma unroll
        for (int k = 0; k < IPTM; ++k) {
            const int i = k * BS + tid;
            if (k < ipt && i < nx) {
                const double r = s_rho[i];
                const bool kin_cell = !cellwise || ((cm >> k) & 1u);
                const double fr = kin_cell ? s_phi[i] : s_phiJ[i];
                const double fl = kin_cell ? s_phi[i - 1] : s_phiJ[i - 1];
                const double y = dtdx * (fr - fl) - comp[k];
                const double t = r + y;
                comp[k] = (t - r) - y;
                put_rho(i, t);
            }
        }
    };

    if (hybrid && !resume) {
        // criterion bits of the initial density (the norms are those of g_in)
        macro_scan();
        __syncthreads();
        macro_field();
        __syncthreads();
        macro_crit();
        __syncthreads();
    }

    // ---------------------------------------------------------- step loop
    for (long long n = step0; n < step1; ++n) {
        const int par = (int)(n & 1), npar = par ^ 1;
        tid = opaque_v(tid);
        lane = tid & (kWave - 1);
        // P1: status of step n, density at step n, prefix sums.
        const unsigned cm_prev = cmbits;
        if (hybrid) status(par, n);
        if (n > 0) density_update(cm_prev);
        macro_scan();
        __syncthreads();  // B1
        // P2: field and cell-centred flux.
        macro_field();
        __syncthreads();  // B2
        // P3: the phase-space pass and the criterion bits (before the pass
        // when the workgroup has one wavefront or an odd count).
        const bool crit_after = NW >= 2 && (NW & 1) == 0;
        if (hybrid && !crit_after) macro_crit();
        // one slab k: coefficients, row pass of a segment with a kinetic
        // interface, flux and norm
        auto slab = [&](int k, auto &&pass) {
            const int i = k * BS + tid;
            const int seg = k * NW + wid;  // wavefront-uniform
            if (seg >= nseg) return;
            const bool valid = i < nx;
            const bool kv = valid && ((kinbits >> k) & 1u);
            kcount += kv ? 1ull : 0ull;
            const int iv = valid ? i : nx - 1;
            const double r = s_rho[iv], rn = s_rho[iv + 1];
            const double E = valid ? s_E[iv] : 0.0;
            const double J = (rn - r) * inv_dx - E * 0.5 * (r + rn);
            double Phi = m2 * J;
            Real Nn = 0;
            if (__ballot(kv)) {
                const int last = min(kWave - 1, nx - 1 - seg * kWave);
                const int segn = seg + 1 == nseg ? 0 : seg + 1;
                const int segp = seg == 0 ? nseg - 1 : seg - 1;
                const Real er = (Real)g_e[iv], ar = (Real)g_a[iv];
                const Real epsr = (Real)g_eps[iv];
                RowCoef<Real> c;
                c.Ep = (Real)(E > 0.0 ? E / dv : 0.0);
                c.Em = (Real)(E < 0.0 ? E / dv : 0.0);
                c.e = kv ? er : Real(0);
                c.a = kv ? ar : Real(0);
                c.aeps = kv ? ar * epsr : Real(0);
                c.aJ = kv ? (Real)((double)ar * J) : Real(0);
                const RowOut<Real> o = pass(k, i, iv, seg, segn, segp, last, c);
                const Real c1n = (Real)((double)c.aeps * (o.Sx * dv));
                if constexpr (RES) {
                    if (valid) s_c1[npar * nx + i] = c1n;
                } else {
                    C1[(size_t)npar * ld + i] = c1n;
                }
                if (kv) Phi = -(o.phi * dx) * dv;
                Nn = (Real)(g_epsn[iv] * sqrt(o.gg * dv));
            }
            if (valid) {
                s_phi[i] = Phi;
                *(i == nx - 1 ? s_phi - 1 : s_sink + lane) = Phi;
                if (cellwise) {
                    s_phiJ[i] = m2 * J;
                    *(i == nx - 1 ? s_phiJ - 1 : s_sink + lane) = m2 * J;
                }
                put_nrm(i, Nn);
            }
        };
        if constexpr (RES) {
#pragma unroll
            for (int k = 0; k < IPTM; ++k) {
                if (k < ipt)
                    slab(k, [&](int kk, int i, int iv, int seg, int segn, int segp, int last, RowCoef<Real> &c) {
                        // halo row addresses as vector registers (LDS addresses must be),
                        // so that each access is the base plus an immediate offset
                        const Real *hn = s_halo + opaque_v((int)HALO(par, 0, segn));
                        const Real *hp = s_halo + opaque_v((int)HALO(par, 1, segp));
                        Real *hno = s_halo + opaque_v((int)HALO(npar, 0, seg));
                        Real *hpo = s_halo + opaque_v((int)HALO(npar, 1, seg));
                        // ragged segment: the lane after the last valid one mirrors the
                        // v<0 half of interface 0 (w form, with its c1)
                        const bool ghost = last < kWave - 1 && lane == last + 1;
                        if (ghost) {
#pragma unroll
                            for (int j = 0; j < HV; ++j) Wr[k][j] = hn[j];
                        }
                        // lanes past the ghost keep zero rows and a zero projection (their
                        // relaxation must leave them at zero)
                        const Real c1v = s_c1[par * nx + (ghost ? 0 : iv)];
                        c.c1 = (i < nx || ghost) ? c1v : Real(0);
                        c.c1n = s_c1[par * nx + wrapi(iv + 1, nx)];
                        c.c1p = s_c1[par * nx + wrapi(iv - 1, nx)];
                        const ConstPtr<Real> vt = opaque(vtr);
                        return row_pass_res<Real, NV>(Wr[k], c, lane == 0, lane == last, vt, hn, hp, hno, hpo);
                    });
            }
        } else {
#pragma unroll 1
            for (int k = 0; k < ipt; ++k) {
                slab(k, [&](int kk, int i, int iv, int seg, int segn, int segp, int last, RowCoef<Real> &c) {
                    const GlobPtr<Real> C1p = C1 + (size_t)par * ld;
                    c.c1 = C1p[i];
                    c.c1n = C1p[wrapi(i + 1, nx)];
                    c.c1p = C1p[wrapi(i - 1, nx)];
                    constexpr unsigned R = sizeof(Real);
                    RowIO io;
                    io.rs = slot;
                    io.vo = (unsigned)i * R;
                    io.rowb = (unsigned)ld * R;
                    io.hn = (unsigned)(hoff + HALO(par, 0, segn)) * R;
                    io.hp = (unsigned)(hoff + HALO(par, 1, segp)) * R;
                    io.hno = (unsigned)(hoff + HALO(npar, 0, seg)) * R;
                    io.hpo = (unsigned)(hoff + HALO(npar, 1, seg)) * R;
                    const ConstPtr<Real> vt = opaque(vtr);
                    return last == kWave - 1 ? row_pass<Real, NV, false, CH>(io, c, lane == 0, lane == last, vt)
                                             : row_pass<Real, NV, true, CH>(io, c, lane == 0, lane == last, vt);
                });
            }
        }
        if (hybrid && crit_after && wid < NW / 2) macro_crit_half();
        __syncthreads();  // B3
    }

    // ---------------------------------------------------------- epilogue
    // End of the slice: status and density of the last step, outputs, rows
    // reconstructed (g = w + M c1).  Suspended slice (step1 < nsteps): the
    // checkpoint of the macroscopic state instead; the resident form also
    // stores its rows (w form), and its lazy projection and halos of both
    // parities (a segment without kinetic interfaces skips its pass and keeps
    // the values of the other parity); the streamed form keeps all of them
    // in the slot.
    const int fpar = (int)(step1 & 1);
    const unsigned cm_last = cmbits;
    if (!suspend) {
        if (hybrid) status(fpar, step1);
        if (nsteps > 0) density_update(cm_last);
    }
    double *ck = U.ckpt;
#pragma unroll
    for (int k = 0; k < IPTM; ++k) {
        const int i = k * BS + tid;
        if (k < ipt && i < nx) {
            if (suspend) {
                ck[i] = s_rho[i];
                ck[(size_t)nx + i] = comp[k];
                ck[2 * (size_t)nx + i] = s_phi[i];
                ck[3 * (size_t)nx + i] = s_phiJ[i];
                ck[4 * (size_t)nx + i] = (double)s_nrm[i];
                ck[5 * (size_t)nx + i] = (double)s_cm[(fpar ^ 1) * ncm + i];
                ck[6 * (size_t)nx + i] = (double)s_crit[i];
            } else {
                U.rho_out[i] = s_rho[i];
                if (U.mask_out) U.mask_out[i] = hybrid ? (int)((cmbits >> k) & 1u) : 1;
            }
            if constexpr (RES) {
                const Real c1 = s_c1[fpar * nx + i];
                const Real cf = suspend ? Real(0) : c1;
#pragma unroll
                for (int j = 0; j < NV; ++j) W[(size_t)j * ld + i] = Wr[k][j] + vtr[4 * j + 1] * cf;
                if (suspend) {
                    C1[i] = s_c1[i];
                    C1[(size_t)ld + i] = s_c1[nx + i];
                }
            } else if (!suspend) {
                const Real c1 = C1[(size_t)fpar * ld + i];
                if (c1 != Real(0)) {
#pragma unroll 1
                    for (int j = 0; j < NV; ++j) W[(size_t)j * ld + i] += vtr[4 * j + 1] * c1;
                }
                C1[i] = Real(0);
                C1[ld + i] = Real(0);
            }
        }
    }
    if constexpr (RES) {
        if (suspend) {
#pragma unroll 1
            for (int k = 0; k < ipt; ++k) {
                const int i = k * BS + tid;
                if (i < nseg * kWave) {
                    const int seg = i / kWave, last = min(kWave - 1, nx - 1 - seg * kWave);
#pragma unroll 1
                    for (int pp = 0; pp < 2; ++pp) {
                        if (lane == 0) {
#pragma unroll 1
                            for (int j = 0; j < HV; ++j) H[HALO(pp, 0, seg) + j] = s_halo[HALO(pp, 0, seg) + j];
                        }
                        if (lane == last) {
#pragma unroll 1
                            for (int j = 0; j < HV; ++j) H[HALO(pp, 1, seg) + j] = s_halo[HALO(pp, 1, seg) + j];
                        }
                    }
                }
            }
        }
    }
    if (U.kin) {
        const unsigned long long tot = wave_sum(kcount);
        if (lane == 0) atomicAdd(U.kin, tot);
    }
#undef HALO
}

template <typename Real, int NV, int IPTM, bool RES, int BLK>
__global__ void __launch_bounds__(BLK) k_fine(const FineUnit *__restrict__ units)
{
    fine_body<Real, NV, IPTM, RES, BLK>(units);
}

// Launch shape of a fine-sweep class: one workgroup per unit, up to 1024
// threads, interfaces distributed over at most kMaxSlabs slabs.
// Rows of one lane fit its registers in the resident form (at most 128
// VGPRs of the 256 that two wavefronts per SIMD leave to each).
__host__ __device__ constexpr bool fine_resident_fits(int realsz, int iptm, int nv)
{
    return iptm * nv * (realsz / 4) <= 128;
}

static int fine_iptm(int ipt) { return ipt <= 2 ? ipt : 4; }

bool fine_wide_ok(int prec, int nv) { return prec == 1 || nv == 32; }

FineShape fine_shape(int prec, int nx, int nv, int force_stream, int force_block)
{
    FineShape s{};
    s.prec = prec;
    s.nv = nv;
    const int realsz = prec == 0 ? 8 : 4;
    int nxr = ((nx + kWave - 1) / kWave) * kWave;
    int b = force_block > 0 ? force_block : kFineBlock;
    // wide workgroups: streamed rows only, in the classes whose streamed
    // kernel fits 128 registers per lane
    const bool wide = b > kFineBlock && force_stream && fine_wide_ok(prec, nv);
    if (b > (wide ? kWideBlock : kFineBlock)) b = wide ? kWideBlock : kFineBlock;
    if (b > nxr) b = nxr;
    s.block = b;
    s.ipt = (nx + b - 1) / b;
    const int nslot = s.ipt * (s.block / kWave);
    const bool res = !force_stream && s.block <= kFineBlock && s.ipt <= kMaxSlabs &&
                     fine_resident_fits(realsz, fine_iptm(s.ipt), nv) &&
                     fine_lds(nx, nv, realsz, nslot, true).total <= kMaxLds;
    s.stream = res ? 0 : 1;
    s.lds = fine_lds(nx, nv, realsz, nslot, res).total;
    if (!res && force_block <= 0 && nxr > kFineBlock && fine_wide_ok(prec, nv)) {
        // default for streamed rows beyond 512 interfaces: the wide workgroup
        // (twice the wavefronts per CU to cover the row loads)
        s.block = std::min(kWideBlock, nxr);
        s.ipt = (nx + s.block - 1) / s.block;
        s.lds = fine_lds(nx, nv, realsz, s.ipt * (s.block / kWave), false).total;
    }
    return s;
}

FineShape fine_group_shape(const FineShape &s, int nx, int block)
{
    FineShape g = s;
    const int realsz = s.prec == 0 ? 8 : 4;
    g.block = block;
    g.ipt = (nx + block - 1) / block;
    const int nslot = g.ipt * (block / kWave);
    const bool res = !s.stream && block <= kFineBlock && g.ipt <= kMaxSlabs &&
                     fine_resident_fits(realsz, fine_iptm(g.ipt), s.nv) &&
                     fine_lds(nx, s.nv, realsz, nslot, true).total <= kMaxLds;
    g.stream = res ? 0 : 1;
    g.lds = fine_lds(nx, s.nv, realsz, nslot, res).total;
    return g;
}

int fine_group_code(const FineShape &g) { return fine_class_code(g.nv, fine_iptm(g.ipt), g.stream == 0); }

template <typename Real, int NV, int IPT, bool RES, int BLK>
static hipError_t launch_one(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    auto kern = k_fine<Real, NV, IPT, RES, BLK>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)s.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n), dim3(s.block), s.lds, st, d);
    return hipGetLastError();
}

template <typename Real, int NV, int IPT>
static hipError_t launch_form(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    if (s.block > kFineBlock) {
        if constexpr (IPT <= 2 && (sizeof(Real) == 4 || NV == 32)) {
            if (s.stream && s.block <= kWideBlock) return launch_one<Real, NV, IPT, false, kWideBlock>(s, d, n, st);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (fine_resident_fits((int)sizeof(Real), IPT, NV)) {
        if (!s.stream) return launch_one<Real, NV, IPT, true, kFineBlock>(s, d, n, st);
    } else {
        if (!s.stream) return hipErrorInvalidValue;
    }
    return launch_one<Real, NV, IPT, false, kFineBlock>(s, d, n, st);
}

template <typename Real, int NV>
static hipError_t launch_nv(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    switch (s.ipt) {
        case 1: return launch_form<Real, NV, 1>(s, d, n, st);
        case 2: return launch_form<Real, NV, 2>(s, d, n, st);
        case 3:
        case 4: return launch_form<Real, NV, 4>(s, d, n, st);
    }
    return hipErrorInvalidValue;
}

// Grouped fine sweep: every workgroup runs the class its unit names.  The
// classes of a group share the precision and the workgroup size, so the
// hardware dispatcher works through one table of units, longest first,
// whatever their class.  Codes without a kernel of this precision and size
// are never produced by the host.
template <typename Real, int BLK, int NV, int IPTM, bool RES>
__device__ __forceinline__ void fine_group_arm(const FineUnit *__restrict__ units)
{
    if constexpr (BLK > kFineBlock) {
        if constexpr (!RES && IPTM <= 2 && (sizeof(Real) == 4 || NV == 32))
            fine_body<Real, NV, IPTM, false, BLK>(units);
    } else if constexpr (!RES || fine_resident_fits((int)sizeof(Real), IPTM, NV)) {
        fine_body<Real, NV, IPTM, RES, BLK>(units);
    }
}

template <typename Real, int BLK>
__global__ void __launch_bounds__(BLK) k_fine_group(const FineUnit *__restrict__ units)
{
    switch (units[blockIdx.x].cls) {
#define STH_ARM(NV, IPTM, RES)                                   \
    case fine_class_code(NV, IPTM, RES):                         \
        fine_group_arm<Real, BLK, NV, IPTM, RES>(units);         \
        return;
#define STH_ARMS(NV) STH_ARM(NV, 1, false) STH_ARM(NV, 1, true) STH_ARM(NV, 2, false) \
                     STH_ARM(NV, 2, true) STH_ARM(NV, 4, false) STH_ARM(NV, 4, true)
        STH_ARMS(16)
        STH_ARMS(32)
        STH_ARMS(64)
        STH_ARMS(128)
#undef STH_ARMS
#undef STH_ARM
        default:
            return;
    }
}

template <typename Real, int BLK>
static hipError_t launch_group(size_t lds, const FineUnit *d, int n, hipStream_t st)
{
    auto kern = k_fine_group<Real, BLK>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n), dim3(BLK), lds, st, d);
    return hipGetLastError();
}

hipError_t launch_fine_group(int prec, int block, size_t lds, const FineUnit *d, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (block == kFineBlock) return prec == 0 ? launch_group<double, kFineBlock>(lds, d, n, st)
                                              : launch_group<float, kFineBlock>(lds, d, n, st);
    if (block == kWideBlock) return prec == 0 ? launch_group<double, kWideBlock>(lds, d, n, st)
                                              : launch_group<float, kWideBlock>(lds, d, n, st);
    return hipErrorInvalidValue;
}

hipError_t launch_fine(const FineShape &s, const FineUnit *d, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (s.ipt > kMaxSlabs || s.block % kWave != 0 || s.block > kWideBlock) return hipErrorInvalidValue;
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
// Poisson on one workgroup: E[p] from rho (global or LDS), zero-mean gauge,
// E_p = s_p - mean(s) with s_p = sum_{i<=p} (rho_i - rhobar) dx.  Each thread
// owns ceil(nx/blockDim) contiguous cells; wavefront DPP scans of the cell
// sums and of sum_i d_i (nx - i) (= sum_p s_p), then one pass over the wave
// totals.  blockDim is a multiple of 64, at most 1024.
__device__ void block_poisson(const double *rho, double *E, int nx, double dx, double rhobar,
                              bool field)
{
    if (!field) {
        for (int p = threadIdx.x; p < nx; p += blockDim.x) E[p] = 0.0;
        __syncthreads();
        return;
    }
    __shared__ double s_wt[2][16];
    const int BS = blockDim.x, t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    const int NW = (BS + kWave - 1) / kWave;
    const int q = (nx + BS - 1) / BS, i0 = t * q;
    double own = 0.0, wsum = 0.0;
    for (int u = 0; u < q; ++u) {
        const int i = i0 + u;
        const double d = i < nx ? (rho[i] - rhobar) * dx : 0.0;
        own += d;
        wsum += i < nx ? d * (double)(nx - i) : 0.0;
    }
    double a = own, b = wsum;
    wave_scan2_f64(a, b);
    if (lane == kWave - 1) {
        s_wt[0][wid] = a;
        s_wt[1][wid] = b;
    }
    __syncthreads();
    double off = 0.0, Wtot = 0.0;
    for (int w = 0; w < NW; ++w) {
        off += w < wid ? s_wt[0][w] : 0.0;
        Wtot += s_wt[1][w];
    }
    const double mean = Wtot / (double)nx;
    double run = off + (a - own);
    for (int u = 0; u < q; ++u) {
        const int i = i0 + u;
        if (i < nx) {
            run += (rho[i] - rhobar) * dx;
            E[i] = run - mean;
        }
    }
    __syncthreads();
}

// Cyclic tridiagonal solve a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i
// (indices mod n, 8 <= n <= 2048, diagonally dominant) by the first
// wavefront of the workgroup; every thread of the workgroup calls it.
// Partition method: lane p owns a contiguous block of m >= 2 rows; the
// interior rows of its block (all but the last) are eliminated by Thomas
// with three right-hand sides, which expresses them through the last rows
// l_{p-1} (previous block) and l_p; substituting into the equations of the
// last rows leaves a cyclic tridiagonal system for l_0..l_{P-1}, solved by
// one lane with Thomas and the Sherman-Morrison correction, then every lane
// reconstructs its rows.  Y, U, V, cp: [n] scratch; x may alias V.
__device__ void cyclic_tridiag_block(const double *a, const double *b, const double *c, const double *d,
                                     double *x, double *Y, double *U, double *V, double *cp, int n)
{
    __shared__ double s_red[8][kWave];
    double *rA = s_red[0], *rB = s_red[1], *rC = s_red[2], *rD = s_red[3];
    double *rL = s_red[4], *rcp = s_red[5], *rdp = s_red[6], *rz = s_red[7];
    const int t = threadIdx.x;
    const int P = min(kWave, n / 2);
    const int base = n / P, rem = n % P;
    auto first_row = [&](int p) { return p * base + min(p, rem); };
    // interior elimination (rows r0 .. last-1), three right-hand sides
    if (t < P) {
        const int r0 = first_row(t), k = base + (t < rem ? 1 : 0) - 1;
        double den = b[r0];
        cp[r0] = c[r0] / den;
        Y[r0] = d[r0] / den;
        U[r0] = -a[r0] / den;
        V[r0] = (k == 1 ? -c[r0] : 0.0) / den;
        for (int i = 1; i < k; ++i) {
            const int row = r0 + i;
            den = b[row] - a[row] * cp[row - 1];
            cp[row] = c[row] / den;
            Y[row] = (d[row] - a[row] * Y[row - 1]) / den;
            U[row] = (-a[row] * U[row - 1]) / den;
            V[row] = ((i == k - 1 ? -c[row] : 0.0) - a[row] * V[row - 1]) / den;
        }
        for (int i = k - 2; i >= 0; --i) {
            const int row = r0 + i;
            Y[row] -= cp[row] * Y[row + 1];
            U[row] -= cp[row] * U[row + 1];
            V[row] -= cp[row] * V[row + 1];
        }
    }
    __syncthreads();
    // reduced system of the last rows
    if (t < P) {
        const int r0 = first_row(t), last = r0 + base + (t < rem ? 1 : 0) - 1, il = last - 1;
        const int f = first_row(t + 1 == P ? 0 : t + 1);
        const double al = a[last], cl = c[last];
        rA[t] = al * U[il];
        rB[t] = al * V[il] + b[last] + cl * U[f];
        rC[t] = cl * V[f];
        rD[t] = d[last] - al * Y[il] - cl * Y[f];
    }
    __syncthreads();
    if (t == 0) {
        // Thomas on the matrix with the corner terms moved into a rank-one
        // update u v^T, u = (gamma, 0, .., 0, C_{P-1}), v = (1, 0, .., 0, A_0/gamma)
        const double gamma = -rB[0];
        const double b0 = rB[0] - gamma;
        const double bl = rB[P - 1] - rA[0] * rC[P - 1] / gamma;
        double m = b0;
        rcp[0] = rC[0] / m;
        rdp[0] = rD[0] / m;
        rz[0] = gamma / m;
        for (int i = 1; i < P; ++i) {
            const double bi = (i == P - 1) ? bl : rB[i];
            m = bi - rA[i] * rcp[i - 1];
            rcp[i] = rC[i] / m;
            rdp[i] = (rD[i] - rA[i] * rdp[i - 1]) / m;
            const double ui = (i == P - 1) ? rC[P - 1] : 0.0;
            rz[i] = (ui - rA[i] * rz[i - 1]) / m;
        }
        rL[P - 1] = rdp[P - 1];
        for (int i = P - 2; i >= 0; --i) {
            rL[i] = rdp[i] - rcp[i] * rL[i + 1];
            rz[i] = rz[i] - rcp[i] * rz[i + 1];
        }
        const double fact = (rL[0] + rA[0] * rL[P - 1] / gamma) / (1.0 + rz[0] + rA[0] * rz[P - 1] / gamma);
        for (int i = 0; i < P; ++i) rL[i] -= fact * rz[i];
    }
    __syncthreads();
    if (t < P) {
        const int r0 = first_row(t), k = base + (t < rem ? 1 : 0) - 1;
        const double lp = rL[t == 0 ? P - 1 : t - 1], lo = rL[t];
        for (int i = 0; i < k; ++i) {
            const int row = r0 + i;
            x[row] = Y[row] + U[row] * lp + V[row] * lo;
        }
        x[r0 + k] = lo;
    }
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
    if (J.stop && *J.stop) return;
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
    const int ld = fine_ld(nx);
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
            g[(size_t)j * ld + p] = (Real)val;
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
    cyclic_tridiag_block(a, b, c, rin, x, dp, z, x, cp, nx);
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

// Explicit limit scheme S^0 (Section 2.3, the paper's coarse propagator of
// Section 3.3) over one coarse interval: coarse_steps steps of
// rho_i += dt/dx m2 (J_{i+1/2} - J_{i-1/2}) with J from the current rho and
// its Gauss-law field.  One workgroup; rho and the fluxes in dynamic LDS;
// each thread owns nx/blockDim contiguous cells, and the Gauss-law prefix
// sums are DPP wavefront scans plus a pass over the wave totals.
__device__ void coarse_explicit_block(const FineConst *C, const double *rin, double *rout, double dtG)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = C->nx, BS = blockDim.x, t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    const int NW = (BS + kWave - 1) / kWave;
    double *r = (double *)smem;  // [nx]
    double *phi = r + nx;        // [nx]
    double *wt = phi + nx;       // [2][16] wave totals
    const int q = (nx + BS - 1) / BS;  // cells per thread, at most 2
    const long long ns = C->coarse_steps > 0 ? C->coarse_steps : 1;
    const double dt = dtG / (double)ns, dx = C->dx, m2 = C->m2, rhobar = C->rhobar;
    const double dtdx = dt / dx, inv_dx = 1.0 / dx, inv_nx = 1.0 / (double)nx;
    const bool field = C->flags & STH_FIELD;
    for (int i = t; i < nx; i += BS) r[i] = rin[i];
    __syncthreads();
    const int i0 = t * q;
    for (long long n = 0; n < ns; ++n) {
        double S[2] = {0.0, 0.0}, own = 0.0, wsum = 0.0;
        for (int u = 0; u < q; ++u) {
            const int i = i0 + u;
            const double d = i < nx ? (r[i] - rhobar) * dx : 0.0;
            own += d;
            S[u] = own;
            wsum += i < nx ? d * (double)(nx - i) : 0.0;
        }
        double a = own, b = wsum;
        wave_scan2_f64(a, b);
        if (lane == kWave - 1) {
            wt[wid] = a;
            wt[16 + wid] = b;
        }
        __syncthreads();
        double off = 0.0, Wtot = 0.0;
        for (int w = 0; w < NW; ++w) {
            const double tw = wt[w];
            off += w < wid ? tw : 0.0;
            Wtot += wt[16 + w];
        }
        const double before = off + (a - own);  // sum of d over the cells before this thread's
        const double mean = Wtot * inv_nx;      // mean of the prefix sums
        for (int u = 0; u < q; ++u) {
            const int i = i0 + u;
            if (i < nx) {
                const double E = field ? (before + S[u]) - mean : 0.0;
                const double ri = r[i], rn = r[wrapi(i + 1, nx)];
                const double Jp = (rn - ri) * inv_dx - E * 0.5 * (ri + rn);
                phi[i] = m2 * Jp;
            }
        }
        __syncthreads();
        for (int u = 0; u < q; ++u) {
            const int i = i0 + u;
            if (i < nx) r[i] = r[i] + dtdx * (phi[i] - phi[wrapi(i - 1, nx)]);
        }
        __syncthreads();
    }
    for (int i = t; i < nx; i += BS) rout[i] = r[i];
    __syncthreads();
}

__device__ void coarse_any_block(const FineConst *C, const double *rin, double *rout, double dtG, double *w)
{
    if (C->flags & STH_COARSE_EXPLICIT) coarse_explicit_block(C, rin, rout, dtG);
    else coarse_step_block(C, rin, rout, dtG, w);
}

// Coarse guess (mode 0) or parareal correction (mode 1) of one problem by
// one workgroup, sequential over the slices (Algorithm 1).
__device__ void coarse_job(const CoarseJob &J)
{
    double *work = J.work;
    const int nx = J.pc->nx;
    const size_t slab = (size_t)nx;
    double *gn = work + 8 * slab;
    if (J.mode == 0) {
        if (J.ctl) {
            if (threadIdx.x == 0) {
                J.ctl[0] = 0;
                J.ctl[1] = 0;
            }
            for (int n = threadIdx.x; n <= J.N; n += blockDim.x) J.kin[n] = 0ull;
        }
        for (int n = 1; n <= J.N; ++n) {
            coarse_any_block(J.pc, J.U + (n - 1) * slab, J.U + n * slab, J.dtG, work);
            for (int i = threadIdx.x; i < nx; i += blockDim.x) J.Gc[n * slab + i] = J.U[n * slab + i];
            __syncthreads();
        }
        return;
    }
    if (J.ctl && J.ctl[1]) return;  // converged: uniform exit
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
        coarse_any_block(J.pc, J.U + (n - 1) * slab, gn, J.dtG, work);
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
    if (threadIdx.x == 0) {
        J.err[0] = e;
        if (J.errh) J.errh[k] = e;
        if (J.ctl) {
            J.ctl[0] = k + 1;
            J.ctl[1] = (e < J.tol || k + 1 >= J.kmax) ? 1 : 0;
        }
    }
}

__global__ void __launch_bounds__(1024) k_coarse(CoarseJob J) { coarse_job(J); }

__global__ void __launch_bounds__(1024) k_coarse_many(const CoarseJob *__restrict__ jobs)
{
    const CoarseJob J = jobs[blockIdx.x];
    coarse_job(J);
}

void coarse_launch_dims(int nx, bool explicit_scheme, int *block, size_t *lds)
{
    int b = ((nx + kWave - 1) / kWave) * kWave;
    if (b > 1024) b = 1024;
    *block = b;
    *lds = explicit_scheme ? sizeof(double) * (2 * (size_t)nx + 32) : 0;
}

hipError_t launch_coarse(const CoarseJob &job, int nx, bool explicit_scheme, hipStream_t st)
{
    int b = 0;
    size_t lds = 0;
    coarse_launch_dims(nx, explicit_scheme, &b, &lds);
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void *)k_coarse, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_coarse, dim3(1), dim3(b), lds, st, job);
    return hipGetLastError();
}

hipError_t launch_coarse_many(const CoarseJob *d_jobs, int njobs, int block, size_t lds, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (block <= 0 || block > 1024 || block % kWave) return hipErrorInvalidValue;
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void *)k_coarse_many,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_coarse_many, dim3(njobs), dim3(block), lds, st, d_jobs);
    return hipGetLastError();
}

// ------------------------------------------------------------ copies
__global__ void __launch_bounds__(256) k_copy(const CopyJob *__restrict__ jobs)
{
    const CopyJob J = jobs[blockIdx.y];
    if (J.stop && *J.stop) return;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < J.n; i += (size_t)gridDim.x * 256)
        J.dst[i] = J.src[i];
}

hipError_t launch_copy(const CopyJob *d_jobs, int njobs, size_t max_n, hipStream_t st)
{
    if (njobs <= 0 || max_n == 0) return hipSuccess;
    if (njobs > 65535) return hipErrorInvalidValue;
    size_t gx = (max_n + 255) / 256;
    if (gx > 256) gx = 256;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)gx, (unsigned)njobs), dim3(256), 0, st, d_jobs);
    return hipGetLastError();
}

// ------------------------------------------------------------ layout conversions
// x-major float64 perturbation -> v-major rows of stride ld (one thread per
// row element, padding lanes zero) and back.
template <typename Real>
__global__ void __launch_bounds__(256) k_to_vmajor(const double *__restrict__ gx, Real *__restrict__ rows, int nx,
                                                  int nv, int ld)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nv * ld) return;
    const int j = (int)(t / ld), p = (int)(t % ld);
    rows[t] = p < nx ? (Real)gx[(size_t)p * nv + j] : Real(0);
}

template <typename Real>
__global__ void __launch_bounds__(256) k_to_xmajor(const Real *__restrict__ rows, double *__restrict__ gx, int nx,
                                                  int nv, int ld)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nx * nv) return;
    const int p = (int)(t / nv), j = (int)(t % nv);
    gx[t] = (double)rows[(size_t)j * ld + p];
}

hipError_t launch_to_vmajor(int prec, const double *gx, void *rows, int nx, int nv, hipStream_t st)
{
    const int ld = fine_ld(nx);
    const size_t n = (size_t)nv * ld;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (prec == 0) hipLaunchKernelGGL(k_to_vmajor<double>, grid, dim3(256), 0, st, gx, (double *)rows, nx, nv, ld);
    else hipLaunchKernelGGL(k_to_vmajor<float>, grid, dim3(256), 0, st, gx, (float *)rows, nx, nv, ld);
    return hipGetLastError();
}

hipError_t launch_to_xmajor(int prec, const void *rows, double *gx, int nx, int nv, hipStream_t st)
{
    const int ld = fine_ld(nx);
    const size_t n = (size_t)nx * nv;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (prec == 0) hipLaunchKernelGGL(k_to_xmajor<double>, grid, dim3(256), 0, st, (const double *)rows, gx, nx, nv, ld);
    else hipLaunchKernelGGL(k_to_xmajor<float>, grid, dim3(256), 0, st, (const float *)rows, gx, nx, nv, ld);
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
    const int ld = fine_ld(nx);
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
                const double gv = (double)g[(size_t)j * ld + p];
                ph += vt[3 * nv + j] * gv * dv;
                q += gv * gv * dv;
            }
        }
        oPhi[p] = -ph;
        oN[p] = C->eps_n[p] * sqrt(q);
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
