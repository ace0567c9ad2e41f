// sth_internal.h -- device-side data layout shared by the kernels and the
// host library of libsth.so (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace sth {

constexpr int kWave = 64;
constexpr int kMaxNx = 2048;
constexpr size_t kMaxLds = 160 * 1024;  // LDS bytes of one gfx950 workgroup
constexpr int kMaxSlabs = 4;          // interfaces per thread (nx <= 2048 with 512 threads)
constexpr int kFineBlock = 512;       // threads per fine-sweep workgroup (default form)
constexpr int kWideBlock = 1024;      // wide workgroups of the streamed form (chosen per class)

// Per-problem constants of the fine propagator (device memory).
struct FineConst {
    int nx, nv;
    int flags;            // STH_HYBRID | STH_FIELD | STH_LITERAL_R
    int pad0;
    double dx, dv, dt, rhobar, m2, eta0, delta0;
    long long nsteps;     // fine steps per slice
    long long coarse_steps; // steps of S^0 per coarse interval (STH_COARSE_EXPLICIT)
    const double *eps_p;  // [nx] eps at interfaces
    const double *eps_c;  // [nx] eps at cell centres
    const double *eps_n;  // [nx] eps_p times the norm scale of the velocity space (norms only)
    const double *e_p;    // [nx] exp(-dt/eps_p^2)
    const double *a_p;    // [nx] -expm1(-dt/eps_p^2)
    const double *vtab;   // [4][nv]: |v_j|/dx, M_j, v_j M_j, v_j
    const double *vrow64; // [nv][4]: |v_j|/dx, M_j, v_j M_j, M_{j+1} (M_nv = 0), float64
    const float *vrow32;  // [nv][4]: the same row table, float32
};

// Row stride of the v-major perturbation arrays: nx padded to a multiple of
// the wavefront, so that every row access of a wavefront is in bounds.
__host__ __device__ inline int fine_ld(int nx) { return (nx + kWave - 1) / kWave * kWave; }

// Per-unit state slot in global memory (elements of the working precision):
// rows W[nv][ld] (v-major, padding lanes zero), the lazy projection
// C1[2][ld] and the halo rows H[2 parity][2 side][ld/64][nv/2] of the
// wavefront segments.  After a sweep W holds the perturbation.
__host__ __device__ inline size_t fine_halo_off(int nx, int nv) { return ((size_t)nv + 2) * (size_t)fine_ld(nx); }
__host__ __device__ inline size_t fine_slot_elems(int nx, int nv)
{
    return fine_halo_off(nx, nv) + 2 * (size_t)(fine_ld(nx) / kWave) * (size_t)nv;
}

// One fine-propagation unit: one slice of one problem.
struct FineUnit {
    FineConst c;              // problem constants by value (scalar loads)
    const double *rho_in;     // [nx] density at the slice start
    double *rho_out;          // [nx] density at the slice end
    const void *g_in;         // [nv][ld] v-major start perturbation, Real; NULL = 0
    void *g_out;              // [nv][ld] v-major end perturbation, Real (a full slot)
                              // (required by the streaming kernels: it is their state)
    unsigned long long *kin;  // kinetic interface-steps counter (atomic add)
    int *mask_out;            // [nx] final cell status, or NULL
    long long nsteps;         // steps of this unit (0: none, the start state after
                              // the status rule; < 0: pc->nsteps)
    const int *stop;          // the problem's stop flag (the unit does nothing
                              // when it is set), or NULL
    // Step range [step0, step1) of the slice run by this launch (step1 <= 0:
    // to the end).  step0 > 0 resumes from the checkpoint and the slot;
    // step1 < nsteps stops after step1 - 1 and leaves the checkpoint and the
    // slot (rows in w form, lazy projection and halos of both parities)
    // instead of the outputs.
    long long step0, step1;
    double *ckpt;             // [kCkptArrays][nx] when the slice is chunked
    // Cell status of every step n = 0..nsteps (row n: the status applied at
    // step n, row nsteps: after the last), one bit per cell, rows of
    // (nx + 63) / 64 words: recorded into mask_hist and/or imposed from
    // mask_replay instead of the rule (hybrid runs; NULL in the sweeps).
    const unsigned long long *mask_replay;
    unsigned long long *mask_hist;
    int cls;                  // class code (fine_class_code) in a grouped launch
};
// Checkpoint of a suspended unit: rho, its compensation, Phi, m2 J, the
// norms, the cell status of the last step and the criterion bits, each nx
// doubles.
constexpr int kCkptArrays = 7;

// Launch shape of a fine-sweep kernel class.
struct FineShape {
    int prec;     // 0 = FP64, 1 = FP32 bulk
    int nv;
    int ipt;      // interfaces per thread (slabs)
    int stream;   // 1 = rows streamed from the unit slot every step; 0 = resident
                  // in registers for the whole slice
    int block;    // threads per workgroup
    size_t lds;   // dynamic LDS bytes
};

FineShape fine_shape(int prec, int nx, int nv, int force_stream, int force_block);
// Code of a kernel class within one precision and workgroup size: velocity
// count (16, 32, 64, 128), slabs per thread (1, 2, 4) and row form.
constexpr int fine_class_code(int nv, int iptm, bool resident)
{
    return ((nv == 16 ? 0 : nv == 32 ? 1 : nv == 64 ? 2 : 3) * 3 + (iptm == 1 ? 0 : iptm == 2 ? 1 : 2)) * 2 +
           (resident ? 1 : 0);
}
// Grouped launch: units of several classes of one precision in one launch of
// `block`-thread workgroups (kFineBlock or kWideBlock), each unit running the
// class of its code (FineUnit::cls); lds is the largest the units need.
hipError_t launch_fine_group(int prec, int block, size_t lds, const FineUnit *d_units, int nunits,
                             hipStream_t st);
// The shape class s takes in a grouped launch of `block` threads: its row
// form where that still fits, else streamed; and the code of that shape.
FineShape fine_group_shape(const FineShape &s, int nx, int block);
int fine_group_code(const FineShape &g);
// The streamed kernel of this class exists with kWideBlock threads.
bool fine_wide_ok(int prec, int nv);
hipError_t launch_fine(const FineShape &s, const FineUnit *d_units, int nunits, hipStream_t st);

// Lifting L^L of rho at interfaces into a v-major Real array.
struct LiftJob {
    const FineConst *pc;
    const double *rho;    // [nx]
    void *g;              // [nv][ld] v-major Real
    int lift_order;
    const int *stop;      // skip when set, or NULL
};
hipError_t launch_lift(int prec, const LiftJob *d_jobs, int njobs, int nx, hipStream_t st);

// Coarse sweep / parareal correction on one problem (single workgroup,
// sequential over slices).
struct CoarseJob {
    const FineConst *pc;
    double *U;            // [(N+1)][nx] iterate
    double *Gc;           // [(N+1)][nx] cached coarse values
    const double *Fv;     // [(N+1)][nx] fine results
    double *err;          // [1] successive error out
    double *work;         // [9][nx] workspace
    double dtG;
    int N;
    int mode;             // 0 = coarse guess, 1 = correction
    int k;                // iteration index (correction)
    // Device-side iteration control, or NULL.  ctl[0] = iterations done,
    // ctl[1] = stop flag.  Mode 0 clears both and the kinetic counters
    // kin[0..N]; mode 1 does nothing when the stop flag is set, else it
    // corrects, stores ctl[0] = k + 1 and sets the flag when
    // err < tol or k + 1 >= kmax.
    int *ctl;
    double *errh;         // [N] error of each iteration (mode 1), or NULL
    unsigned long long *kin;
    double tol;
    int kmax;
    int pad;
};
// One problem (one workgroup, job by value).
hipError_t launch_coarse(const CoarseJob &job, int nx, bool explicit_scheme, hipStream_t st);
// Several problems in one launch, one workgroup each: block threads and
// dynamic LDS bytes cover the largest job (coarse_launch_dims).
void coarse_launch_dims(int nx, bool explicit_scheme, int *block, size_t *lds);
hipError_t launch_coarse_many(const CoarseJob *d_jobs, int njobs, int block, size_t lds, hipStream_t st);

// Device-to-device copy of n 16-byte words, skipped when *stop is set.
struct CopyJob {
    const uint4 *src;
    uint4 *dst;
    size_t n;
    const int *stop;
};
hipError_t launch_copy(const CopyJob *d_jobs, int njobs, size_t max_n, hipStream_t st);

// Perturbation layout conversions of the allocation-free single-slice run:
// x-major float64 g[p*nv + j] <-> the v-major working-precision rows
// rows[j*ld + p] of a unit slot (padding lanes zero).
hipError_t launch_to_vmajor(int prec, const double *gx, void *rows, int nx, int nv, hipStream_t st);
hipError_t launch_to_xmajor(int prec, const void *rows, double *gx, int nx, int nv, hipStream_t st);

// Diagnostics of a state (rho, g).
struct DiagJob {
    const FineConst *pc;
    const double *rho;    // [nx]
    const void *g;        // [nv][ld] v-major Real or NULL (0)
    double *out;          // [5][nx]: E, J, Phi, N, R
    int *mask;            // [nx]
};
hipError_t launch_diag(int prec, const DiagJob &job, int nx, hipStream_t st);

}  // namespace sth
