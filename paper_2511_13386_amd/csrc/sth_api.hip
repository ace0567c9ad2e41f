// sth_api.hip -- host side of libsth.so: problem set-up, device layout,
// parareal bookkeeping and the C-ABI declared in include/sth.h.
//
// Host arithmetic here is set-up only (grids, Maxwellian table, stable step,
// relaxation factors); every step of the solver runs in the kernels of
// sth_kernels.hip.
#include "sth.h"
#include "sth_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace sth;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// Device (or managed) memory, as a kernel argument must be; a host pointer
// makes the query fail, and its error is cleared here.
bool is_device_ptr(const void *ptr)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(STH_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #call);   \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Device layout of one problem (offsets from the arena base).
struct Layout {
    size_t cst, eps_p, eps_c, eps_n, e_p, a_p, vtab, vrow64, vrow32, U, Gc, Fv, err, errh, ctl, work, kin, mask, g0, gend,
        gst, ckpt, units, total;
};

Layout layout(int nx, int nv, int N, int realsz)
{
    Layout L;
    size_t o = 0;
    const size_t gsz = fine_slot_elems(nx, nv) * realsz;
    L.cst = o;   o = al256(o + sizeof(FineConst));
    L.eps_p = o; o = al256(o + sizeof(double) * nx);
    L.eps_c = o; o = al256(o + sizeof(double) * nx);
    L.eps_n = o; o = al256(o + sizeof(double) * nx);
    L.e_p = o;   o = al256(o + sizeof(double) * nx);
    L.a_p = o;   o = al256(o + sizeof(double) * nx);
    L.vtab = o;  o = al256(o + sizeof(double) * 4 * nv);
    L.vrow64 = o; o = al256(o + sizeof(double) * 4 * nv);
    L.vrow32 = o; o = al256(o + sizeof(float) * 4 * nv);
    L.U = o;     o = al256(o + sizeof(double) * (size_t)(N + 1) * nx);
    L.Gc = o;    o = al256(o + sizeof(double) * (size_t)(N + 1) * nx);
    L.Fv = o;    o = al256(o + sizeof(double) * (size_t)(N + 1) * nx);
    L.err = o;   o = al256(o + sizeof(double) * 4);
    L.errh = o;  o = al256(o + sizeof(double) * (size_t)(N + 1));
    L.ctl = o;   o = al256(o + sizeof(int) * 4);
    L.work = o;  o = al256(o + sizeof(double) * 9 * (size_t)nx);
    L.kin = o;   o = al256(o + sizeof(unsigned long long) * (size_t)(N + 1));
    L.mask = o;  o = al256(o + sizeof(int) * (size_t)nx);
    L.g0 = o;    o = al256(o + gsz);
    L.gend = o;  o = al256(o + gsz * (size_t)(N + 1));
    L.gst = o;   o = al256(o + gsz * (size_t)(N + 1));
    L.ckpt = o;  o = al256(o + sizeof(double) * kCkptArrays * (size_t)nx * (size_t)(N + 1));
    L.units = o; o = al256(o + sizeof(FineUnit) * (size_t)(N + 1));
    L.total = o;
    return L;
}

int validate(const sth_problem_desc *d)
{
    if (!d) return fail(STH_EINVAL, "null description");
    if (d->nx < 8 || d->nx > kMaxNx) return fail(STH_EINVAL, "nx must be in [8, 2048]");
    if (!(d->nv == 16 || d->nv == 32 || d->nv == 64 || d->nv == 128))
        return fail(STH_EINVAL, "nv must be 16, 32, 64 or 128");
    if (!(d->Lx > 0) || !(d->vstar > 0)) return fail(STH_EINVAL, "Lx and vstar must be > 0");
    if (!(d->T > 0) || d->n_slices < 1 || d->k_max < 1)
        return fail(STH_EINVAL, "T > 0, n_slices >= 1 and k_max >= 1 required");
    if (d->lift_order < 1 || d->lift_order > 3) return fail(STH_EINVAL, "lift_order must be 1, 2 or 3");
    if (d->start_mode != STH_START_LIFT && d->start_mode != STH_START_CARRY)
        return fail(STH_EINVAL, "unknown start_mode");
    if (!(d->cfl_theta > 0) || d->cfl_theta > 1) return fail(STH_EINVAL, "cfl_theta must be in (0, 1]");
    if (d->precision != STH_FP64 && d->precision != STH_FP32_BULK)
        return fail(STH_EINVAL, "unknown precision");
    if (d->flags & ~(STH_HYBRID | STH_FIELD | STH_LITERAL_R | STH_LITERAL_FLUX | STH_COARSE_EXPLICIT))
        return fail(STH_EINVAL, "unknown flags");
    if (fine_shape(d->precision == STH_FP64 ? 0 : 1, d->nx, d->nv, 0, 0).lds > kMaxLds)
        return fail(STH_EINVAL, "unit too large for one workgroup's LDS");
    if ((d->nv_y == 0) != (d->nv_z == 0)) return fail(STH_EINVAL, "nv_y and nv_z must be both 0 or both set");
    if (d->nv_y != 0 && (d->nv_y < 2 || d->nv_y > 512 || (d->nv_y & 1) || d->nv_z < 2 || d->nv_z > 512 || (d->nv_z & 1)))
        return fail(STH_EINVAL, "nv_y and nv_z must be even, in [2, 512]");
    return STH_OK;
}

// Pool of tables for batched launches: a device table and its pinned host
// mirror.  A table is staged in the mirror and copied asynchronously from
// there (never from a caller's pageable buffer, which may be gone before the
// copy runs); it is reserved from acquisition until release_table records
// the event after the launches that read it, and reused once that event
// has completed.
struct TableSlot {
    void *ptr = nullptr;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;      // ev marks the last launches that read it
    bool reserved = false;  // acquired, release_table not called yet
};
std::mutex g_pool_mu;
std::vector<TableSlot> g_pool;

int acquire_table(size_t bytes, int *slot_out)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t s = 0; s < g_pool.size(); ++s) {
        TableSlot &t = g_pool[s];
        if (t.cap < bytes || t.reserved) continue;
        if (t.used && hipEventQuery(t.ev) != hipSuccess) continue;
        t.reserved = true;
        *slot_out = (int)s;
        return STH_OK;
    }
    TableSlot t;
    t.cap = std::max(bytes, size_t(64) << 10);
    HIPCHK(hipMalloc(&t.ptr, t.cap));
    HIPCHK(hipHostMalloc(&t.host, t.cap, hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&t.ev, hipEventDisableTiming));
    t.reserved = true;
    g_pool.push_back(t);
    *slot_out = (int)g_pool.size() - 1;
    return STH_OK;
}

// Acquire a table, stage `bytes` of src in its mirror and copy it to the
// device on st.  Returns the device table in *dptr.
int put_table(const void *src, size_t bytes, hipStream_t st, int *slot_out, void **dptr)
{
    int slot = 0;
    int rc = acquire_table(bytes, &slot);
    if (rc) return rc;
    void *dev = nullptr, *host = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        dev = g_pool[slot].ptr;
        host = g_pool[slot].host;
    }
    if (bytes) std::memcpy(host, src, bytes);
    HIPCHK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, st));
    *slot_out = slot;
    *dptr = dev;
    return STH_OK;
}

// The launches that read the table have been issued on st.
int release_table(int slot, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    TableSlot &t = g_pool[slot];
    t.reserved = false;
    HIPCHK(hipEventRecord(t.ev, st));
    t.used = true;
    return STH_OK;
}

// Lanes of a device for batches with several kernel classes: each class
// runs on one of kLanes streams, forked from and joined back into the
// caller's stream with events.  Classes on one hardware queue run one after
// the other, and plain streams share the process's few hardware queues with
// every other stream in use (the caller's among them), so the lanes are
// created with a CU mask of every CU: a mask belongs to a hardware queue, and
// a masked stream gets a queue of its own.  Where the runtime refuses a
// masked stream, the lane is an ordinary non-blocking stream.
constexpr int kLanes = 4;
struct SidePool {
    hipStream_t s[kLanes] = {};
    hipEvent_t fork = nullptr, join[kLanes] = {};
    bool ready = false;
};
std::mutex g_side_mu, g_side_issue_mu;
std::vector<SidePool> g_side;

int side_pool(SidePool **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_side_mu);
    if ((int)g_side.size() <= dev) g_side.resize(dev + 1);
    SidePool &P = g_side[dev];
    if (!P.ready) {
        int cus = 0;
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        std::vector<uint32_t> mask((size_t)std::max(1, (cus + 31) / 32), 0u);
        for (int c = 0; c < cus; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
        for (int i = 0; i < kLanes; ++i) {
            if (hipExtStreamCreateWithCUMask(&P.s[i], (uint32_t)mask.size(), mask.data()) != hipSuccess) {
                (void)hipGetLastError();
                HIPCHK(hipStreamCreateWithFlags(&P.s[i], hipStreamNonBlocking));
            }
            HIPCHK(hipEventCreateWithFlags(&P.join[i], hipEventDisableTiming));
        }
        HIPCHK(hipEventCreateWithFlags(&P.fork, hipEventDisableTiming));
        P.ready = true;
    }
    *out = &P;
    return STH_OK;
}

// Launch configurations chosen for kernel classes (sth_set_fine_config),
// keyed by (precision, nv, nx rounded up to the wavefront).
struct ClassKey {
    int prec, nv, nxr;
    bool operator<(const ClassKey &o) const
    {
        return prec != o.prec ? prec < o.prec : (nv != o.nv ? nv < o.nv : nxr < o.nxr);
    }
};
std::mutex g_tune_mu;
std::map<ClassKey, sth_fine_config> g_tune;

ClassKey class_key(int prec, int nx, int nv) { return {prec, nv, (nx + kWave - 1) / kWave * kWave}; }

// A launch configuration is supported for nx when the workgroup is a
// multiple of the wavefront no larger than nx rounded up, covers nx with at
// most kMaxSlabs interfaces per thread, its LDS fits, and (resident) the
// rows fit in registers.
bool config_ok(int prec, int nx, int nv, const sth_fine_config &c)
{
    const int nxr = (nx + kWave - 1) / kWave * kWave;
    const int bmax = (!c.resident && fine_wide_ok(prec, nv)) ? kWideBlock : kFineBlock;
    if (c.block < kWave || c.block > bmax || c.block % kWave || c.block > nxr) return false;
    if ((nx + c.block - 1) / c.block > (c.block > kFineBlock ? 2 : kMaxSlabs)) return false;
    const FineShape sh = fine_shape(prec, nx, nv, c.resident ? 0 : 1, c.block);
    return sh.block == c.block && sh.lds <= kMaxLds && (sh.stream == 0) == (c.resident != 0);
}

// Candidate configurations for nx: for each count of interfaces per thread
// (1..kMaxSlabs) the smallest workgroup that covers nx with it, and the
// largest workgroups of both kinds; each resident (where supported) and
// streamed.
std::vector<sth_fine_config> class_candidates(int prec, int nx, int nv)
{
    std::vector<int> blocks;
    for (int ipt = 1; ipt <= kMaxSlabs; ++ipt) {
        const int per = (nx + ipt - 1) / ipt;
        blocks.push_back((per + kWave - 1) / kWave * kWave);
    }
    blocks.push_back(std::min(kFineBlock, (nx + kWave - 1) / kWave * kWave));
    blocks.push_back(std::min(kWideBlock, (nx + kWave - 1) / kWave * kWave));
    std::sort(blocks.begin(), blocks.end(), [](int a, int b) { return a > b; });
    blocks.erase(std::unique(blocks.begin(), blocks.end()), blocks.end());
    std::vector<sth_fine_config> out;
    for (int b : blocks)
        for (int res = 1; res >= 0; --res) {
            const sth_fine_config c{b, res};
            if (config_ok(prec, nx, nv, c)) out.push_back(c);
        }
    return out;
}

// Shape of the fine kernel for a class: the chosen configuration if one is
// set, else the default rule.
FineShape class_shape(int prec, int nx, int nv)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(class_key(prec, nx, nv));
        if (it != g_tune.end() && config_ok(prec, nx, nv, it->second))
            return fine_shape(prec, nx, nv, it->second.resident ? 0 : 1, it->second.block);
    }
    return fine_shape(prec, nx, nv, 0, 0);
}

}  // namespace

struct sth_problem {
    int nx, nv, N, K, prec, realsz, flags, start_mode, lift_order;
    double Lx, vstar, T, tol, dx, dv, dt, dtG, m2, rhobar, eta0, delta0;
    long long ns, coarse_steps = 1;
    double nscale = 1.0;    // 3D norm of a g(x, vx) M(vy) M(vz) state over its vx norm
    char *base = nullptr;
    size_t bytes = 0;
    bool owned = false;
    Layout L;
    FineConst fc{};         // host copy of the device constants
    int k = 0;              // completed parareal iterations
    bool coarse_done = false;
    bool swept = false;     // a fine sweep ran since the last correction
    bool has_g0 = false;
    std::vector<char> have_end;  // slice n has an end-of-slice perturbation
    double last_err = -1.0;
    long long chunk_pos = -1;    // next step of a chunked sweep in progress (-1: none)
    std::vector<FineUnit> chunk_units;

    template <typename T>
    T *at(size_t off) const { return (T *)(base + off); }
    // one slice's perturbation slot: rows [nv][nx] plus the lazy projection [2][nx]
    size_t gslab() const { return fine_slot_elems(nx, nv) * realsz; }
};

// A recorded whole solve of several problems (see sth_graph_create).
struct sth_graph {
    std::vector<sth_problem *> probs;
    std::vector<int> kmax;        // iterations of each problem at most
    int iters = 0;                // iterations recorded
    char *dbuf = nullptr;         // device tables the graph reads
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;    // capture stream
    bool launched = false;
};

namespace {

// Host set-up: velocity grid, discretely normalised Maxwellian, m2.
void velocity_table(int nv, double vstar, double dx, std::vector<double> &vtab, double &m2)
{
    const double dv = 2.0 * vstar / nv;
    std::vector<double> v(nv), M(nv);
    double Z = 0.0;
    // midpoint nodes, mirrored exactly (v_{nv-1-j} = -v_j) so that the fine
    // sweep can share one table row between a velocity and its mirror
    for (int j = 0; j < nv / 2; ++j) {
        v[j] = -vstar + (j + 0.5) * dv;
        v[nv - 1 - j] = -v[j];
    }
    for (int j = 0; j < nv; ++j) {
        M[j] = std::exp(-0.5 * v[j] * v[j]);
        Z += M[j] * dv;
    }
    m2 = 0.0;
    for (int j = 0; j < nv; ++j) {
        M[j] /= Z;
        m2 += v[j] * v[j] * M[j] * dv;
    }
    vtab.assign(4 * (size_t)nv, 0.0);
    for (int j = 0; j < nv; ++j) {
        vtab[j] = std::fabs(v[j]) / dx;
        vtab[nv + j] = M[j];
        vtab[2 * nv + j] = v[j] * M[j];
        vtab[3 * nv + j] = v[j];
    }
}

// sum_j M_j^2 dv for the discrete normalised Maxwellian on n midpoint nodes
// of [-vstar, vstar] (a transverse axis of the 1D3V velocity box).
double axis_m2sum(int n, double vstar)
{
    const double dv = 2.0 * vstar / n;
    std::vector<double> M(n);
    double Z = 0.0;
    for (int j = 0; j < n; ++j) {
        const double v = -vstar + (j + 0.5) * dv;
        M[j] = std::exp(-0.5 * v * v);
        Z += M[j] * dv;
    }
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += (M[j] / Z) * (M[j] / Z) * dv;
    return s;
}

// Stable fine step of the exponential-relaxation / upwind micro step:
// eps^2 ln((c+1)/(c-1)) for c = 2 eps (vmax/dx + Emax/dv) > 1, else the
// diffusive bound dx^2/(2 m2); 0.75 margin; theta the CFL fraction.
double stable_dt(const std::vector<double> &eps_p, double dx, double dv, double vstar, double m2,
                 double Emax, double theta)
{
    const double vmax = vstar - 0.5 * dv;
    const double sdiff = dx * dx / (2.0 * m2);
    double smin = sdiff;
    for (double eps : eps_p) {
        const double c = 2.0 * eps * (vmax / dx + Emax / dv);
        double s = sdiff;
        if (c > 1.0) s = std::min(s, eps * eps * std::log((c + 1.0) / (c - 1.0)));
        smin = std::min(smin, s);
    }
    return theta * 0.75 * smin;
}

// max |E| of the Gauss-law field of rho (zero-mean gauge).
double field_max(const std::vector<double> &rho, double rhobar, double dx)
{
    const int nx = (int)rho.size();
    std::vector<double> E(nx);
    double s = 0.0, m = 0.0;
    for (int p = 0; p < nx; ++p) {
        s += (rho[p] - rhobar) * dx;
        E[p] = s;
        m += s;
    }
    m /= nx;
    double mx = 0.0;
    for (int p = 0; p < nx; ++p) {
        const double a = std::fabs(E[p] - m);
        mx = (a > mx || a != a) ? a : mx;  // a NaN propagates
    }
    return mx;
}

// x-major double host array -> v-major Real device rows of stride ld
// (host staging; padding zero).
std::vector<char> to_vmajor(const double *g, int nx, int nv, int prec)
{
    const int ld = fine_ld(nx);
    std::vector<char> out((size_t)ld * nv * (prec == 0 ? 8 : 4), 0);
    for (int p = 0; p < nx; ++p)
        for (int j = 0; j < nv; ++j) {
            const double x = g[(size_t)p * nv + j];
            if (prec == 0) ((double *)out.data())[(size_t)j * ld + p] = x;
            else ((float *)out.data())[(size_t)j * ld + p] = (float)x;
        }
    return out;
}

void from_vmajor(const std::vector<char> &in, int nx, int nv, int prec, double *g)
{
    const int ld = fine_ld(nx);
    for (int p = 0; p < nx; ++p)
        for (int j = 0; j < nv; ++j)
            g[(size_t)p * nv + j] = prec == 0 ? ((const double *)in.data())[(size_t)j * ld + p]
                                              : (double)((const float *)in.data())[(size_t)j * ld + p];
}

size_t vmajor_bytes(int nx, int nv, int realsz) { return (size_t)fine_ld(nx) * nv * realsz; }

FineUnit make_unit(const sth_problem *p, int n)
{
    FineUnit u{};
    u.c = p->fc;
    u.rho_in = p->at<double>(p->L.U) + (size_t)(n - 1) * p->nx;
    u.rho_out = p->at<double>(p->L.Fv) + (size_t)n * p->nx;
    u.g_out = p->base + p->L.gend + (size_t)n * p->gslab();
    u.kin = p->at<unsigned long long>(p->L.kin) + n;
    u.mask_out = nullptr;
    u.nsteps = p->ns;
    u.ckpt = p->at<double>(p->L.ckpt) + (size_t)n * kCkptArrays * p->nx;
    return u;
}

// One fine unit of a batched sweep with its kernel class and cost.
struct SweepItem {
    FineShape shape;
    FineUnit unit;
    double cost;
};

// Units of iteration k of one problem (slices n = k+1..N), with the jobs
// that prepare their start perturbations: the given g0 for slice 1, a copy
// of the previous slice's end state (carry mode, when one exists), else the
// lifting of the slice-start density.  `have_end` says which slices have an
// end state; `stop` goes into every unit and job.
void plan_problem_sweep(sth_problem *p, int k, const std::vector<char> &have_end, const int *stop,
                        std::vector<SweepItem> &items, std::vector<LiftJob> &lifts, std::vector<CopyJob> &copies)
{
    const FineShape sh = class_shape(p->prec, p->nx, p->nv);
    for (int n = k + 1; n <= p->N; ++n) {
        FineUnit u = make_unit(p, n);
        u.stop = stop;
        void *gst = p->base + p->L.gst + (size_t)n * p->gslab();
        if (n == 1) {
            u.g_in = p->has_g0 ? (const void *)(p->base + p->L.g0) : nullptr;
        } else if (p->start_mode == STH_START_CARRY && have_end[n - 1]) {
            CopyJob c{};
            c.src = (const uint4 *)(p->base + p->L.gend + (size_t)(n - 1) * p->gslab());
            c.dst = (uint4 *)gst;
            c.n = p->gslab() / sizeof(uint4);
            c.stop = stop;
            copies.push_back(c);
            u.g_in = gst;
        } else {
            LiftJob lj{};
            lj.pc = p->at<FineConst>(p->L.cst);
            lj.rho = p->at<double>(p->L.U) + (size_t)(n - 1) * p->nx;
            lj.g = gst;
            lj.lift_order = p->lift_order;
            lj.stop = stop;
            lifts.push_back(lj);
            u.g_in = gst;
        }
        items.push_back({sh, u, (double)p->ns * p->nx * p->nv});
    }
}

bool same_class(const FineShape &a, const FineShape &b)
{
    return a.prec == b.prec && a.nv == b.nv && a.stream == b.stream && a.ipt == b.ipt && a.block == b.block;
}

// Group by kernel class, longest units first within a class (LPT order of
// dispatch).
void sort_items(std::vector<SweepItem> &items)
{
    std::stable_sort(items.begin(), items.end(), [](const SweepItem &a, const SweepItem &b) {
        if (a.shape.prec != b.shape.prec) return a.shape.prec < b.shape.prec;
        if (a.shape.nv != b.shape.nv) return a.shape.nv < b.shape.nv;
        if (a.shape.stream != b.shape.stream) return a.shape.stream < b.shape.stream;
        if (a.shape.ipt != b.shape.ipt) return a.shape.ipt < b.shape.ipt;
        if (a.shape.block != b.shape.block) return a.shape.block < b.shape.block;
        return a.cost > b.cost;
    });
}

// Launch the sorted units (device table dtab, same order): one launch per
// kernel class.  With several classes, each goes to the lane with the least
// work so far, costliest class first (longest-processing-time order), all
// lanes concurrent and joined back into st.
int issue_classes(const std::vector<SweepItem> &items, FineUnit *dtab, hipStream_t st)
{
    struct Group {
        FineShape sh;
        size_t begin, end;
        double cost;
    };
    std::vector<Group> groups;
    size_t begin = 0;
    while (begin < items.size()) {
        size_t end = begin + 1;
        FineShape sh = items[begin].shape;
        size_t lds = sh.lds;
        double cost = items[begin].cost;
        while (end < items.size() && same_class(items[end].shape, sh)) {
            lds = std::max(lds, items[end].shape.lds);
            cost += items[end].cost;
            ++end;
        }
        sh.lds = lds;
        groups.push_back({sh, begin, end, cost});
        begin = end;
    }
    if (groups.empty()) return STH_OK;
    if (groups.size() == 1) {
        HIPCHK(launch_fine(groups[0].sh, dtab, (int)items.size(), st));
        return STH_OK;
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group &a, const Group &b) { return a.cost > b.cost; });
    SidePool *P = nullptr;
    int rc = side_pool(&P);
    if (rc) return rc;
    // the fork/join events are shared: issue one batch at a time
    std::lock_guard<std::mutex> lk(g_side_issue_mu);
    const int nlanes = std::min<int>(kLanes, (int)groups.size());
    double load[kLanes] = {};
    HIPCHK(hipEventRecord(P->fork, st));
    for (int i = 0; i < nlanes; ++i) HIPCHK(hipStreamWaitEvent(P->s[i], P->fork, 0));
    for (const Group &g : groups) {
        int lane = 0;
        for (int i = 1; i < nlanes; ++i)
            if (load[i] < load[lane]) lane = i;
        load[lane] += g.cost;
        HIPCHK(launch_fine(g.sh, dtab + g.begin, (int)(g.end - g.begin), P->s[lane]));
    }
    for (int i = 0; i < nlanes; ++i) {
        HIPCHK(hipEventRecord(P->join[i], P->s[i]));
        HIPCHK(hipStreamWaitEvent(st, P->join[i], 0));
    }
    return STH_OK;
}

// Lift jobs of a batch, one launch per problem, from one staged table.
struct LiftBatch {
    std::vector<LiftJob> jobs;
    struct Run {
        int prec, nx;
        size_t begin, n;
    };
    std::vector<Run> runs;
    void add(const sth_problem *p, const std::vector<LiftJob> &l)
    {
        if (l.empty()) return;
        runs.push_back({p->prec, p->nx, jobs.size(), l.size()});
        jobs.insert(jobs.end(), l.begin(), l.end());
    }
    int issue(hipStream_t st) const
    {
        if (jobs.empty()) return STH_OK;
        int slot = 0;
        void *tab = nullptr;
        int rc = put_table(jobs.data(), sizeof(LiftJob) * jobs.size(), st, &slot, &tab);
        if (rc) return rc;
        hipError_t e = hipSuccess;
        for (const Run &r : runs) {
            if (e == hipSuccess) e = launch_lift(r.prec, (const LiftJob *)tab + r.begin, (int)r.n, r.nx, st);
        }
        rc = release_table(slot, st);
        if (e != hipSuccess) return hip_fail(e, "launch_lift");
        return rc;
    }
};

// Sort the units into kernel classes, stage their table and launch them.
// Units of several kernel classes in grouped launches: one launch per
// (precision, workgroup size), every workgroup running the class its unit
// names, the units of a launch longest first whatever their class, so that
// the hardware dispatcher starts the slices that bound the sweep first and
// fills the compute units with the rest behind them.  Classes of at most
// kFineBlock threads run in kFineBlock-thread workgroups (a small slice then
// leaves some wavefronts without cells), the wide streamed ones in
// kWideBlock.
struct GroupLaunch {
    int group;                 // precision * 2 + (1 for kWideBlock workgroups)
    size_t begin, end, lds;    // unit range in the table, LDS bytes
    double cost;
};

// The unit table (in launch order, class codes set) and the launches of a
// grouped sweep; false when some class does not fit a grouped launch.
bool plan_grouped(const std::vector<SweepItem> &items, std::vector<FineUnit> &table,
                  std::vector<GroupLaunch> &launches)
{
    std::vector<int> grp(items.size());
    std::vector<size_t> lds(items.size());
    std::vector<int> code(items.size());
    for (size_t t = 0; t < items.size(); ++t) {
        const SweepItem &it = items[t];
        const bool wide = it.shape.block > kFineBlock;
        const FineShape g = fine_group_shape(it.shape, it.unit.c.nx, wide ? kWideBlock : kFineBlock);
        if (g.lds > kMaxLds || (wide && (!g.stream || !fine_wide_ok(g.prec, g.nv)))) return false;
        grp[t] = it.shape.prec * 2 + (wide ? 1 : 0);
        lds[t] = g.lds;
        code[t] = fine_group_code(g);
    }
    std::vector<size_t> order(items.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        if (grp[a] != grp[b]) return grp[a] < grp[b];
        return items[a].cost > items[b].cost;
    });
    table.resize(items.size());
    launches.clear();
    for (size_t t = 0; t < order.size(); ++t) {
        const size_t u = order[t];
        table[t] = items[u].unit;
        table[t].cls = code[u];
        if (launches.empty() || launches.back().group != grp[u]) launches.push_back({grp[u], t, t, 0, 0.0});
        GroupLaunch &L = launches.back();
        L.end = t + 1;
        L.lds = std::max(L.lds, lds[u]);
        L.cost += items[u].cost;
    }
    return true;
}

// Issue the launches of a grouped sweep (device table dtab in plan order):
// one launch on st, or several concurrently on the lanes, costliest first.
int issue_grouped(std::vector<GroupLaunch> launches, const FineUnit *dtab, hipStream_t st)
{
    auto launch = [&](const GroupLaunch &L, hipStream_t s) {
        return launch_fine_group(L.group / 2, (L.group & 1) ? kWideBlock : kFineBlock, L.lds, dtab + L.begin,
                                 (int)(L.end - L.begin), s);
    };
    if (launches.size() == 1) {
        HIPCHK(launch(launches[0], st));
        return STH_OK;
    }
    std::stable_sort(launches.begin(), launches.end(),
                     [](const GroupLaunch &a, const GroupLaunch &b) { return a.cost > b.cost; });
    SidePool *P = nullptr;
    int rc = side_pool(&P);
    if (rc) return rc;
    // the fork/join events are shared: issue one batch at a time
    std::lock_guard<std::mutex> lk(g_side_issue_mu);
    const int nl = std::min<int>(kLanes, (int)launches.size());
    double load[kLanes] = {};
    HIPCHK(hipEventRecord(P->fork, st));
    for (int i = 0; i < nl; ++i) HIPCHK(hipStreamWaitEvent(P->s[i], P->fork, 0));
    for (const GroupLaunch &L : launches) {
        int lane = 0;
        for (int i = 1; i < nl; ++i)
            if (load[i] < load[lane]) lane = i;
        load[lane] += L.cost;
        HIPCHK(launch(L, P->s[lane]));
    }
    for (int i = 0; i < nl; ++i) {
        HIPCHK(hipEventRecord(P->join[i], P->s[i]));
        HIPCHK(hipStreamWaitEvent(st, P->join[i], 0));
    }
    return STH_OK;
}

bool several_classes(const std::vector<SweepItem> &items)
{
    for (size_t t = 1; t < items.size(); ++t)
        if (!same_class(items[t].shape, items[0].shape)) return true;
    return false;
}

int issue_units(std::vector<SweepItem> &items, hipStream_t st)
{
    if (items.empty()) return STH_OK;
    sort_items(items);
    std::vector<FineUnit> table;
    std::vector<GroupLaunch> launches;
    if (several_classes(items) && plan_grouped(items, table, launches)) {
        int slot = 0;
        void *tab = nullptr;
        int rc = put_table(table.data(), sizeof(FineUnit) * table.size(), st, &slot, &tab);
        if (rc) return rc;
        const int rc2 = issue_grouped(launches, (const FineUnit *)tab, st);
        rc = release_table(slot, st);
        return rc2 ? rc2 : rc;
    }
    std::vector<FineUnit> host(items.size());
    for (size_t t = 0; t < items.size(); ++t) host[t] = items[t].unit;
    int slot = 0;
    void *tab = nullptr;
    int rc = put_table(host.data(), sizeof(FineUnit) * host.size(), st, &slot, &tab);
    if (rc) return rc;
    const int rc2 = issue_classes(items, (FineUnit *)tab, st);
    rc = release_table(slot, st);
    return rc2 ? rc2 : rc;
}

CoarseJob coarse_job_of(sth_problem *p, int mode, int k)
{
    CoarseJob j{};
    j.pc = p->at<FineConst>(p->L.cst);
    j.U = p->at<double>(p->L.U);
    j.Gc = p->at<double>(p->L.Gc);
    j.Fv = p->at<double>(p->L.Fv);
    j.err = p->at<double>(p->L.err);
    j.work = p->at<double>(p->L.work);
    j.dtG = p->dtG;
    j.N = p->N;
    j.mode = mode;
    j.k = k;
    j.errh = p->at<double>(p->L.errh);
    return j;
}

}  // namespace

extern "C" {

const char *sth_last_error(void) { return g_err.c_str(); }

int sth_footprint_bytes(const sth_problem_desc *d, size_t *out)
{
    int rc = validate(d);
    if (rc) return rc;
    if (!out) return fail(STH_EINVAL, "null output");
    *out = layout(d->nx, d->nv, d->n_slices, d->precision == STH_FP64 ? 8 : 4).total;
    return STH_OK;
}

int sth_create(const sth_problem_desc *d, void *arena, size_t arena_bytes, sth_problem **out)
{
    int rc = validate(d);
    if (rc) return rc;
    if (!out) return fail(STH_EINVAL, "null output");
    if (!d->eps_iface || !d->eps_cell || !d->rho0) return fail(STH_EINVAL, "eps and rho0 are required");
    const int nx = d->nx, nv = d->nv, N = d->n_slices;
    std::vector<double> eps_p(d->eps_iface, d->eps_iface + nx), eps_c(d->eps_cell, d->eps_cell + nx);
    std::vector<double> rho0(d->rho0, d->rho0 + nx);
    for (int i = 0; i < nx; ++i) {
        if (!(eps_p[i] > 0) || !(eps_c[i] > 0) || !std::isfinite(eps_p[i]) || !std::isfinite(eps_c[i]))
            return fail(STH_EINVAL, "eps must be finite and > 0");
        if (!std::isfinite(rho0[i])) return fail(STH_ENONFINITE, "rho0 is not finite");
    }

    sth_problem *p = new sth_problem();
    p->nx = nx; p->nv = nv; p->N = N; p->K = d->k_max;
    p->prec = d->precision; p->realsz = d->precision == STH_FP64 ? 8 : 4;
    p->flags = d->flags; p->start_mode = d->start_mode; p->lift_order = d->lift_order;
    p->Lx = d->Lx; p->vstar = d->vstar; p->T = d->T; p->tol = d->tol;
    p->eta0 = d->eta0; p->delta0 = d->delta0;
    p->dx = d->Lx / nx;
    p->dv = 2.0 * d->vstar / nv;
    p->nscale = d->nv_y ? std::sqrt(axis_m2sum(d->nv_y, d->vstar) * axis_m2sum(d->nv_z, d->vstar)) : 1.0;
    std::vector<double> vtab;
    velocity_table(nv, d->vstar, p->dx, vtab, p->m2);
    double s = 0.0;
    for (int i = 0; i < nx; ++i) s += rho0[i];
    p->rhobar = s / nx;
    const double Emax = (d->flags & STH_FIELD) ? field_max(rho0, p->rhobar, p->dx) : 0.0;
    const double dtmax = stable_dt(eps_p, p->dx, p->dv, d->vstar, p->m2, Emax, d->cfl_theta);
    p->dtG = d->T / N;
    if (!std::isfinite(p->rhobar) || !std::isfinite(Emax)) {
        delete p;
        return fail(STH_ENONFINITE, "the mean density or its field overflows");
    }
    if (d->steps_override <= 0 && !(dtmax > 0.0 && std::isfinite(dtmax))) {
        delete p;
        return fail(STH_EINVAL, "no positive stable fine step for this data");
    }
    const double nsd = d->steps_override > 0 ? (double)d->steps_override : std::ceil(p->dtG / dtmax);
    if (!(nsd <= 1e15)) {
        delete p;
        return fail(STH_EINVAL, "more than 1e15 fine steps per slice");
    }
    long long ns = (long long)nsd;
    if (ns < 1) ns = 1;
    p->ns = ns;
    p->dt = p->dtG / (double)ns;
    std::vector<double> e_p(nx), a_p(nx);
    for (int i = 0; i < nx; ++i) {
        const double r = p->dt / (eps_p[i] * eps_p[i]);
        e_p[i] = std::exp(-r);
        a_p[i] = -std::expm1(-r);
    }

    p->L = layout(nx, nv, N, p->realsz);
    if (arena) {
        if (arena_bytes < p->L.total) {
            delete p;
            return fail(STH_ENOMEM, "arena smaller than sth_footprint_bytes");
        }
        if (((uintptr_t)arena & 255) != 0) {
            delete p;
            return fail(STH_EINVAL, "arena must be 256-byte aligned");
        }
        if (!is_device_ptr(arena)) {
            delete p;
            return fail(STH_EINVAL, "arena must be device memory");
        }
        p->base = (char *)arena;
        p->owned = false;
    } else {
        hipError_t e = hipMalloc((void **)&p->base, p->L.total);
        if (e != hipSuccess) {
            delete p;
            return fail(STH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        p->owned = true;
    }
    p->bytes = p->L.total;
    p->have_end.assign(N + 1, 0);

    FineConst c{};
    c.nx = nx; c.nv = nv; c.flags = d->flags;
    c.dx = p->dx; c.dv = p->dv; c.dt = p->dt; c.rhobar = p->rhobar; c.m2 = p->m2;
    c.eta0 = d->eta0; c.delta0 = d->delta0; c.nsteps = ns;
    // explicit coarse scheme: its diffusive stable step with the fine step's margin
    c.coarse_steps = (long long)std::ceil(p->dtG / (d->cfl_theta * 0.75 * p->dx * p->dx / (2.0 * p->m2)));
    if (c.coarse_steps < 1) c.coarse_steps = 1;
    p->coarse_steps = c.coarse_steps;
    c.eps_p = p->at<double>(p->L.eps_p);
    c.eps_c = p->at<double>(p->L.eps_c);
    c.eps_n = p->at<double>(p->L.eps_n);
    c.e_p = p->at<double>(p->L.e_p);
    c.a_p = p->at<double>(p->L.a_p);
    c.vtab = p->at<double>(p->L.vtab);
    c.vrow64 = p->at<double>(p->L.vrow64);
    c.vrow32 = p->at<float>(p->L.vrow32);
    std::vector<double> vrow64(4 * (size_t)nv);
    std::vector<float> vrow32(4 * (size_t)nv);
    // row table of the fine sweep: |v_j|/dx, M_j, v_j M_j, M_{j+1} (M_nv = 0)
    for (int j = 0; j < nv; ++j)
        for (int q = 0; q < 4; ++q) {
            const double x = q < 3 ? vtab[(size_t)q * nv + j] : (j + 1 < nv ? vtab[(size_t)nv + j + 1] : 0.0);
            vrow64[4 * j + q] = x;
            vrow32[4 * j + q] = (float)x;
        }

    p->fc = c;
    auto up = [&](size_t off, const void *src, size_t n) { return hipMemcpy(p->base + off, src, n, hipMemcpyHostToDevice); };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(p->L.cst, &c, sizeof(c));
    if (e == hipSuccess) e = up(p->L.eps_p, eps_p.data(), sizeof(double) * nx);
    if (e == hipSuccess) e = up(p->L.eps_c, eps_c.data(), sizeof(double) * nx);
    {
        std::vector<double> eps_n(nx);
        for (int i = 0; i < nx; ++i) eps_n[i] = eps_p[i] * p->nscale;
        if (e == hipSuccess) e = up(p->L.eps_n, eps_n.data(), sizeof(double) * nx);
    }
    if (e == hipSuccess) e = up(p->L.e_p, e_p.data(), sizeof(double) * nx);
    if (e == hipSuccess) e = up(p->L.a_p, a_p.data(), sizeof(double) * nx);
    if (e == hipSuccess) e = up(p->L.vtab, vtab.data(), sizeof(double) * 4 * nv);
    if (e == hipSuccess) e = up(p->L.vrow64, vrow64.data(), sizeof(double) * 4 * nv);
    if (e == hipSuccess) e = up(p->L.vrow32, vrow32.data(), sizeof(float) * 4 * nv);
    if (e == hipSuccess) e = hipMemset(p->base + p->L.U, 0, p->L.err - p->L.U);
    if (e == hipSuccess) e = up(p->L.U, rho0.data(), sizeof(double) * nx);
    if (e == hipSuccess) e = hipMemset(p->base + p->L.kin, 0, sizeof(unsigned long long) * (N + 1));
    if (e == hipSuccess) e = hipMemset(p->base + p->L.gend, 0, p->gslab() * (size_t)(N + 1));
    if (e == hipSuccess && d->g0) {
        std::vector<char> gv = to_vmajor(d->g0, nx, nv, p->prec);
        e = up(p->L.g0, gv.data(), gv.size());
        p->has_g0 = true;
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (p->owned) (void)hipFree(p->base);
        delete p;
        return hip_fail(e, "sth_create upload");
    }
    *out = p;
    return STH_OK;
}

void sth_destroy(sth_problem *p)
{
    if (!p) return;
    if (p->owned && p->base) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->base);
    }
    delete p;
}

int sth_coarse_sweep(sth_problem *p, void *stream)
{
    if (!p) return fail(STH_EINVAL, "null problem");
    const CoarseJob j = coarse_job_of(p, 0, 0);
    HIPCHK(launch_coarse(j, p->nx, (p->flags & STH_COARSE_EXPLICIT) != 0, (hipStream_t)stream));
    p->coarse_done = true;
    p->k = 0;
    p->swept = false;
    p->chunk_pos = -1;
    std::fill(p->have_end.begin(), p->have_end.end(), 0);
    return STH_OK;
}

int sth_coarse_sweep_batched(sth_problem *const *probs, int count, void *stream)
{
    if (count < 0 || (count > 0 && !probs)) return fail(STH_EINVAL, "bad batch");
    for (int b = 0; b < count; ++b) {
        if (!probs[b]) return fail(STH_EINVAL, "null problem in batch");
        for (int c = 0; c < b; ++c)
            if (probs[c] == probs[b]) return fail(STH_EINVAL, "a problem appears twice in the batch");
    }
    if (count == 0) return STH_OK;
    hipStream_t st = (hipStream_t)stream;
    std::vector<CoarseJob> jobs(count);
    int block = kWave;
    size_t lds = 0;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        jobs[b] = coarse_job_of(p, 0, 0);
        int bb = 0;
        size_t ll = 0;
        coarse_launch_dims(p->nx, (p->flags & STH_COARSE_EXPLICIT) != 0, &bb, &ll);
        block = std::max(block, bb);
        lds = std::max(lds, ll);
    }
    int slot = 0;
    void *tab = nullptr;
    int rc = put_table(jobs.data(), sizeof(CoarseJob) * jobs.size(), st, &slot, &tab);
    if (rc) return rc;
    const hipError_t le = launch_coarse_many((const CoarseJob *)tab, count, block, lds, st);
    rc = release_table(slot, st);
    if (le != hipSuccess) return hip_fail(le, "launch_coarse_many");
    if (rc) return rc;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        p->coarse_done = true;
        p->k = 0;
        p->swept = false;
        p->chunk_pos = -1;
        std::fill(p->have_end.begin(), p->have_end.end(), 0);
    }
    return STH_OK;
}

int sth_fine_sweep_batched(sth_problem *const *probs, int count, void *stream)
{
    if (count < 0 || (count > 0 && !probs)) return fail(STH_EINVAL, "bad batch");
    hipStream_t st = (hipStream_t)stream;
    for (int b = 0; b < count; ++b) {
        if (!probs[b]) return fail(STH_EINVAL, "null problem in batch");
        if (!probs[b]->coarse_done) return fail(STH_ESTATE, "sth_coarse_sweep must precede the fine sweep");
        if (probs[b]->chunk_pos >= 0) return fail(STH_ESTATE, "a chunked fine sweep is in progress");
        for (int c = 0; c < b; ++c)
            if (probs[c] == probs[b]) return fail(STH_EINVAL, "a problem appears twice in the batch");
    }
    std::vector<SweepItem> items;
    LiftBatch lb;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        if (p->k >= p->N) continue;
        std::vector<LiftJob> lifts;
        std::vector<CopyJob> copies;
        plan_problem_sweep(p, p->k, p->have_end, nullptr, items, lifts, copies);
        for (const CopyJob &c : copies)
            HIPCHK(hipMemcpyAsync(c.dst, c.src, c.n * sizeof(uint4), hipMemcpyDeviceToDevice, st));
        lb.add(p, lifts);
    }
    int rc = lb.issue(st);
    if (rc) return rc;
    rc = issue_units(items, st);
    if (rc) return rc;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        for (int n = p->k + 1; n <= p->N; ++n) p->have_end[n] = 1;
        p->swept = true;
    }
    return STH_OK;
}

int sth_fine_sweep_chunk(sth_problem *const *probs, int count, long long max_steps, int *done_out, void *stream)
{
    if (count < 0 || (count > 0 && !probs)) return fail(STH_EINVAL, "bad batch");
    if (max_steps < 1) return fail(STH_EINVAL, "max_steps must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    for (int b = 0; b < count; ++b) {
        if (!probs[b]) return fail(STH_EINVAL, "null problem in batch");
        if (!probs[b]->coarse_done) return fail(STH_ESTATE, "sth_coarse_sweep must precede the fine sweep");
        for (int c = 0; c < b; ++c)
            if (probs[c] == probs[b]) return fail(STH_EINVAL, "a problem appears twice in the batch");
    }
    std::vector<SweepItem> items;
    LiftBatch lb;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        if (done_out) done_out[b] = p->swept ? 1 : 0;
        if (p->k >= p->N || p->swept) continue;
        if (p->chunk_pos < 0) {
            // a new sweep: slice starts prepared now, units kept for the chunks
            std::vector<SweepItem> mine;
            std::vector<LiftJob> lifts;
            std::vector<CopyJob> copies;
            plan_problem_sweep(p, p->k, p->have_end, nullptr, mine, lifts, copies);
            for (const CopyJob &c : copies)
                HIPCHK(hipMemcpyAsync(c.dst, c.src, c.n * sizeof(uint4), hipMemcpyDeviceToDevice, st));
            lb.add(p, lifts);
            p->chunk_units.clear();
            for (const SweepItem &it : mine) p->chunk_units.push_back(it.unit);
            p->chunk_pos = 0;
        }
        const long long s0 = p->chunk_pos, s1 = std::min(p->ns, s0 + max_steps);
        const FineShape sh = class_shape(p->prec, p->nx, p->nv);
        for (FineUnit u : p->chunk_units) {
            u.step0 = s0;
            u.step1 = s1;
            items.push_back({sh, u, (double)(s1 - s0) * p->nx * p->nv});
        }
    }
    int rc = lb.issue(st);
    if (rc) return rc;
    rc = issue_units(items, st);
    if (rc) return rc;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        if (p->k >= p->N || p->swept || p->chunk_pos < 0) continue;
        p->chunk_pos = std::min(p->ns, p->chunk_pos + max_steps);
        if (p->chunk_pos >= p->ns) {
            for (int n = p->k + 1; n <= p->N; ++n) p->have_end[n] = 1;
            p->swept = true;
            p->chunk_pos = -1;
            p->chunk_units.clear();
            if (done_out) done_out[b] = 1;
        }
    }
    return STH_OK;
}

int sth_parareal_correct(sth_problem *p, double *err_out, int *k_out, void *stream)
{
    if (!p) return fail(STH_EINVAL, "null problem");
    if (!p->swept) return fail(STH_ESTATE, "sth_fine_sweep_batched must precede the correction");
    if (p->k >= p->N) return fail(STH_ESTATE, "all slices converged");
    hipStream_t st = (hipStream_t)stream;
    const CoarseJob j = coarse_job_of(p, 1, p->k);
    HIPCHK(launch_coarse(j, p->nx, (p->flags & STH_COARSE_EXPLICIT) != 0, st));
    p->k += 1;
    p->swept = false;
    if (err_out) {
        double e = 0.0;
        HIPCHK(hipMemcpyAsync(&e, j.err, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *err_out = e;
        p->last_err = e;
    }
    if (k_out) *k_out = p->k;
    if (err_out && !std::isfinite(*err_out)) return fail(STH_ENONFINITE, "non-finite density after the correction");
    return STH_OK;
}

int sth_parareal_correct_batched(sth_problem *const *probs, int count, double *errs_out, void *stream)
{
    if (count < 0 || (count > 0 && !probs)) return fail(STH_EINVAL, "bad batch");
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        if (!p) return fail(STH_EINVAL, "null problem in batch");
        if (!p->swept) return fail(STH_ESTATE, "sth_fine_sweep_batched must precede the correction");
        if (p->k >= p->N) return fail(STH_ESTATE, "all slices converged");
        for (int c = 0; c < b; ++c)
            if (probs[c] == p) return fail(STH_EINVAL, "a problem appears twice in the batch");
    }
    if (count == 0) return STH_OK;
    hipStream_t st = (hipStream_t)stream;
    // table: the jobs, then one error slot per job (one read-back for all)
    const size_t jbytes = al256(sizeof(CoarseJob) * (size_t)count);
    int slot = 0;
    int rc = acquire_table(jbytes + sizeof(double) * (size_t)count, &slot);
    if (rc) return rc;
    char *tab = nullptr, *htab = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        tab = (char *)g_pool[slot].ptr;
        htab = (char *)g_pool[slot].host;
    }
    double *derr = (double *)(tab + jbytes);
    std::vector<CoarseJob> jobs(count);
    int block = kWave;
    size_t lds = 0;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        jobs[b] = coarse_job_of(p, 1, p->k);
        jobs[b].err = derr + b;
        int bb = 0;
        size_t ll = 0;
        coarse_launch_dims(p->nx, (p->flags & STH_COARSE_EXPLICIT) != 0, &bb, &ll);
        block = std::max(block, bb);
        lds = std::max(lds, ll);
    }
    std::memcpy(htab, jobs.data(), sizeof(CoarseJob) * jobs.size());
    hipError_t e = hipMemcpyAsync(tab, htab, sizeof(CoarseJob) * jobs.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_coarse_many((const CoarseJob *)tab, count, block, lds, st);
    // errors back through the pinned mirror, past the jobs
    double *herr = (double *)(htab + jbytes);
    if (e == hipSuccess && errs_out)
        e = hipMemcpyAsync(herr, derr, sizeof(double) * count, hipMemcpyDeviceToHost, st);
    std::vector<double> errs(count, 0.0);
    if (e == hipSuccess && errs_out) {
        // the errors are read from the mirror before the table is released,
        // so that no other caller can reuse the slot and overwrite them
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) std::memcpy(errs.data(), herr, sizeof(double) * count);
    }
    rc = release_table(slot, st);
    if (e != hipSuccess) return hip_fail(e, "sth_parareal_correct_batched");
    if (rc) return rc;
    bool finite = true;
    for (int b = 0; b < count; ++b) {
        sth_problem *p = probs[b];
        p->k += 1;
        p->swept = false;
        if (errs_out) {
            errs_out[b] = errs[b];
            p->last_err = errs[b];
            finite = finite && std::isfinite(errs[b]);
        }
    }
    if (!finite) return fail(STH_ENONFINITE, "non-finite density after the correction (see errs_out)");
    return STH_OK;
}

namespace {

// Operations of a recorded solve, in issue order; offsets into the graph's
// device table buffer.
struct GraphOp {
    enum Kind { COARSE, LIFT, COPY, FINE } kind;
    size_t off;
    int n;              // jobs or units
    int a;              // COARSE: block; LIFT: precision
    size_t b;           // COARSE: LDS bytes; LIFT: nx; COPY: largest job (16-byte words)
    size_t items_begin; // FINE: range in the graph's item list
    size_t items_end;
    int group = -1;     // FINE: index of its grouped plan, or -1 (one launch per class)
};

struct TableBuilder {
    std::vector<char> host;
    size_t put(const void *src, size_t bytes)
    {
        const size_t off = al256(host.size());
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        return off;
    }
};

void destroy_graph(sth_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    if (g->dbuf) (void)hipFree(g->dbuf);
    delete g;
}

}  // namespace

int sth_graph_create(sth_problem *const *probs, int count, sth_graph **out)
{
    if (!out) return fail(STH_EINVAL, "null output");
    *out = nullptr;
    if (count <= 0 || !probs) return fail(STH_EINVAL, "bad batch");
    for (int b = 0; b < count; ++b) {
        if (!probs[b]) return fail(STH_EINVAL, "null problem in batch");
        for (int c = 0; c < b; ++c)
            if (probs[c] == probs[b]) return fail(STH_EINVAL, "a problem appears twice in the batch");
    }
    sth_graph *g = new sth_graph();
    g->probs.assign(probs, probs + count);
    for (sth_problem *p : g->probs) {
        const int km = std::max(0, std::min(p->K, p->N));
        g->kmax.push_back(km);
        g->iters = std::max(g->iters, km);
    }
    // plan every launch of the solve on the host
    TableBuilder tb;
    std::vector<GraphOp> ops;
    std::vector<SweepItem> all_items;
    std::vector<std::vector<GroupLaunch>> group_plans;
    auto coarse_op = [&](int mode, int k) {
        std::vector<CoarseJob> jobs;
        int block = kWave;
        size_t lds = 0;
        for (size_t b = 0; b < g->probs.size(); ++b) {
            sth_problem *p = g->probs[b];
            if (mode == 1 && k >= g->kmax[b]) continue;
            CoarseJob j = coarse_job_of(p, mode, k);
            j.ctl = p->at<int>(p->L.ctl);
            j.kin = p->at<unsigned long long>(p->L.kin);
            j.tol = p->tol;
            j.kmax = g->kmax[b];
            jobs.push_back(j);
            int bb = 0;
            size_t ll = 0;
            coarse_launch_dims(p->nx, (p->flags & STH_COARSE_EXPLICIT) != 0, &bb, &ll);
            block = std::max(block, bb);
            lds = std::max(lds, ll);
        }
        if (jobs.empty()) return;
        GraphOp op{GraphOp::COARSE, tb.put(jobs.data(), sizeof(CoarseJob) * jobs.size()), (int)jobs.size(), block,
                   lds, 0, 0};
        ops.push_back(op);
    };
    coarse_op(0, 0);
    std::vector<std::vector<char>> have(g->probs.size());
    for (size_t b = 0; b < g->probs.size(); ++b) have[b].assign(g->probs[b]->N + 1, 0);
    for (int k = 0; k < g->iters; ++k) {
        std::vector<SweepItem> items;
        std::vector<CopyJob> copies;
        size_t max_copy = 0;
        for (size_t b = 0; b < g->probs.size(); ++b) {
            sth_problem *p = g->probs[b];
            if (k >= g->kmax[b]) continue;
            const int *stop = p->at<int>(p->L.ctl) + 1;
            std::vector<LiftJob> lifts;
            plan_problem_sweep(p, k, have[b], stop, items, lifts, copies);
            if (!lifts.empty()) {
                GraphOp op{GraphOp::LIFT, tb.put(lifts.data(), sizeof(LiftJob) * lifts.size()), (int)lifts.size(),
                           p->prec, (size_t)p->nx, 0, 0};
                ops.push_back(op);
            }
            for (int n = k + 1; n <= p->N; ++n) have[b][n] = 1;
        }
        for (const CopyJob &c : copies) max_copy = std::max(max_copy, c.n);
        for (size_t c0 = 0; c0 < copies.size(); c0 += 65535) {
            const size_t nc = std::min<size_t>(65535, copies.size() - c0);
            GraphOp op{GraphOp::COPY, tb.put(copies.data() + c0, sizeof(CopyJob) * nc), (int)nc, 0, max_copy, 0, 0};
            ops.push_back(op);
        }
        sort_items(items);
        std::vector<FineUnit> units;
        std::vector<GroupLaunch> gl;
        const bool grouped = several_classes(items) && plan_grouped(items, units, gl);
        if (!grouped) {
            units.resize(items.size());
            for (size_t t = 0; t < items.size(); ++t) units[t] = items[t].unit;
        }
        GraphOp op{GraphOp::FINE, tb.put(units.data(), sizeof(FineUnit) * units.size()), (int)units.size(), 0, 0,
                   all_items.size(), all_items.size() + items.size()};
        op.group = grouped ? (int)group_plans.size() : -1;
        if (grouped) group_plans.push_back(gl);
        ops.push_back(op);
        all_items.insert(all_items.end(), items.begin(), items.end());
        coarse_op(1, k);
    }
    // upload the tables, then record the launches
    hipError_t e = hipMalloc(&g->dbuf, std::max<size_t>(tb.host.size(), 256));
    if (e == hipSuccess) e = hipMemcpy(g->dbuf, tb.host.data(), tb.host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_graph(g);
        return hip_fail(e, "sth_graph_create: set-up");
    }
    e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        destroy_graph(g);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    int rc = STH_OK;
    for (const GraphOp &op : ops) {
        void *tab = g->dbuf + op.off;
        hipError_t le = hipSuccess;
        switch (op.kind) {
            case GraphOp::COARSE: le = launch_coarse_many((const CoarseJob *)tab, op.n, op.a, op.b, g->cap); break;
            case GraphOp::LIFT: le = launch_lift(op.a, (const LiftJob *)tab, op.n, (int)op.b, g->cap); break;
            case GraphOp::COPY: le = launch_copy((const CopyJob *)tab, op.n, op.b, g->cap); break;
            case GraphOp::FINE: {
                if (op.group >= 0) {
                    rc = issue_grouped(group_plans[op.group], (const FineUnit *)tab, g->cap);
                } else {
                    std::vector<SweepItem> items(all_items.begin() + op.items_begin, all_items.begin() + op.items_end);
                    rc = issue_classes(items, (FineUnit *)tab, g->cap);
                }
                break;
            }
        }
        if (le != hipSuccess) rc = hip_fail(le, "sth_graph_create: recording a launch");
        if (rc) break;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g->cap, &graph);
    g->graph = graph;
    if (rc) {
        destroy_graph(g);
        return rc;
    }
    if (e != hipSuccess) {
        destroy_graph(g);
        return hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_graph(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = g;
    return STH_OK;
}

int sth_graph_launch(sth_graph *g, void *stream)
{
    if (!g || !g->exec) return fail(STH_EINVAL, "null graph");
    HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
    g->launched = true;
    for (sth_problem *p : g->probs) {
        // host bookkeeping is settled by sth_graph_wait
        p->coarse_done = false;
        p->swept = false;
    }
    return STH_OK;
}

int sth_graph_wait(sth_graph *g, void *stream, int *iters_out, double *last_err_out)
{
    if (!g) return fail(STH_EINVAL, "null graph");
    if (!g->launched) return fail(STH_ESTATE, "the graph has not been launched");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    bool nonfinite = false;
    for (size_t b = 0; b < g->probs.size(); ++b) {
        sth_problem *p = g->probs[b];
        int ctl[2] = {0, 0};
        HIPCHK(hipMemcpy(ctl, p->at<int>(p->L.ctl), sizeof(ctl), hipMemcpyDeviceToHost));
        const int k = std::max(0, std::min(ctl[0], p->N));
        double e = -1.0;
        if (k > 0) HIPCHK(hipMemcpy(&e, p->at<double>(p->L.errh) + (k - 1), sizeof(double), hipMemcpyDeviceToHost));
        p->k = k;
        p->last_err = e;
        p->coarse_done = true;
        p->swept = false;
        p->chunk_pos = -1;
        std::fill(p->have_end.begin(), p->have_end.end(), 0);
        if (k > 0)
            for (int n = 1; n <= p->N; ++n) p->have_end[n] = 1;
        if (iters_out) iters_out[b] = k;
        if (last_err_out) last_err_out[b] = e;
        if (k > 0 && !std::isfinite(e)) nonfinite = true;
    }
    if (nonfinite) return fail(STH_ENONFINITE, "non-finite density in a recorded solve (see last_err_out)");
    return STH_OK;
}

int sth_get_errors(const sth_problem *p, double *host_out)
{
    if (!p || !host_out) return fail(STH_EINVAL, "null argument");
    HIPCHK(hipDeviceSynchronize());
    if (p->k > 0) HIPCHK(hipMemcpy(host_out, p->at<double>(p->L.errh), sizeof(double) * p->k, hipMemcpyDeviceToHost));
    return STH_OK;
}

void sth_graph_destroy(sth_graph *g) { destroy_graph(g); }

int sth_fine_config_candidates(int precision, int nx, int nv, sth_fine_config *out, int cap, int *count)
{
    if (!count || cap < 0 || (cap > 0 && !out)) return fail(STH_EINVAL, "null argument");
    if (precision != STH_FP64 && precision != STH_FP32_BULK) return fail(STH_EINVAL, "unknown precision");
    if (nx < 8 || nx > kMaxNx) return fail(STH_EINVAL, "nx must be in [8, 2048]");
    if (!(nv == 16 || nv == 32 || nv == 64 || nv == 128)) return fail(STH_EINVAL, "nv must be 16, 32, 64 or 128");
    const std::vector<sth_fine_config> c = class_candidates(precision == STH_FP64 ? 0 : 1, nx, nv);
    *count = (int)c.size();
    for (int i = 0; i < cap && i < (int)c.size(); ++i) out[i] = c[i];
    return STH_OK;
}

int sth_set_fine_config(int precision, int nx, int nv, const sth_fine_config *cfg)
{
    if (precision != STH_FP64 && precision != STH_FP32_BULK) return fail(STH_EINVAL, "unknown precision");
    if (nx < 8 || nx > kMaxNx) return fail(STH_EINVAL, "nx must be in [8, 2048]");
    if (!(nv == 16 || nv == 32 || nv == 64 || nv == 128)) return fail(STH_EINVAL, "nv must be 16, 32, 64 or 128");
    const int prec = precision == STH_FP64 ? 0 : 1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!cfg) {
        g_tune.erase(class_key(prec, nx, nv));
        return STH_OK;
    }
    // a configuration must be valid for every nx of the class
    const ClassKey key = class_key(prec, nx, nv);
    const sth_fine_config c{cfg->block, cfg->resident ? 1 : 0};
    for (int x = key.nxr - kWave + 1; x <= key.nxr; ++x) {
        if (x < 8 || x > kMaxNx) continue;
        if (!config_ok(prec, x, nv, c)) return fail(STH_EINVAL, "launch configuration not supported for this class");
    }
    g_tune[key] = c;
    return STH_OK;
}

int sth_get_fine_config(int precision, int nx, int nv, sth_fine_config *out)
{
    if (!out) return fail(STH_EINVAL, "null argument");
    if (precision != STH_FP64 && precision != STH_FP32_BULK) return fail(STH_EINVAL, "unknown precision");
    if (nx < 8 || nx > kMaxNx) return fail(STH_EINVAL, "nx must be in [8, 2048]");
    if (!(nv == 16 || nv == 32 || nv == 64 || nv == 128)) return fail(STH_EINVAL, "nv must be 16, 32, 64 or 128");
    const FineShape sh = class_shape(precision == STH_FP64 ? 0 : 1, nx, nv);
    out->block = sh.block;
    out->resident = sh.stream ? 0 : 1;
    return STH_OK;
}

int sth_moments_criteria(const sth_problem *p, int slice, double *E, double *J, double *Phi, double *N,
                         double *R, int *cell_mask, void *stream)
{
    if (!p) return fail(STH_EINVAL, "null problem");
    if (slice < 0 || slice > p->N) return fail(STH_EINVAL, "slice out of range");
    hipStream_t st = (hipStream_t)stream;
    const int nx = p->nx;
    DiagJob j{};
    j.pc = p->at<FineConst>(p->L.cst);
    j.rho = p->at<double>(p->L.U) + (size_t)slice * nx;
    j.g = (slice >= 1 && p->have_end[slice]) ? (const void *)(p->base + p->L.gend + (size_t)slice * p->gslab())
                                             : nullptr;
    // outputs in the coarse workspace (5*nx doubles) and the mask buffer
    j.out = p->at<double>(p->L.work);
    j.mask = p->at<int>(p->L.mask);
    HIPCHK(launch_diag(p->prec, j, nx, st));
    std::vector<double> h(5 * (size_t)nx);
    std::vector<int> m(nx);
    HIPCHK(hipMemcpyAsync(h.data(), j.out, sizeof(double) * 5 * nx, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(m.data(), j.mask, sizeof(int) * nx, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double *outs[5] = {E, J, Phi, N, R};
    for (int q = 0; q < 5; ++q)
        if (outs[q]) std::memcpy(outs[q], h.data() + (size_t)q * nx, sizeof(double) * nx);
    if (cell_mask) std::memcpy(cell_mask, m.data(), sizeof(int) * nx);
    return STH_OK;
}

int sth_get_rho(const sth_problem *p, double *host_out)
{
    if (!p || !host_out) return fail(STH_EINVAL, "null argument");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host_out, p->base + p->L.U, sizeof(double) * (size_t)(p->N + 1) * p->nx,
                     hipMemcpyDeviceToHost));
    return STH_OK;
}

int sth_get_g(const sth_problem *p, int slice, double *host_out)
{
    if (!p || !host_out) return fail(STH_EINVAL, "null argument");
    if (slice < 1 || slice > p->N) return fail(STH_EINVAL, "slice must be in 1..N");
    HIPCHK(hipDeviceSynchronize());
    std::vector<char> buf(vmajor_bytes(p->nx, p->nv, p->realsz));
    HIPCHK(hipMemcpy(buf.data(), p->base + p->L.gend + (size_t)slice * p->gslab(), buf.size(),
                     hipMemcpyDeviceToHost));
    from_vmajor(buf, p->nx, p->nv, p->prec, host_out);
    return STH_OK;
}

int sth_get_info(const sth_problem *p, sth_info *out)
{
    if (!p || !out) return fail(STH_EINVAL, "null argument");
    HIPCHK(hipDeviceSynchronize());
    std::vector<unsigned long long> kin(p->N + 1);
    HIPCHK(hipMemcpy(kin.data(), p->base + p->L.kin, sizeof(unsigned long long) * (p->N + 1),
                     hipMemcpyDeviceToHost));
    double tot = 0.0;
    for (int n = 1; n <= p->N; ++n) tot += (double)kin[n];
    out->dx = p->dx; out->dv = p->dv; out->dt = p->dt; out->dtG = p->dtG;
    out->m2 = p->m2; out->rhobar = p->rhobar; out->steps_per_slice = p->ns;
    out->k_done = p->k; out->n_slices = p->N;
    out->kinetic_iface_steps = tot;
    out->last_err = p->last_err;
    out->footprint_bytes = p->bytes;
    const FineShape sh = class_shape(p->prec, p->nx, p->nv);
    out->fine_resident = sh.stream ? 0 : 1;
    out->fine_block = sh.block;
    out->coarse_steps = (p->flags & STH_COARSE_EXPLICIT) ? p->coarse_steps : 1;
    out->norm_scale = p->nscale;
    return STH_OK;
}

int sth_fine_run(sth_problem *p, const double *rho_in, const double *g_in, long long nsteps,
                 double *rho_out, double *g_out, int *cell_mask_out, double *kin_out, void *stream)
{
    return sth_fine_run_masks(p, rho_in, g_in, nsteps, nullptr, nullptr, 0, rho_out, g_out, cell_mask_out,
                              kin_out, stream);
}

int sth_fine_run_masks(sth_problem *p, const double *rho_in, const double *g_in, long long nsteps,
                       const uint64_t *mask_replay, uint64_t *mask_hist, long long mask_words, double *rho_out,
                       double *g_out, int *cell_mask_out, double *kin_out, void *stream)
{
    if (!p || !rho_in) return fail(STH_EINVAL, "null argument");
    if (nsteps < 0) return fail(STH_EINVAL, "nsteps must be >= 0");
    if ((mask_replay || mask_hist) && !(p->flags & STH_HYBRID))
        return fail(STH_EINVAL, "a cell status history needs STH_HYBRID");
    if (mask_replay || mask_hist) {
        // (nsteps + 1) rows of ceil(nx/64) words, computed without overflow
        const long long mw = (p->nx + kWave - 1) / kWave;
        if (mask_words < 0 || nsteps + 1 > mask_words / mw)
            return fail(STH_EINVAL, "mask_words is smaller than (nsteps + 1) * ceil(nx / 64)");
    }
    if (mask_replay && !is_device_ptr(mask_replay)) return fail(STH_EINVAL, "mask_replay must be device memory");
    if (mask_hist && !is_device_ptr(mask_hist)) return fail(STH_EINVAL, "mask_hist must be device memory");
    hipStream_t st = (hipStream_t)stream;
    const int nx = p->nx;
    HIPCHK(hipDeviceSynchronize());
    double *d_rin = p->at<double>(p->L.work);
    double *d_rout = d_rin + nx;
    void *d_gin = p->base + p->L.gst;     // slot 0 of the start buffer
    void *d_gout = p->base + p->L.gend;   // slot 0 of the end buffer
    unsigned long long *d_kin = p->at<unsigned long long>(p->L.kin);
    HIPCHK(hipMemcpy(d_rin, rho_in, sizeof(double) * nx, hipMemcpyHostToDevice));
    if (g_in) {
        std::vector<char> gv = to_vmajor(g_in, nx, p->nv, p->prec);
        HIPCHK(hipMemcpy(d_gin, gv.data(), gv.size(), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemset(d_kin, 0, sizeof(unsigned long long)));
    FineUnit u{};
    u.c = p->fc;
    u.rho_in = d_rin;
    u.rho_out = d_rout;
    u.g_in = g_in ? d_gin : nullptr;
    u.g_out = d_gout;
    u.kin = d_kin;
    u.mask_out = p->at<int>(p->L.mask);
    u.nsteps = nsteps;  // 0: the start state after the status rule
    u.mask_replay = (const unsigned long long *)mask_replay;
    u.mask_hist = (unsigned long long *)mask_hist;
    FineUnit *dt = p->at<FineUnit>(p->L.units);
    HIPCHK(hipMemcpy(dt, &u, sizeof(u), hipMemcpyHostToDevice));
    const FineShape sh = class_shape(p->prec, nx, p->nv);
    HIPCHK(launch_fine(sh, dt, 1, st));
    HIPCHK(hipStreamSynchronize(st));
    if (rho_out) HIPCHK(hipMemcpy(rho_out, d_rout, sizeof(double) * nx, hipMemcpyDeviceToHost));
    if (g_out) {
        std::vector<char> buf(vmajor_bytes(nx, p->nv, p->realsz));
        HIPCHK(hipMemcpy(buf.data(), d_gout, buf.size(), hipMemcpyDeviceToHost));
        from_vmajor(buf, nx, p->nv, p->prec, g_out);
    }
    if (cell_mask_out) HIPCHK(hipMemcpy(cell_mask_out, u.mask_out, sizeof(int) * nx, hipMemcpyDeviceToHost));
    if (kin_out) {
        unsigned long long k = 0;
        HIPCHK(hipMemcpy(&k, d_kin, sizeof(k), hipMemcpyDeviceToHost));
        *kin_out = (double)k;
    }
    return STH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free single-slice run.  Its unit table, slice slot (rows,
// lazy projection, halos), densities, status, counter and the x-major
// staging of the perturbation live in one file-scope device array instead
// of the problem's arena: kNoAllocScratchBytes per device, held until the
// process ends.  Host code never uses the array's name as an address (it is
// a host-side stand-in there); the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(2) << 20;  // 2 MiB
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of the current device's copy of scratch.
int scratch_address(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(STH_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return STH_OK;
}

// Offsets of one run in scratch (256-byte aligned blocks).
struct NoAllocLayout {
    size_t unit, rin, rout, mask, kin, slot, gx, total;
};

NoAllocLayout noalloc_layout(int nx, int nv, int realsz, bool staging)
{
    NoAllocLayout L{};
    size_t o = 0;
    L.unit = o; o = al256(o + sizeof(FineUnit));
    L.rin = o;  o = al256(o + sizeof(double) * nx);
    L.rout = o; o = al256(o + sizeof(double) * nx);
    L.mask = o; o = al256(o + sizeof(int) * nx);
    L.kin = o;  o = al256(o + sizeof(unsigned long long));
    L.slot = o; o = al256(o + fine_slot_elems(nx, nv) * (size_t)realsz);
    L.gx = o;   if (staging) o = al256(o + sizeof(double) * (size_t)nx * nv);
    L.total = o;
    return L;
}

const unsigned long long kZeroCounter = 0;

}  // namespace

extern "C" {

int sth_fine_run_noalloc(const sth_problem *p, const double *rho_in, const double *g_in, long long nsteps,
                         double *rho_out, double *g_out, int *cell_mask_out, double *kin_out, void *stream)
{
    if (!p || !rho_in) return fail(STH_EINVAL, "null argument");
    if (nsteps < 0) return fail(STH_EINVAL, "nsteps must be >= 0");
    const int nx = p->nx, nv = p->nv;
    const NoAllocLayout L = noalloc_layout(nx, nv, p->realsz, g_in || g_out);
    if (L.total > kNoAllocScratchBytes)
        return fail(STH_EINVAL, "sth_fine_run_noalloc: the run needs more than the 2 MiB static workspace "
                                "(use sth_fine_run)");
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    char *b = (char *)base;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(b + L.rin, rho_in, sizeof(double) * nx, hipMemcpyHostToDevice));
    // the counter starts at zero (the workspace keeps the last run's contents)
    HIPCHK(hipMemcpy(b + L.kin, &kZeroCounter, sizeof(kZeroCounter), hipMemcpyHostToDevice));
    if (g_in) {
        HIPCHK(hipMemcpy(b + L.gx, g_in, sizeof(double) * (size_t)nx * nv, hipMemcpyHostToDevice));
        // the start rows go to the slot's own rows: the kernel reads each
        // start value before the same thread writes that element
        HIPCHK(launch_to_vmajor(p->prec, (const double *)(b + L.gx), b + L.slot, nx, nv, st));
    }
    FineUnit u{};
    u.c = p->fc;
    u.rho_in = (const double *)(b + L.rin);
    u.rho_out = (double *)(b + L.rout);
    u.g_in = g_in ? (const void *)(b + L.slot) : nullptr;
    u.g_out = b + L.slot;
    u.kin = (unsigned long long *)(b + L.kin);
    u.mask_out = (int *)(b + L.mask);
    u.nsteps = nsteps;  // 0: the start state after the status rule
    HIPCHK(hipMemcpy(b + L.unit, &u, sizeof(u), hipMemcpyHostToDevice));
    const FineShape sh = class_shape(p->prec, nx, nv);
    HIPCHK(launch_fine(sh, (const FineUnit *)(b + L.unit), 1, st));
    if (g_out) HIPCHK(launch_to_xmajor(p->prec, b + L.slot, (double *)(b + L.gx), nx, nv, st));
    HIPCHK(hipStreamSynchronize(st));
    if (rho_out) HIPCHK(hipMemcpy(rho_out, b + L.rout, sizeof(double) * nx, hipMemcpyDeviceToHost));
    if (g_out) HIPCHK(hipMemcpy(g_out, b + L.gx, sizeof(double) * (size_t)nx * nv, hipMemcpyDeviceToHost));
    if (cell_mask_out) HIPCHK(hipMemcpy(cell_mask_out, b + L.mask, sizeof(int) * nx, hipMemcpyDeviceToHost));
    if (kin_out) {
        unsigned long long k = 0;
        HIPCHK(hipMemcpy(&k, b + L.kin, sizeof(k), hipMemcpyDeviceToHost));
        *kin_out = (double)k;
    }
    return STH_OK;
}

}  // extern "C"
